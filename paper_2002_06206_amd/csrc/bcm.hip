// Building-cube grid (Sec. 2.2): two fixed levels of cubes of n^3 cells, a factor of two
// apart, each stored with two halo layers per face; the halo exchange between cubes
// (copy from a cube of the same or a coarser level, mean of the 8 fine cells from a
// finer one, mirror at the domain boundary; axis directions only) and the 7-point
// operator on the cubes.
//
// The host resolves, once, every face-halo cell to the interior cells it reads (one for
// a copy, eight for a mean, in z, y, x order), as compressed lists; the exchange is then
// one gather per halo cell.  It reads interior cells only and writes halo cells only, so
// all halo cells of all cubes are filled by one launch without ordering.  Compiled
// without FMA contraction: means and operator values are one fixed FP64 computation.
//
// The pressure solve on the cubes (Sec. 2.1's BiCGStab and red-black SOR on this grid)
// keeps its scalars on the device: each dot product is a launch of block partials and a
// one-block launch that sums them in block order and takes the iteration's decision
// (stop, breakdown, the next coefficient) into a small state; every later vector
// kernel reads that state and does nothing once the solve has stopped.  The host only
// reads the state every check_every iterations.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "common.h"

namespace ibm {
// device state of a solve on the cubes
struct BcmState {
    double bb, rr, rho, rho_old, alpha, omega, beta;
    int done;    // BCM_RUNNING or the reason the solve stopped
    int iters;   // iterations made when it stopped
};
}  // namespace ibm

struct ibm_bcm {
    int device;
    int K[3];
    int n;
    int side;                      // n + 2 * BCM_H
    double dx0;
    double origin[3];
    std::vector<uint8_t> refine;   // Kz * Ky * Kx
    std::vector<long long> first;  // first cube of each coarse cube
    std::vector<int> level;        // per cube
    std::vector<int> org;          // per cube, origin in fine-cell units (x, y, z)
    long long ncubes;
    long long size;                // values of the cube storage
    long long nhalo;
    int* d_dst = nullptr;          // storage index of each halo cell
    int* d_off = nullptr;          // nhalo + 1 offsets into d_src
    int* d_src = nullptr;          // source storage indices
    uint8_t* d_level = nullptr;    // per cube
    uint8_t* d_mask = nullptr;     // blocked bits per interior cell (ncubes * n^3), or null
    int32_t* d_org = nullptr;      // per cube, origin in fine-cell units (for set_blocked)
    double* d_ws = nullptr;        // BiCGStab vectors r, r0, p, v, s, t (storage size each)
    double* d_part = nullptr;      // block partial sums of the solve (2 x BCM_NB)
    ibm::BcmState* d_state = nullptr;
};

namespace ibm {
namespace {

constexpr int BCM_H = 2;

inline long long fdiv(long long a, long long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// cube storage index of cell (i, j, k) of cube q (interior 0..n-1, halo -H..n+H-1)
inline long long sidx(const ibm_bcm* m, long long q, int i, int j, int k) {
    const long long s = m->side;
    return q * s * s * s + (i + BCM_H) + s * ((j + BCM_H) + s * (long long)(k + BCM_H));
}

// the cube and cell containing a point given in half-fine-cell units (integers); false
// outside the domain
bool locate(const ibm_bcm* m, const long long p2[3], long long& q, int& lvl, int cell[3]) {
    const long long n = m->n;
    long long kc[3];
    for (int a = 0; a < 3; ++a) {
        if (p2[a] < 0 || p2[a] >= (long long)m->K[a] * 4 * n) return false;
        kc[a] = fdiv(p2[a], 4 * n);
    }
    const long long cc = kc[0] + (long long)m->K[0] * (kc[1] + (long long)m->K[1] * kc[2]);
    const long long first = m->first[cc];
    if (m->refine[cc]) {
        long long sub[3];
        for (int a = 0; a < 3; ++a) sub[a] = fdiv(p2[a] - kc[a] * 4 * n, 2 * n);
        q = first + sub[0] + 2 * sub[1] + 4 * sub[2];
        lvl = 1;
        for (int a = 0; a < 3; ++a) cell[a] = (int)fdiv(p2[a] - 2 * (long long)m->org[3 * q + a], 2);
    } else {
        q = first;
        lvl = 0;
        for (int a = 0; a < 3; ++a) cell[a] = (int)fdiv(p2[a] - 2 * (long long)m->org[3 * q + a], 4);
    }
    return true;
}

__global__ void __launch_bounds__(256) k_bcm_exchange(long long nhalo, const int* __restrict__ dst,
                                                      const int* __restrict__ off, const int* __restrict__ src,
                                                      double* __restrict__ x) {
    for (long long h = (long long)blockIdx.x * 256 + threadIdx.x; h < nhalo; h += (long long)gridDim.x * 256) {
        const int a = off[h], b = off[h + 1];
        double v;
        if (b - a == 1) {
            v = x[src[a]];
        } else {
            double s = 0.0;
            for (int e = a; e < b; ++e) s += x[src[e]];
            v = s / (double)(b - a);
        }
        x[dst[h]] = v;
    }
}

// (L x)_c = (x_-x + x_+x + x_-y + x_+y + x_-z + x_+z - 6 x_c) / dx^2 on every interior
// cell, from the cube's own storage (halos included)
// sum of the six neighbours of storage cell c in the order -x, +x, -y, +y, -z, +z, with
// the Neumann ghost x_c behind a blocked face (bit d of msk)
__device__ inline double bcm_nbsum(const double* __restrict__ x, long long c, long long side, long long s2,
                                   unsigned msk) {
    const double xc = x[c];
    double s = (msk & 1u) ? xc : x[c - 1];
    s = s + ((msk & 2u) ? xc : x[c + 1]);
    s = s + ((msk & 4u) ? xc : x[c - side]);
    s = s + ((msk & 8u) ? xc : x[c + side]);
    s = s + ((msk & 16u) ? xc : x[c - s2]);
    s = s + ((msk & 32u) ? xc : x[c + s2]);
    return s;
}

__global__ void __launch_bounds__(256) k_bcm_lap(long long ncubes, int n, int side, double dx0,
                                                 const uint8_t* __restrict__ level, const uint8_t* __restrict__ mask,
                                                 const double* __restrict__ x, double* __restrict__ y) {
    const long long per = (long long)n * n * n;
    const long long total = ncubes * per;
    const long long s2 = (long long)side * side, s3 = s2 * side;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const long long q = t / per;
        const long long r = t - q * per;
        const int i = (int)(r % n), j = (int)((r / n) % n), k = (int)(r / ((long long)n * n));
        const long long c = q * s3 + (i + BCM_H) + side * ((j + BCM_H) + (long long)side * (k + BCM_H));
        const double dx = level[q] ? 0.5 * dx0 : dx0;
        const double s = bcm_nbsum(x, c, side, s2, mask ? (unsigned)mask[t] : 0u);
        y[c] = (s - 6.0 * x[c]) / (dx * dx);
    }
}

__global__ void __launch_bounds__(256) k_bcm_zero(long long n, uint8_t* __restrict__ p) {
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long long)gridDim.x * 256) p[t] = 0;
}

// blocked bits of the cubes of one level from the level's uniform-grid tagging
// (gn cells per axis): cube cell (i, j, k) takes grid cell origin + (i, j, k)
__global__ void __launch_bounds__(256) k_bcm_mask(long long ncubes, int n, int lvl, const uint8_t* __restrict__ level,
                                                  const int32_t* __restrict__ org, int gx, int gy,
                                                  const uint8_t* __restrict__ blocked, uint8_t* __restrict__ mask) {
    const long long per = (long long)n * n * n;
    const long long total = ncubes * per;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const long long q = t / per;
        if (level[q] != lvl) continue;
        const long long r = t - q * per;
        const int i = (int)(r % n), j = (int)((r / n) % n), k = (int)(r / ((long long)n * n));
        const int f = lvl ? 1 : 2;   // the cube's cell size in fine units
        const long long ci = org[3 * q] / f + i, cj = org[3 * q + 1] / f + j, ck = org[3 * q + 2] / f + k;
        mask[t] = blocked[ci + (long long)gx * (cj + (long long)gy * ck)];
    }
}

// One half sweep of red-black SOR on the cubes: every interior cell of the colour
// (parity of its cube-local i + j + k) gets x_c += omega (b_c - (L x)_c) / (-6 / dx^2);
// it reads cells of the other colour and halo copies only (exchanged before the launch).
__global__ void __launch_bounds__(256) k_bcm_sor(long long ncubes, int n, int side, double dx0,
                                                 const uint8_t* __restrict__ level, const uint8_t* __restrict__ mask,
                                                 const double* __restrict__ b, double* __restrict__ x, int colour,
                                                 double omega) {
    const long long per = (long long)n * n * n;
    const long long total = ncubes * per;
    const long long s2 = (long long)side * side, s3 = s2 * side;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const long long q = t / per;
        const long long r = t - q * per;
        const int i = (int)(r % n), j = (int)((r / n) % n), k = (int)(r / ((long long)n * n));
        if (((i + j + k) & 1) != colour) continue;
        const long long c = q * s3 + (i + BCM_H) + side * ((j + BCM_H) + (long long)side * (k + BCM_H));
        const double dx = level[q] ? 0.5 * dx0 : dx0;
        const unsigned msk = mask ? (unsigned)mask[t] : 0u;
        const int nopen = 6 - __builtin_popcount(msk & 63u);
        if (nopen == 0) continue;   // a cell without open faces keeps its value
        const double s = bcm_nbsum(x, c, side, s2, msk);
        const double xc = x[c];
        const double lx = (s - 6.0 * xc) / (dx * dx);
        const double diag = -(double)nopen / (dx * dx);
        x[c] = xc + omega * (b[c] - lx) / diag;
    }
}

// ------------------------------------------------------------ solve on the cubes

constexpr int BCM_NB = 1024;   // blocks of the reduction launches (partials per sum)
enum { BCM_RUNNING = 0, BCM_CONVERGED = 1, BCM_CONVERGED_HALF = 2, BCM_BREAKDOWN = 3, BCM_MAX_ITER = 4,
       BCM_NAN = 5, BCM_ZERO_RHS = 6 };
enum { BS_INIT, BS_RHO, BS_ALPHA, BS_HALF, BS_OMEGA, BS_RES };

// storage index of interior cell t = q n^3 + i + n (j + n k)
__device__ inline long long bcm_cell(long long t, long long per, int n, long long side) {
    const long long q = t / per;
    const long long r = t - q * per;
    const long long i = r % n, j = (r / n) % n, k = r / ((long long)n * n);
    return q * side * side * side + (i + BCM_H) + side * ((j + BCM_H) + side * (k + BCM_H));
}

// block partials of a0 . b0 (and a1 . b1) over the interiors, written to part[blockIdx]
// (and part[gridDim + blockIdx]); nothing once the solve has stopped
template <int NV>
__global__ void __launch_bounds__(NT) k_bcm_dot(long long total, int n, int side, const double* __restrict__ a0,
                                                const double* __restrict__ b0, const double* __restrict__ a1,
                                                const double* __restrict__ b1, double* __restrict__ part,
                                                const BcmState* __restrict__ st) {
    if (st->done) return;
    const long long per = (long long)n * n * n;
    double v[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) v[a] = 0.0;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < total; t += (long long)gridDim.x * NT) {
        const long long c = bcm_cell(t, per, n, side);
        v[0] += a0[c] * b0[c];
        if (NV > 1) v[NV - 1] += a1[c] * b1[c];
    }
    __shared__ double sh[4 * NV];
    block_reduce<NV>(v, sh);
    if (threadIdx.x == 0)
        for (int a = 0; a < NV; ++a) part[a * gridDim.x + blockIdx.x] = v[a];
}

// One block: the two sums of nb partials each (in block order), then the decision of
// the step `mode` of iteration it (the BiCGStab steps of the flow solver's algorithm;
// BS_RES stores a residual check).
__global__ void __launch_bounds__(NT) k_bcm_scalar(const double* __restrict__ part, int nb, BcmState* st, int mode,
                                                   int it, int max_iter, double tol) {
    if (st->done && mode != BS_RES) return;
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += NT) {
        v[0] += part[b];
        v[1] += part[nb + b];
    }
    __shared__ double sh[8];
    block_reduce<2>(v, sh);
    if (threadIdx.x != 0) return;
    const double tol2 = tol * tol * st->bb;
    auto stop = [&](int why, int iters) {
        st->done = why;
        st->iters = iters;
    };
    switch (mode) {
    case BS_INIT:   // v = (b . b, r . r)
        st->bb = v[0];
        st->rr = v[1];
        st->rho_old = st->alpha = st->omega = 1.0;
        st->beta = 0.0;
        st->iters = 0;
        if (!(v[0] == v[0]) || !(v[1] == v[1])) st->done = BCM_NAN;
        else if (v[0] == 0.0) st->done = BCM_ZERO_RHS;
        break;
    case BS_RHO:    // v = (r0 . r, r . r), at the start of iteration it
        st->rr = v[1];
        if (!(v[1] == v[1]) || !(v[0] == v[0])) stop(BCM_NAN, it);
        else if (v[1] <= tol2) stop(BCM_CONVERGED, it);
        else if (it >= max_iter) stop(BCM_MAX_ITER, it);
        else if (v[0] == 0.0) stop(BCM_BREAKDOWN, it);
        else {
            st->beta = (v[0] / st->rho_old) * (st->alpha / st->omega);
            st->rho = v[0];
        }
        break;
    case BS_ALPHA:  // v = (r0 . v, -)
        if (!(v[0] == v[0])) stop(BCM_NAN, it);
        else if (v[0] == 0.0) stop(BCM_BREAKDOWN, it);
        else st->alpha = st->rho / v[0];
        break;
    case BS_HALF:   // v = (s . s, -): halfway stop, x += alpha p follows
        if (!(v[0] == v[0])) stop(BCM_NAN, it);
        else if (v[0] <= tol2) stop(BCM_CONVERGED_HALF, it + 1);
        break;
    case BS_OMEGA:  // v = (t . s, t . t)
        if (!(v[0] == v[0]) || !(v[1] == v[1])) stop(BCM_NAN, it);
        else if (v[1] == 0.0 || v[0] == 0.0) stop(BCM_BREAKDOWN, it);
        else {
            st->omega = v[0] / v[1];
            st->rho_old = st->rho;
        }
        break;
    default:        // BS_RES: v = ((b - L x) . (b - L x), b . b)
        st->rr = v[0];
        st->bb = v[1];
        break;
    }
}

// r = b - y (y = L x), r0 = r, p = v = 0; partials of b . b and r . r
__global__ void __launch_bounds__(NT) k_bcm_bs_init(long long total, int n, int side, const double* __restrict__ b,
                                                    const double* __restrict__ y, double* __restrict__ r,
                                                    double* __restrict__ r0, double* __restrict__ p,
                                                    double* __restrict__ v, double* __restrict__ part) {
    const long long per = (long long)n * n * n;
    double acc[2] = {0.0, 0.0};
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < total; t += (long long)gridDim.x * NT) {
        const long long c = bcm_cell(t, per, n, side);
        const double rc = b[c] - y[c];
        r[c] = rc;
        r0[c] = rc;
        p[c] = 0.0;
        v[c] = 0.0;
        acc[0] += b[c] * b[c];
        acc[1] += rc * rc;
    }
    __shared__ double sh[8];
    block_reduce<2>(acc, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc[0];
        part[gridDim.x + blockIdx.x] = acc[1];
    }
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(NT) k_bcm_bs_p(long long total, int n, int side, const double* __restrict__ r,
                                                 const double* __restrict__ v, double* __restrict__ p,
                                                 const BcmState* __restrict__ st) {
    if (st->done) return;
    const long long per = (long long)n * n * n;
    const double beta = st->beta, omega = st->omega;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < total; t += (long long)gridDim.x * NT) {
        const long long c = bcm_cell(t, per, n, side);
        p[c] = r[c] + beta * (p[c] - omega * v[c]);
    }
}

// s = r - alpha v, with partials of s . s
__global__ void __launch_bounds__(NT) k_bcm_bs_s(long long total, int n, int side, const double* __restrict__ r,
                                                 const double* __restrict__ v, double* __restrict__ s,
                                                 double* __restrict__ part, const BcmState* __restrict__ st) {
    if (st->done) return;
    const long long per = (long long)n * n * n;
    const double alpha = st->alpha;
    double acc[1] = {0.0};
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < total; t += (long long)gridDim.x * NT) {
        const long long c = bcm_cell(t, per, n, side);
        const double sc = r[c] - alpha * v[c];
        s[c] = sc;
        acc[0] += sc * sc;
    }
    __shared__ double sh[4];
    block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc[0];
        part[gridDim.x + blockIdx.x] = 0.0;
    }
}

// the halfway stop of iteration it: x += alpha p (exactly once: only the launch of the
// iteration that stopped there matches)
__global__ void __launch_bounds__(NT) k_bcm_bs_xhalf(long long total, int n, int side, const double* __restrict__ p,
                                                     double* __restrict__ x, const BcmState* __restrict__ st, int it) {
    if (st->done != BCM_CONVERGED_HALF || st->iters != it + 1) return;
    const long long per = (long long)n * n * n;
    const double alpha = st->alpha;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < total; t += (long long)gridDim.x * NT) {
        const long long c = bcm_cell(t, per, n, side);
        x[c] = x[c] + alpha * p[c];
    }
}

// x += alpha p + omega s; r = s - omega t
__global__ void __launch_bounds__(NT) k_bcm_bs_xr(long long total, int n, int side, const double* __restrict__ p,
                                                  const double* __restrict__ s, const double* __restrict__ tv,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  const BcmState* __restrict__ st) {
    if (st->done) return;
    const long long per = (long long)n * n * n;
    const double alpha = st->alpha, omega = st->omega;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < total; t += (long long)gridDim.x * NT) {
        const long long c = bcm_cell(t, per, n, side);
        x[c] = x[c] + alpha * p[c] + omega * s[c];
        r[c] = s[c] - omega * tv[c];
    }
}

// partials of |b - L x|^2 and |b|^2 over the interiors (x exchanged before the launch)
__global__ void __launch_bounds__(NT) k_bcm_resid(long long ncubes, int n, int side, double dx0,
                                                  const uint8_t* __restrict__ level, const uint8_t* __restrict__ mask,
                                                  const double* __restrict__ b, const double* __restrict__ x,
                                                  double* __restrict__ part) {
    const long long per = (long long)n * n * n;
    const long long total = ncubes * per;
    const long long s2 = (long long)side * side;
    double acc[2] = {0.0, 0.0};
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < total; t += (long long)gridDim.x * NT) {
        const long long q = t / per;
        const long long c = bcm_cell(t, per, n, side);
        const double dx = level[q] ? 0.5 * dx0 : dx0;
        const double lx = (bcm_nbsum(x, c, side, s2, mask ? (unsigned)mask[t] : 0u) - 6.0 * x[c]) / (dx * dx);
        const double rc = b[c] - lx;
        acc[0] += rc * rc;
        acc[1] += b[c] * b[c];
    }
    __shared__ double sh[8];
    block_reduce<2>(acc, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc[0];
        part[gridDim.x + blockIdx.x] = acc[1];
    }
}

__global__ void __launch_bounds__(NT) k_bcm_zero_interior(long long total, int n, int side, double* __restrict__ x) {
    const long long per = (long long)n * n * n;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < total; t += (long long)gridDim.x * NT)
        x[bcm_cell(t, per, n, side)] = 0.0;
}

__global__ void k_bcm_state_reset(BcmState* st) {
    if (threadIdx.x == 0) {
        st->bb = st->rr = st->rho = st->rho_old = st->alpha = st->omega = st->beta = 0.0;
        st->done = BCM_RUNNING;
        st->iters = 0;
    }
}

}  // namespace
}  // namespace ibm

using namespace ibm;

extern "C" {

int ibm_bcm_create(const int32_t K[3], int32_t n, double dx0, const double origin[3], const uint8_t* refine_host,
                   ibm_bcm** out) try {
    if (!K || !origin || !refine_host || !out) {
        set_error("ibm_bcm_create: null argument");
        return IBM_ERR_ARG;
    }
    *out = nullptr;
    if (K[0] < 1 || K[1] < 1 || K[2] < 1 || n < 2 || (n & 1) || n > 1024 || !(dx0 > 0.0)) {
        set_error("ibm_bcm_create: need K >= 1, even n in [2, 1024], dx0 > 0");
        return IBM_ERR_ARG;
    }
    {
        // sizes first, before any table is built: origins in fine cells are 32-bit, and
        // the storage and the halo tables hold 32-bit indices (up to 8 sources per halo
        // cell)
        const long long side = n + 2 * BCM_H;
        for (int a = 0; a < 3; ++a)
            if ((long long)K[a] * 2 * n >= 0x7fffffffLL) {
                set_error("ibm_bcm_create: the domain exceeds 2^31 fine cells along an axis");
                return IBM_ERR_ARG;
            }
        const long long nc = (long long)K[0] * K[1] * K[2];
        if (nc >= 0x7fffffffLL / (side * side * side)) {
            set_error("ibm_bcm_create: cube storage exceeds 2^31 entries");
            return IBM_ERR_ARG;
        }
        long long nref = 0;
        for (long long cc = 0; cc < nc; ++cc) nref += refine_host[cc] ? 1 : 0;
        const long long ncubes = nc + 7 * nref;
        if (ncubes * side * side * side >= 0x7fffffffLL || 8 * ncubes * 6LL * BCM_H * n * n >= 0x7fffffffLL) {
            set_error("ibm_bcm_create: cube storage or halo tables exceed 2^31 entries");
            return IBM_ERR_ARG;
        }
    }
    ibm_bcm* m = new (std::nothrow) ibm_bcm();
    if (!m) {
        set_error("ibm_bcm_create: host allocation failed");
        return IBM_ERR_OOM;
    }
    if (hipGetDevice(&m->device) != hipSuccess) {
        (void)hipGetLastError();
        delete m;
        set_error("ibm_bcm_create: no current HIP device");
        return IBM_ERR_HIP;
    }
    for (int a = 0; a < 3; ++a) {
        m->K[a] = K[a];
        m->origin[a] = origin[a];
    }
    m->n = n;
    m->side = n + 2 * BCM_H;
    m->dx0 = dx0;
    const long long nc = (long long)K[0] * K[1] * K[2];
    m->refine.assign(refine_host, refine_host + nc);
    m->first.resize(nc);
    for (int kz = 0; kz < K[2]; ++kz)
        for (int ky = 0; ky < K[1]; ++ky)
            for (int kx = 0; kx < K[0]; ++kx) {
                const long long cc = kx + (long long)K[0] * (ky + (long long)K[1] * kz);
                m->first[cc] = (long long)m->level.size();
                const int base[3] = {kx * 2 * n, ky * 2 * n, kz * 2 * n};
                if (m->refine[cc]) {
                    for (int cz = 0; cz < 2; ++cz)
                        for (int cy = 0; cy < 2; ++cy)
                            for (int cx = 0; cx < 2; ++cx) {
                                m->level.push_back(1);
                                m->org.push_back(base[0] + cx * n);
                                m->org.push_back(base[1] + cy * n);
                                m->org.push_back(base[2] + cz * n);
                            }
                } else {
                    m->level.push_back(0);
                    m->org.push_back(base[0]);
                    m->org.push_back(base[1]);
                    m->org.push_back(base[2]);
                }
            }
    m->ncubes = (long long)m->level.size();
    m->size = m->ncubes * (long long)m->side * m->side * m->side;
    // the halo tables hold 32-bit storage indices and 32-bit source offsets (up to 8
    // sources per halo cell)
    const long long halo_bound = m->ncubes * 6LL * BCM_H * n * n;
    if (m->size >= 0x7fffffffLL || 8 * halo_bound >= 0x7fffffffLL) {
        delete m;
        set_error("ibm_bcm_create: cube storage or halo tables exceed 2^31 entries");
        return IBM_ERR_ARG;
    }
    // face-halo sources
    std::vector<int> dst, off(1, 0), src;
    dst.reserve((size_t)(m->ncubes * 6 * BCM_H * n * n));
    for (long long q = 0; q < m->ncubes; ++q) {
        const int lvl = m->level[q];
        const long long w2 = lvl ? 2 : 4;   // this cube's cell size in half-fine units
        const long long o2[3] = {2LL * m->org[3 * q], 2LL * m->org[3 * q + 1], 2LL * m->org[3 * q + 2]};
        for (int axis = 0; axis < 3; ++axis)
            for (int sgn = -1; sgn <= 1; sgn += 2)
                for (int layer = 1; layer <= BCM_H; ++layer) {
                    const int ci = sgn > 0 ? n - 1 + layer : -layer;
                    for (int a = 0; a < n; ++a)
                        for (int b = 0; b < n; ++b) {
                            int c[3];
                            c[axis] = ci;
                            c[(axis + 1) % 3] = a;
                            c[(axis + 2) % 3] = b;
                            long long p2[3];
                            for (int d = 0; d < 3; ++d) p2[d] = o2[d] + (2LL * c[d] + 1) * (w2 / 2);
                            dst.push_back((int)sidx(m, q, c[0], c[1], c[2]));
                            long long q2;
                            int l2, cell[3];
                            if (!locate(m, p2, q2, l2, cell)) {
                                int mm[3] = {c[0], c[1], c[2]};
                                mm[axis] = sgn > 0 ? n - layer : layer - 1;
                                src.push_back((int)sidx(m, q, mm[0], mm[1], mm[2]));
                            } else if (l2 <= lvl || lvl == 1) {
                                src.push_back((int)sidx(m, q2, cell[0], cell[1], cell[2]));
                            } else {
                                // coarse halo cell over 8 fine cells, z, y, x order
                                for (int dz = 0; dz < 2; ++dz)
                                    for (int dy = 0; dy < 2; ++dy)
                                        for (int dxx = 0; dxx < 2; ++dxx) {
                                            const int dd[3] = {dxx, dy, dz};
                                            long long pp[3];
                                            for (int d = 0; d < 3; ++d)
                                                pp[d] = o2[d] + 4LL * c[d] + 2LL * dd[d] + 1;
                                            long long q3 = -1;
                                            int l3 = 0, c3[3] = {0, 0, 0};
                                            // inside by construction; a miss is caught below
                                            if (locate(m, pp, q3, l3, c3))
                                                src.push_back((int)sidx(m, q3, c3[0], c3[1], c3[2]));
                                            else
                                                src.push_back(-1);
                                        }
                            }
                            off.push_back((int)src.size());
                        }
                }
    }
    m->nhalo = (long long)dst.size();
    // every destination is a halo cell and every source an interior cell of the storage
    // (the exchange then neither reads what it writes nor leaves the storage)
    {
        const long long s = m->side, s3 = s * s * s;
        auto decode = [&](long long v, int& i, int& j, int& k) {
            const long long r = v % s3;
            i = (int)(r % s) - BCM_H;
            j = (int)((r / s) % s) - BCM_H;
            k = (int)(r / (s * s)) - BCM_H;
        };
        bool ok = (long long)off.size() == m->nhalo + 1;
        for (long long h = 0; ok && h < m->nhalo; ++h) {
            int i, j, k;
            if (dst[h] < 0 || dst[h] >= m->size) ok = false;
            else {
                decode(dst[h], i, j, k);
                const int inside = (i >= 0 && i < n) + (j >= 0 && j < n) + (k >= 0 && k < n);
                if (inside != 2) ok = false;    // a face halo cell: exactly one coordinate outside
            }
            const int cnt = off[h + 1] - off[h];
            if (cnt != 1 && cnt != 8) ok = false;
        }
        for (size_t e = 0; ok && e < src.size(); ++e) {
            int i, j, k;
            if (src[e] < 0 || src[e] >= m->size) ok = false;
            else {
                decode(src[e], i, j, k);
                if (i < 0 || i >= n || j < 0 || j >= n || k < 0 || k >= n) ok = false;
            }
        }
        if (!ok) {
            delete m;
            set_error("ibm_bcm_create: inconsistent halo tables");
            return IBM_ERR_ARG;
        }
    }
    std::vector<uint8_t> lv(m->level.begin(), m->level.end());
    if (ibm::dev_malloc((void**)&m->d_dst, sizeof(int) * dst.size()) != hipSuccess ||
        ibm::dev_malloc((void**)&m->d_off, sizeof(int) * off.size()) != hipSuccess ||
        ibm::dev_malloc((void**)&m->d_src, sizeof(int) * src.size()) != hipSuccess ||
        ibm::dev_malloc((void**)&m->d_level, lv.size()) != hipSuccess ||
        ibm::dev_malloc((void**)&m->d_org, sizeof(int32_t) * m->org.size()) != hipSuccess) {
        (void)hipGetLastError();
        set_error("ibm_bcm_create: out of device memory");
        (void)hipFree(m->d_dst);
        (void)hipFree(m->d_off);
        (void)hipFree(m->d_src);
        (void)hipFree(m->d_level);
        (void)hipFree(m->d_org);
        delete m;
        return IBM_ERR_OOM;
    }
    if (hipMemcpy(m->d_dst, dst.data(), sizeof(int) * dst.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_src, src.data(), sizeof(int) * src.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_level, lv.data(), lv.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_org, m->org.data(), sizeof(int32_t) * m->org.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        set_error("ibm_bcm_create: copy of the halo tables failed");
        ibm_bcm_destroy(m);
        return IBM_ERR_HIP;
    }
    *out = m;
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_bcm_destroy(ibm_bcm* m) try {
    if (!m) return IBM_OK;
    (void)hipFree(m->d_dst);
    (void)hipFree(m->d_off);
    (void)hipFree(m->d_src);
    (void)hipFree(m->d_level);
    (void)hipFree(m->d_org);
    (void)hipFree(m->d_mask);
    (void)hipFree(m->d_ws);
    (void)hipFree(m->d_part);
    (void)hipFree(m->d_state);
    delete m;
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_bcm_info(const ibm_bcm* m, int64_t* ncubes, int64_t* size, int64_t* nhalo, int32_t* levels_host,
                 int32_t* origins_host) try {
    if (!m) {
        set_error("ibm_bcm_info: null grid");
        return IBM_ERR_ARG;
    }
    if (ncubes) *ncubes = m->ncubes;
    if (size) *size = m->size;
    if (nhalo) *nhalo = m->nhalo;
    if (levels_host)
        for (long long q = 0; q < m->ncubes; ++q) levels_host[q] = m->level[q];
    if (origins_host)
        for (long long q = 0; q < 3 * m->ncubes; ++q) origins_host[q] = m->org[q];
    return IBM_OK;
} IBM_CATCH_ALL

// the grid's tables live on the device it was created on
static int bcm_device_ok(const ibm_bcm* m) {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess || d != m->device) {
        (void)hipGetLastError();
        set_error("building-cube grid used on another device than the one it was created on");
        return IBM_ERR_ARG;
    }
    return IBM_OK;
}

int ibm_bcm_exchange(const ibm_bcm* m, double* data_dev, void* stream) try {
    if (!m || !data_dev) {
        set_error("ibm_bcm_exchange: null argument");
        return IBM_ERR_ARG;
    }
    if (int rc = bcm_device_ok(m)) return rc;
    const long long nb = std::min<long long>((m->nhalo + 255) / 256, 8192);
    if (nb > 0)
        k_bcm_exchange<<<(int)nb, 256, 0, (hipStream_t)stream>>>(m->nhalo, m->d_dst, m->d_off, m->d_src, data_dev);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_bcm_laplacian(const ibm_bcm* m, const double* x_dev, double* y_dev, void* stream) try {
    if (!m || !x_dev || !y_dev || x_dev == y_dev) {
        set_error("ibm_bcm_laplacian: null or aliased argument");
        return IBM_ERR_ARG;
    }
    if (int rc = bcm_device_ok(m)) return rc;
    const long long total = m->ncubes * (long long)m->n * m->n * m->n;
    const long long nb = std::min<long long>((total + 255) / 256, 16384);
    if (nb > 0)
        k_bcm_lap<<<(int)nb, 256, 0, (hipStream_t)stream>>>(m->ncubes, m->n, m->side, m->dx0, m->d_level,
                                                             m->d_mask, x_dev, y_dev);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_bcm_sor(const ibm_bcm* m, const double* b_dev, double* x_dev, double omega, int32_t sweeps, void* stream) try {
    if (!m || !b_dev || !x_dev || b_dev == x_dev || sweeps < 0 || !(omega > 0.0 && omega < 2.0)) {
        set_error("ibm_bcm_sor: need distinct b and x, sweeps >= 0, 0 < omega < 2");
        return IBM_ERR_ARG;
    }
    if (int rc = bcm_device_ok(m)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const long long total = m->ncubes * (long long)m->n * m->n * m->n;
    const int nb = (int)std::min<long long>((total + 255) / 256, 16384);
    for (int it = 0; it < sweeps; ++it)
        for (int colour = 0; colour < 2; ++colour) {
            if (int rc = ibm_bcm_exchange(m, x_dev, stream)) return rc;
            k_bcm_sor<<<nb, 256, 0, s>>>(m->ncubes, m->n, m->side, m->dx0, m->d_level, m->d_mask, b_dev, x_dev,
                                         colour, omega);
        }
    IBM_HIP(hipGetLastError());
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_bcm_set_blocked(ibm_bcm* m, int32_t level, const uint8_t* blocked_dev, void* stream) try {
    if (!m || !blocked_dev || (level != 0 && level != 1)) {
        set_error("ibm_bcm_set_blocked: need a grid, level 0 or 1 and the level's blocked bits");
        return IBM_ERR_ARG;
    }
    if (int rc = bcm_device_ok(m)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const long long total = m->ncubes * (long long)m->n * m->n * m->n;
    if (!m->d_mask) {
        // set-up: the mask starts all open, each level is filled by its own call
        if (ibm::dev_malloc((void**)&m->d_mask, (size_t)total) != hipSuccess) {
            (void)hipGetLastError();
            m->d_mask = nullptr;
            set_error("ibm_bcm_set_blocked: out of device memory for the cube masks");
            return IBM_ERR_OOM;
        }
        k_bcm_zero<<<(int)std::min<long long>((total + 255) / 256, 16384), 256, 0, s>>>(total, m->d_mask);
    }
    const int f = level ? 2 : 1;
    const int gx = m->K[0] * m->n * f, gy = m->K[1] * m->n * f;
    const int nb = (int)std::min<long long>((total + 255) / 256, 16384);
    k_bcm_mask<<<nb, 256, 0, s>>>(m->ncubes, m->n, level, m->d_level, m->d_org, gx, gy, blocked_dev, m->d_mask);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_bcm_solve(ibm_bcm* m, int32_t kind, const double* b_dev, double* x_dev, double omega, double tol,
                  int32_t max_iter, int32_t check_every, int32_t* iters_out, double* rel_residual_out,
                  void* stream) try {
    if (!m || !b_dev || !x_dev || b_dev == x_dev || (kind != IBM_BCM_BICGSTAB && kind != IBM_BCM_SOR) ||
        !(tol > 0.0) || max_iter < 0 || check_every < 1 ||
        (kind == IBM_BCM_SOR && !(omega > 0.0 && omega < 2.0))) {
        set_error("ibm_bcm_solve: need distinct b and x, kind BICGSTAB or SOR, tol > 0, max_iter >= 0, "
                  "check_every >= 1 and 0 < omega < 2 for SOR");
        return IBM_ERR_ARG;
    }
    if (int rc = bcm_device_ok(m)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const long long total = m->ncubes * (long long)m->n * m->n * m->n;
    const int nb = (int)std::max<long long>(1, std::min<long long>((total + NT - 1) / NT, BCM_NB));
    const int nbc = (int)std::min<long long>((total + 255) / 256, 16384);
    // set-up: the partial sums and the state, and for BiCGStab its six vectors
    auto grab = [&](void** p, size_t bytes) {
        if (*p) return true;
        if (ibm::dev_malloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return false;
        }
        return true;
    };
    if (!grab((void**)&m->d_part, 2 * BCM_NB * sizeof(double)) || !grab((void**)&m->d_state, sizeof(BcmState)) ||
        (kind == IBM_BCM_BICGSTAB && !grab((void**)&m->d_ws, 6 * (size_t)m->size * sizeof(double)))) {
        set_error("ibm_bcm_solve: out of device memory for the solve's workspace");
        return IBM_ERR_OOM;
    }
    BcmState* st = m->d_state;
    double* part = m->d_part;
    BcmState h{};
    auto read_state = [&]() -> int {
        IBM_HIP(hipMemcpyAsync(&h, st, sizeof(BcmState), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        return IBM_OK;
    };
    auto exchange = [&](double* v) {
        const long long nbx = std::min<long long>((m->nhalo + 255) / 256, 8192);
        if (nbx > 0) k_bcm_exchange<<<(int)nbx, 256, 0, s>>>(m->nhalo, m->d_dst, m->d_off, m->d_src, v);
    };
    auto lap = [&](const double* v, double* y) {
        k_bcm_lap<<<nbc, 256, 0, s>>>(m->ncubes, m->n, m->side, m->dx0, m->d_level, m->d_mask, v, y);
    };
    // the true relative residual of x into h (rr, bb)
    auto true_residual = [&]() -> int {
        exchange(x_dev);
        k_bcm_resid<<<nb, NT, 0, s>>>(m->ncubes, m->n, m->side, m->dx0, m->d_level, m->d_mask, b_dev, x_dev, part);
        k_bcm_scalar<<<1, NT, 0, s>>>(part, nb, st, BS_RES, 0, 0, tol);
        IBM_HIP(hipGetLastError());
        return read_state();
    };
    k_bcm_state_reset<<<1, 64, 0, s>>>(st);
    IBM_HIP(hipGetLastError());
    int iters = 0, rc = IBM_OK;
    double rel = 0.0;
    if (kind == IBM_BCM_SOR) {
        // red-black SOR in groups of check_every sweeps, the true residual checked
        // before the first and after every group
        while (true) {
            if (int e = true_residual()) return e;
            if (!(h.rr == h.rr) || !(h.bb == h.bb)) {
                rc = IBM_ERR_NAN;
                rel = h.rr;
                break;
            }
            rel = h.bb == 0.0 ? 0.0 : std::sqrt(h.rr / h.bb);
            if (rel <= tol) break;
            if (iters >= max_iter) {
                rc = IBM_NOT_CONVERGED;
                break;
            }
            const int k = std::min(check_every, max_iter - iters);
            for (int it = 0; it < k; ++it)
                for (int colour = 0; colour < 2; ++colour) {
                    exchange(x_dev);
                    k_bcm_sor<<<nbc, 256, 0, s>>>(m->ncubes, m->n, m->side, m->dx0, m->d_level, m->d_mask, b_dev,
                                                  x_dev, colour, omega);
                }
            IBM_HIP(hipGetLastError());
            iters += k;
        }
    } else {
        const long long sz = m->size;
        double *r = m->d_ws, *r0 = r + sz, *p = r0 + sz, *v = p + sz, *sv = v + sz, *tv = sv + sz;
        // r = b - L x (L x into t, free until the first iteration's second product)
        exchange(x_dev);
        lap(x_dev, tv);
        k_bcm_bs_init<<<nb, NT, 0, s>>>(total, m->n, m->side, b_dev, tv, r, r0, p, v, part);
        k_bcm_scalar<<<1, NT, 0, s>>>(part, nb, st, BS_INIT, 0, max_iter, tol);
        IBM_HIP(hipGetLastError());
        if (int e = read_state()) return e;
        if (h.done == BCM_ZERO_RHS) {
            // b = 0: x = 0
            k_bcm_zero_interior<<<nb, NT, 0, s>>>(total, m->n, m->side, x_dev);
            IBM_HIP(hipGetLastError());
        } else if (h.done == BCM_RUNNING) {
            for (int it = 0; it <= max_iter; ++it) {
                k_bcm_dot<2><<<nb, NT, 0, s>>>(total, m->n, m->side, r0, r, r, r, part, st);
                k_bcm_scalar<<<1, NT, 0, s>>>(part, nb, st, BS_RHO, it, max_iter, tol);
                if (it == max_iter) break;
                k_bcm_bs_p<<<nb, NT, 0, s>>>(total, m->n, m->side, r, v, p, st);
                exchange(p);
                lap(p, v);
                k_bcm_dot<1><<<nb, NT, 0, s>>>(total, m->n, m->side, r0, v, nullptr, nullptr, part, st);
                k_bcm_scalar<<<1, NT, 0, s>>>(part, nb, st, BS_ALPHA, it, max_iter, tol);
                k_bcm_bs_s<<<nb, NT, 0, s>>>(total, m->n, m->side, r, v, sv, part, st);
                k_bcm_scalar<<<1, NT, 0, s>>>(part, nb, st, BS_HALF, it, max_iter, tol);
                k_bcm_bs_xhalf<<<nb, NT, 0, s>>>(total, m->n, m->side, p, x_dev, st, it);
                exchange(sv);
                lap(sv, tv);
                k_bcm_dot<2><<<nb, NT, 0, s>>>(total, m->n, m->side, tv, sv, tv, tv, part, st);
                k_bcm_scalar<<<1, NT, 0, s>>>(part, nb, st, BS_OMEGA, it, max_iter, tol);
                k_bcm_bs_xr<<<nb, NT, 0, s>>>(total, m->n, m->side, p, sv, tv, x_dev, r, st);
                IBM_HIP(hipGetLastError());
                if ((it + 1) % check_every == 0) {
                    if (int e = read_state()) return e;
                    if (h.done != BCM_RUNNING) break;
                }
            }
            if (int e = read_state()) return e;
        }
        const int why = h.done;
        iters = h.iters;
        if (why == BCM_NAN) rc = IBM_ERR_NAN;
        else if (why == BCM_MAX_ITER || why == BCM_BREAKDOWN) rc = IBM_NOT_CONVERGED;
        if (int e = true_residual()) return e;
        rel = h.bb == 0.0 ? 0.0 : std::sqrt(h.rr / h.bb);
        if (rc == IBM_OK && !(rel == rel)) rc = IBM_ERR_NAN;
    }
    if (iters_out) *iters_out = iters;
    if (rel_residual_out) *rel_residual_out = rel;
    if (rc == IBM_ERR_NAN) set_error("ibm_bcm_solve: non-finite residual");
    else if (rc == IBM_NOT_CONVERGED) set_error("ibm_bcm_solve: tolerance not met (iteration cap or breakdown)");
    return rc;
} IBM_CATCH_ALL

}  // extern "C"
