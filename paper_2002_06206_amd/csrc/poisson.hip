// Pressure Poisson solve (eq. poisson) on the immersed-boundary stencil.
//
// A = -L, L p = (1/dx^2)[sum over open faces (p_nb - p_c) - 2 p_c per outlet face],
// is symmetric positive semi-definite (blocking is per face, seen from both sides),
// so the plain solver is Jacobi-preconditioned conjugate gradients in FP64, warm
// started.
//
// MI355X design:
//  * one byte per cell ("pressure code": bits 0-5 open faces incl. periodic wraps,
//    bits 6-7 number of outlet faces) carries the whole operator: the diagonal is
//    popcount(open) + 2 * outlets, every open face couples with weight 1;
//  * the SpMV marches each 64x4 column tile through a slab of z-planes keeping the
//    planes z-1, z, z+1 in registers; the slabs are laid out so each XCD owns a
//    contiguous range of z and its L2 serves the x/y neighbours;
//  * no grid-wide fences: a reduction kernel only writes one partial per block, and
//    every block of the consumer kernel sums those partials itself in a fixed order
//    (identical in every block, so the scalars alpha, beta and the convergence test
//    agree everywhere and the result is deterministic);
//  * the two <r,*> reductions ping-pong between two partial sets by iteration
//    parity so that rz of the previous iteration is still available.
// Convergence is decided on the device after every update; later sweeps of the
// batch exit at once.  The host polls between batches.

#include <type_traits>

#include <cmath>

#include "common.h"

namespace ibm {
namespace {

__device__ inline double jacobi_count(uint8_t pc) {
    return (double)(__builtin_popcount((unsigned)(pc & 0x3F)) + 2 * (pc >> 6));
}

// Work item = (column tile, z slab).  Items are ordered slab-major; the XCD chunk
// remap hands every XCD a contiguous run of slabs.
struct Slabs {
    int nzc;         // slabs
    long long items; // tiles_xy * nzc
};


// (L x)_c from the pressure code and the three planes of the column
__device__ inline double lap_code(uint8_t pc, double xc, double xw, double xe, double xs, double xn, double xb,
                                  double xt, double idx2) {
    double acc = -jacobi_count(pc) * xc;
    if (pc & 1) acc += xw;
    if (pc & 2) acc += xe;
    if (pc & 4) acc += xs;
    if (pc & 8) acc += xn;
    if (pc & 16) acc += xb;
    if (pc & 32) acc += xt;
    return acc * idx2;
}

// Generic z-marching sweep over (tile, slab) items.  For each cell it hands the
// functor the code byte and the 7 values of x needed by L.
template <class T, class F>
__device__ inline void march(const Geo& g, const uint8_t* __restrict__ pcode, const T* __restrict__ x, F&& f) {
    const int nzc = slab_count(g.nz);
    const long long tiles = (long long)g.ntx * g.nty;
    const long long items = tiles * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    for (long long w = w0; w < w1; ++w) {
        const int zc = (int)(w / tiles);
        const long long t = w % tiles;
        const int i = (int)(t % g.ntx) * TX + (threadIdx.x % TX);
        const int j = (int)(t / g.ntx) * TY + (threadIdx.x / TX);
        const int z0 = (int)((long long)g.nz * zc / nzc), z1 = (int)((long long)g.nz * (zc + 1) / nzc);
        if (i >= g.nx || j >= g.ny) continue;
        const int iw = i == 0 ? g.nx - 1 : i - 1, ie = i == g.nx - 1 ? 0 : i + 1;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j == g.ny - 1 ? 0 : j + 1;
        const long long col = (long long)i + (long long)g.nx * j;
        const long long ow = (long long)iw + (long long)g.nx * j - col;
        const long long oe = (long long)ie + (long long)g.nx * j - col;
        const long long os = (long long)i + (long long)g.nx * js - col;
        const long long on = (long long)i + (long long)g.nx * jn - col;
        int zb = z0 == 0 ? g.nz - 1 : z0 - 1;
        double xb = x[col + plane * zb];
        double xc = x[col + plane * z0];
#pragma unroll 4
        for (int k = z0; k < z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = col + plane * k;
            const double xt = x[col + plane * zt];
            f(c, pcode[c], xc, x[c + ow], x[c + oe], x[c + os], x[c + on], xb, xt);
            xb = xc;
            xc = xt;
        }
    }
}

// --------------------------------------------------------------- kernels
//
// Conjugate gradients fused into two stencil passes per iteration i:
//   pass A_i: x_i = x_{i-1} + alpha_{i-1} d_{i-1};  d_i = M^-1 r_i + beta_{i-1} d_{i-1}
//             (formed on the fly for the cell and its six neighbours);
//             q = A d_i (not stored);  partial <d_i, q>;  writes x, d_i
//   pass B_i: q = A d_i again from the cached halo;  r_{i+1} = r_i - alpha_i q;
//             z_{i+1} = M^-1 r_{i+1}; partials <r_{i+1}, r_{i+1}>, <r_{i+1}, z_{i+1}>;
//             writes r, z
// with alpha_i = rz_i / <d_i, A d_i> and beta_{i-1} = rz_i / rz_{i-1}.  The test
// ||r_i|| <= tol ||b|| is made at the start of A_i, which then only applies the last
// x update.  d ping-pongs between two buffers (neighbours read d_{i-1} while d_i is
// written); partial slots ping-pong by iteration parity.
// Algorithmic traffic per cell and iteration: A reads z, d, x, code and writes x, d
// (41 B); B reads d, r, code and writes r, z (33 B).  Storing z = M^-1 r lets pass A
// form each neighbour's new direction from two plain loads.

// slots: <r,r> and <r,z> of r_i live in RR[i & 1], RZ[i & 1]; <d_i, A d_i> in DQ[i & 1]
__device__ inline int slot_rr(int i) { return (i & 1) ? 1 : 0; }
__device__ inline int slot_rz(int i) { return (i & 1) ? 3 : 2; }
__device__ inline int slot_dq(int i) { return (i & 1) ? 5 : 4; }
inline int slot_rr_host(int i) { return (i & 1) ? 1 : 0; }
inline int slot_rz_host(int i) { return (i & 1) ? 3 : 2; }
// flexible CG: <r,r> of the generic update kernel, <z,r> ping-pong, <z, r_prev>, <d,q>
constexpr int FCG_RR = 10, FCG_ZR = 11, FCG_ZRP = 13, FCG_DQ = 14;
constexpr int FCG_R1 = 15;    // <r1,r1> of the smoothed preconditioner's pre-smoothing
constexpr int SLOT_B2 = 6;    // <b,b>
constexpr int SLOT_R2D = 7;   // <r,r> of the double residual before any rounding
constexpr int SLOT_RES0 = 8, SLOT_RES1 = 9;

// dx^2 / (Jacobi count) for every code, 0 for cells without open faces
__device__ inline void fill_inv(double* inv, double dx2) {
    if (threadIdx.x < 16) inv[threadIdx.x] = threadIdx.x ? dx2 / (double)threadIdx.x : 0.0;
    __syncthreads();
}

__device__ inline int jcount(uint8_t pc) { return __builtin_popcount((unsigned)(pc & 0x3F)) + 2 * (pc >> 6); }

// value as stored in T, carried in double
template <class T>
__device__ inline double rnd(double v) { return (double)(T)v; }

// sum of one partial slot over nparts blocks, in block order, by the whole block
__device__ inline double sum_slot(const double* partials, int slot, int nparts, double* sh) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) v[0] += partials[slot * MAX_BLOCKS + b];
    block_reduce<1>(v, sh);
    return v[0];
}

// sums of K partial slots over nparts blocks in one pass (same order as sum_slot)
template <int K>
__device__ inline void sum_slots(const double* partials, const int (&slot)[K], int nparts, double* sh,
                                 double (&out)[K]) {
#pragma unroll
    for (int q = 0; q < K; ++q) out[q] = 0.0;
    for (int b = threadIdx.x; b < nparts; b += NT) {
#pragma unroll
        for (int q = 0; q < K; ++q) out[q] += partials[slot[q] * MAX_BLOCKS + b];
    }
    block_reduce<K>(out, sh);
}

// r_0 = -b + L x_0 (double), stored as T together with z_0 = M^-1 r_0; partials
// <b,b>, <r_0,r_0> (double), and <r_0,r_0>, <r_0,z_0> of the stored T values (in the
// RR/RZ slots of iteration parity par).  For the
// FP64 solve this starts CG on A x = -b; for iterative refinement the stored vector is
// the right-hand side -(b - L x) of the FP32 correction solve A e = -(b - L x).
template <class T>
__global__ void __launch_bounds__(NT) k_pcg_init(Geo g, const uint8_t* __restrict__ pcode,
                                                 const double* __restrict__ b, const double* __restrict__ x,
                                                 T* __restrict__ r, T* __restrict__ zz, double* __restrict__ partials,
                                                 int par) {
    __shared__ double sh[4 * NT];
    __shared__ double inv[16];
    const double idx2 = 1.0 / (g.dx * g.dx);
    fill_inv(inv, g.dx * g.dx);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    march(g, pcode, x, [&](long long c, uint8_t pc, double xc, double xw, double xe, double xs, double xn,
                           double xb, double xt) {
        const double bc = b[c];
        const double rc = -bc + lap_code(pc, xc, xw, xe, xs, xn, xb, xt, idx2);
        const T rt = (T)rc;
        const T zt = (T)(inv[jcount(pc)] * (double)rt);
        r[c] = rt;
        zz[c] = zt;
        v[0] += bc * bc;
        v[1] += rc * rc;
        v[2] += (double)rt * (double)rt;
        v[3] += (double)rt * (double)zt;
    });
    block_reduce<4>(v, sh);
    if (threadIdx.x == 0) {
        partials[SLOT_B2 * MAX_BLOCKS + blockIdx.x] = v[0];
        partials[SLOT_R2D * MAX_BLOCKS + blockIdx.x] = v[1];
        partials[slot_rr(par) * MAX_BLOCKS + blockIdx.x] = v[2];
        partials[slot_rz(par) * MAX_BLOCKS + blockIdx.x] = v[3];
    }
}

// one block: totals of the init partials -> solver state.  ref_slot chooses the norm
// the tolerance is relative to (<b,b> for a plain solve, the double residual for a
// refinement correction).
__global__ void __launch_bounds__(NT) k_pcg_start(const double* partials, int nparts, Solver* sv, double tol,
                                                  int ref_slot) {
    __shared__ double sh[4 * NT];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) {
        v[0] += partials[SLOT_B2 * MAX_BLOCKS + b];
        v[1] += partials[SLOT_R2D * MAX_BLOCKS + b];
        v[2] += partials[0 * MAX_BLOCKS + b];
        v[3] += partials[2 * MAX_BLOCKS + b];
    }
    block_reduce<4>(v, sh);
    if (threadIdx.x == 0) {
        const double ref = ref_slot == SLOT_B2 ? v[0] : v[1];
        sv->bnorm2 = v[0];
        sv->r64norm2 = v[1];
        sv->fnorm2 = ref;
        sv->tol2 = tol * tol * ref;
        sv->rr = v[2];
        sv->rz = v[3];
        sv->iters = 0;
        sv->nan_seen = 0;
        if (!(v[2] == v[2]) || !(ref == ref) || !(v[3] == v[3])) {
            sv->nan_seen = 1;
            sv->converged = 3;
        } else if (ref == 0.0) {
            sv->converged = 2;
        } else {
            sv->converged = v[2] <= sv->tol2 ? 1 : 0;
        }
        sv->stop_it = sv->converged ? -1 : STOP_NONE;
    }
}

__global__ void k_zero_if_trivial(long long n, double* x, const Solver* sv) {
    if (sv->converged != 2) return;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

// Pass A of iteration it (see above); z = M^-1 r_it is stored by the previous pass.
// final_only: apply the last x update only (used when the iteration cap is reached).
template <class T>
__global__ void __launch_bounds__(NT) k_pcg_a(Geo g, const uint8_t* __restrict__ pcode, const T* __restrict__ zz,
                                              const T* __restrict__ dold, T* __restrict__ dnew, T* __restrict__ x,
                                              double* __restrict__ partials, int nparts, int it, int final_only,
                                              int skip_x, int fresh, Solver* sv) {
    if (stopped_before(sv, it)) return;
    __shared__ double sh[NT];
    const double idx2 = 1.0 / (g.dx * g.dx);
    double alpha = 0.0, beta = 0.0;
    bool stop = final_only != 0;
    if (it > 0) {
        const int sl[4] = {slot_rr(it), slot_rz(it), slot_rz(it - 1), slot_dq(it - 1)};
        double tot[4];
        sum_slots<4>(partials, sl, nparts, sh, tot);
        const double rr = tot[0], rz = tot[1], rzp = tot[2], dq = tot[3];
        alpha = skip_x ? 0.0 : rzp / dq;
        beta = rz / rzp;
        if (!(rr == rr)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sv->nan_seen = 1;
                sv->converged = 3;
                sv->iters = it;
                sv->stop_it = it;
            }
            return;
        }
        if (rr <= sv->tol2) stop = true;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sv->rr = rr;
            sv->iters = it;
            if (stop && !final_only) {
                sv->converged = 1;
                sv->stop_it = it;
            }
        }
    }
    const long long N = (long long)g.nx * g.ny * g.nz;
    if (stop) {
        // last x update only: x_it = x_{it-1} + alpha_{it-1} d_{it-1}
        for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
             c += (long long)gridDim.x * blockDim.x)
            x[c] = (T)((double)x[c] + alpha * (double)dold[c]);
        return;
    }
    const bool first = it == 0 || fresh;
    double v[1] = {0.0};
    const int nzc = slab_count(g.nz);
    const long long tiles = (long long)g.ntx * g.nty;
    const long long items = tiles * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    for (long long w = w0; w < w1; ++w) {
        const int zc = (int)(w / tiles);
        const long long t = w % tiles;
        const int i = (int)(t % g.ntx) * TX + (threadIdx.x % TX);
        const int j = (int)(t / g.ntx) * TY + (threadIdx.x / TX);
        const int z0 = (int)((long long)g.nz * zc / nzc), z1 = (int)((long long)g.nz * (zc + 1) / nzc);
        if (i >= g.nx || j >= g.ny) continue;
        const int iw = i == 0 ? g.nx - 1 : i - 1, ie = i == g.nx - 1 ? 0 : i + 1;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j == g.ny - 1 ? 0 : j + 1;
        const long long col = (long long)i + (long long)g.nx * j;
        const long long ow = (long long)iw + (long long)g.nx * j - col;
        const long long oe = (long long)ie + (long long)g.nx * j - col;
        const long long os = (long long)i + (long long)g.nx * js - col;
        const long long on = (long long)i + (long long)g.nx * jn - col;
        const int zb = z0 == 0 ? g.nz - 1 : z0 - 1;
        if (first) {
            // d_0 = z_0
            double db = zz[col + plane * zb];
            double dc = zz[col + plane * z0];
#pragma unroll 4
            for (int k = z0; k < z1; ++k) {
                const int zt = k == g.nz - 1 ? 0 : k + 1;
                const long long c = col + plane * k;
                const double dt = zz[col + plane * zt];
                const double q = -lap_code(pcode[c], dc, zz[c + ow], zz[c + oe], zz[c + os], zz[c + on], db, dt, idx2);
                dnew[c] = (T)dc;
                v[0] += dc * q;
                db = dc;
                dc = dt;
            }
            continue;
        }
        const long long cb0 = col + plane * zb, cc0 = col + plane * z0;
        double db = rnd<T>(zz[cb0] + beta * dold[cb0]);
        double oc = dold[cc0];
        double dc = rnd<T>(zz[cc0] + beta * oc);
#pragma unroll 2
        for (int k = z0; k < z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = col + plane * k;
            const long long ct = col + plane * zt;
            const double ot = dold[ct];
            const double dt = rnd<T>(zz[ct] + beta * ot);
            const double dw = rnd<T>(zz[c + ow] + beta * dold[c + ow]);
            const double de = rnd<T>(zz[c + oe] + beta * dold[c + oe]);
            const double ds = rnd<T>(zz[c + os] + beta * dold[c + os]);
            const double dn = rnd<T>(zz[c + on] + beta * dold[c + on]);
            const double q = -lap_code(pcode[c], dc, dw, de, ds, dn, db, dt, idx2);
            x[c] = (T)((double)x[c] + alpha * oc);
            dnew[c] = (T)dc;
            v[0] += dc * q;
            db = dc;
            dc = dt;
            oc = ot;
        }
    }
    block_reduce<1>(v, sh);
    if (threadIdx.x == 0) partials[slot_dq(it) * MAX_BLOCKS + blockIdx.x] = v[0];
}

// Pass B of iteration it: r_{it+1} = r_it - alpha_it A d_it; partials for r_{it+1}
template <class T>
__global__ void __launch_bounds__(NT) k_pcg_b(Geo g, const uint8_t* __restrict__ pcode, const T* __restrict__ d,
                                              T* __restrict__ r, T* __restrict__ zz, double* __restrict__ partials,
                                              int nparts, int it, const Solver* sv) {
    if (stopped_before(sv, it + 1)) return;
    __shared__ double sh[2 * NT];
    __shared__ double inv[16];
    const double idx2 = 1.0 / (g.dx * g.dx);
    fill_inv(inv, g.dx * g.dx);
    const int sl[2] = {slot_rz(it), slot_dq(it)};
    double tot[2];
    sum_slots<2>(partials, sl, nparts, sh, tot);
    const double rz = tot[0], dq = tot[1];
    const double alpha = rz / dq;
    double v[2] = {0.0, 0.0};
    march(g, pcode, d, [&](long long c, uint8_t pc, double xc, double xw, double xe, double xs, double xn,
                           double xb, double xt) {
        const double q = -lap_code(pc, xc, xw, xe, xs, xn, xb, xt, idx2);
        const T rn = (T)((double)r[c] - alpha * q);
        const T z = (T)(inv[jcount(pc)] * (double)rn);
        r[c] = rn;
        zz[c] = z;
        v[0] += (double)rn * (double)rn;
        v[1] += (double)rn * (double)z;
    });
    block_reduce<2>(v, sh);
    if (threadIdx.x == 0) {
        partials[slot_rr(it + 1) * MAX_BLOCKS + blockIdx.x] = v[0];
        partials[slot_rz(it + 1) * MAX_BLOCKS + blockIdx.x] = v[1];
    }
}


// ----------------------------------------------------- vector (double2) passes
//
// On grids with an even number of cells in x every thread owns an aligned pair of
// cells; a block owns a 128x4 column tile.  Pass A shares the new direction of the
// current plane through a double-buffered LDS tile with a one-cell halo (one
// barrier per plane).  Every result is written with non-temporal stores (measured
// faster than regular stores for all four vectors on the full-size solve).

constexpr int VTX = 128;               // cells of a tile row (64 lanes x 2)
constexpr int VW = VTX + 2;            // LDS row with halo

__host__ __device__ inline int vslab_count(int nz) {
    int want = (nz + 15) / 16;               // about 16 planes per slab
    want = ((want + 7) / 8) * 8;             // multiple of the XCD count
    if (want > nz) want = nz;
    return want < 1 ? 1 : want;
}

struct VItem {
    int i, j, z0, z1;     // first cell of this thread's pair, row, slab
    int i0, j0;           // tile origin
    bool valid;
};

__device__ inline VItem vitem(const Geo& g, long long w, int ntx2, int nzc) {
    const long long tiles = (long long)ntx2 * g.nty;
    VItem v;
    const int zc = (int)(w / tiles);
    const long long t = w % tiles;
    v.i0 = (int)(t % ntx2) * VTX;
    v.j0 = (int)(t / ntx2) * TY;
    v.i = v.i0 + 2 * (threadIdx.x % 64);
    v.j = v.j0 + (int)(threadIdx.x / 64);
    v.z0 = (int)((long long)g.nz * zc / nzc);
    v.z1 = (int)((long long)g.nz * (zc + 1) / nzc);
    v.valid = v.i < g.nx && v.j < g.ny;
    return v;
}

__device__ inline double2 ld2(const double* __restrict__ p, long long c) {
    return *reinterpret_cast<const double2*>(p + c);
}

__device__ inline double2 ld2(const float* __restrict__ p, long long c) {
    const float2 f = *reinterpret_cast<const float2*>(p + c);
    return make_double2((double)f.x, (double)f.y);
}

template <class T>
__device__ inline void st2nt(T* __restrict__ p, long long c, double a, double b) {
    __builtin_nontemporal_store((T)a, p + c);
    __builtin_nontemporal_store((T)b, p + c + 1);
}

// Pass A, vector form (see the scalar k_pcg_a for the mathematics).
template <class T, bool FIRST>
__global__ void __launch_bounds__(NT) k_pcg_a_v(Geo g, const uint8_t* __restrict__ pcode,
                                                const T* __restrict__ zz, const T* __restrict__ dold,
                                                T* __restrict__ dnew, T* __restrict__ x,
                                                double* __restrict__ partials, int nparts, int it, int skip_x,
                                                Solver* sv) {
    if (stopped_before(sv, it)) return;
    __shared__ double sh[NT];
    __shared__ double pln[2][(TY + 2) * VW];
    const double idx2 = 1.0 / (g.dx * g.dx);
    double alpha = 0.0, beta = 0.0;
    const long long N = (long long)g.nx * g.ny * g.nz;
    if (!FIRST) {
        const int sl[4] = {slot_rr(it), slot_rz(it), slot_rz(it - 1), slot_dq(it - 1)};
        double tot[4];
        sum_slots<4>(partials, sl, nparts, sh, tot);
        const double rr = tot[0], rz = tot[1], rzp = tot[2], dq = tot[3];
        alpha = skip_x ? 0.0 : rzp / dq;
        beta = rz / rzp;
        if (!(rr == rr)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sv->nan_seen = 1;
                sv->converged = 3;
                sv->iters = it;
                sv->stop_it = it;
            }
            return;
        }
        const bool stop = rr <= sv->tol2;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sv->rr = rr;
            sv->iters = it;
            if (stop) {
                sv->converged = 1;
                sv->stop_it = it;
            }
        }
        if (stop) {
            for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
                 c += (long long)gridDim.x * blockDim.x)
                x[c] = (T)((double)x[c] + alpha * (double)dold[c]);
            return;
        }
    }
    auto dn1 = [&](long long c) -> double {
        return FIRST ? (double)zz[c] : rnd<T>((double)zz[c] + beta * (double)dold[c]);
    };
    auto dn2 = [&](long long c) -> double2 {
        double2 a = ld2(zz, c);
        if (FIRST) return a;
        double2 o = ld2(dold, c);
        return make_double2(rnd<T>(a.x + beta * o.x), rnd<T>(a.y + beta * o.y));
    };
    const int ntx2 = (g.nx + VTX - 1) / VTX;
    const int nzc = vslab_count(g.nz);
    const long long items = (long long)ntx2 * g.nty * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    const int lane = threadIdx.x % 64, lj = threadIdx.x / 64;
    const int li = 2 * lane;
    double v = 0.0;
    int buf = 0;
    for (long long w = w0; w < w1; ++w) {
        const VItem it_ = vitem(g, w, ntx2, nzc);
        const int i = it_.i, j = it_.j;
        // last valid pair and row of the tile own the east / north halo
        const int lane_max = min(63, (g.nx - it_.i0) / 2 - 1);
        const int row_max = min(TY - 1, g.ny - it_.j0 - 1);
        const int iw = it_.i0 == 0 ? g.nx - 1 : it_.i0 - 1;
        const int ie = i + 2 >= g.nx ? 0 : i + 2;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j >= g.ny - 1 ? 0 : j + 1;
        const long long col = it_.valid ? (long long)i + (long long)g.nx * j : 0;
        const int zb = it_.z0 == 0 ? g.nz - 1 : it_.z0 - 1;
        double2 db = make_double2(0.0, 0.0), dc = db, oc = db;
        if (it_.valid) {
            db = dn2(col + plane * zb);
            const double2 zc2 = ld2(zz, col + plane * it_.z0);
            if (!FIRST) oc = ld2(dold, col + plane * it_.z0);
            dc = FIRST ? zc2 : make_double2(rnd<T>(zc2.x + beta * oc.x), rnd<T>(zc2.y + beta * oc.y));
        }
        for (int k = it_.z0; k < it_.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            double* P = pln[buf];
            double2 dt = make_double2(0.0, 0.0), ot = dt;
            if (it_.valid) {
                const long long ct = col + plane * zt;
                const double2 zt2 = ld2(zz, ct);
                if (!FIRST) ot = ld2(dold, ct);
                dt = FIRST ? zt2 : make_double2(rnd<T>(zt2.x + beta * ot.x), rnd<T>(zt2.y + beta * ot.y));
                P[(lj + 1) * VW + li + 1] = dc.x;
                P[(lj + 1) * VW + li + 2] = dc.y;
                const long long pk = plane * k;
                if (lane == 0) P[(lj + 1) * VW] = dn1((long long)iw + (long long)g.nx * j + pk);
                if (lane == lane_max) P[(lj + 1) * VW + li + 3] = dn1((long long)ie + (long long)g.nx * j + pk);
                if (lj == 0) {
                    const double2 s2 = dn2((long long)i + (long long)g.nx * js + pk);
                    P[li + 1] = s2.x;
                    P[li + 2] = s2.y;
                }
                if (lj == row_max) {
                    const double2 n2 = dn2((long long)i + (long long)g.nx * jn + pk);
                    P[(lj + 2) * VW + li + 1] = n2.x;
                    P[(lj + 2) * VW + li + 2] = n2.y;
                }
            }
            __syncthreads();
            if (it_.valid) {
                const long long c = col + plane * k;
                const double w_ = P[(lj + 1) * VW + li], e_ = P[(lj + 1) * VW + li + 3];
                const double s0 = P[lj * VW + li + 1], s1 = P[lj * VW + li + 2];
                const double n0 = P[(lj + 2) * VW + li + 1], n1 = P[(lj + 2) * VW + li + 2];
                const uint8_t pc0 = pcode[c], pc1 = pcode[c + 1];
                const double q0 = -lap_code(pc0, dc.x, w_, dc.y, s0, n0, db.x, dt.x, idx2);
                const double q1 = -lap_code(pc1, dc.y, dc.x, e_, s1, n1, db.y, dt.y, idx2);
                if (!FIRST) {
                    const double2 xx = ld2(x, c);
                    st2nt(x, c, xx.x + alpha * oc.x, xx.y + alpha * oc.y);
                }
                st2nt(dnew, c, dc.x, dc.y);
                v += dc.x * q0 + dc.y * q1;
            }
            db = dc;
            dc = dt;
            oc = ot;
            buf ^= 1;
        }
    }
    double vv[1] = {v};
    block_reduce<1>(vv, sh);
    if (threadIdx.x == 0) partials[slot_dq(it) * MAX_BLOCKS + blockIdx.x] = vv[0];
}

// Pass B, vector form: r_{it+1} = r_it - alpha A d_it, z = M^-1 r; partials.
template <class T>
__global__ void __launch_bounds__(NT) k_pcg_b_v(Geo g, const uint8_t* __restrict__ pcode, const T* __restrict__ d,
                                                T* __restrict__ r, T* __restrict__ zz,
                                                double* __restrict__ partials, int nparts, int it, const Solver* sv) {
    if (stopped_before(sv, it + 1)) return;
    __shared__ double sh[2 * NT];
    __shared__ double inv[16];
    const double idx2 = 1.0 / (g.dx * g.dx);
    fill_inv(inv, g.dx * g.dx);
    const int sl[2] = {slot_rz(it), slot_dq(it)};
    double tot[2];
    sum_slots<2>(partials, sl, nparts, sh, tot);
    const double rz = tot[0], dq = tot[1];
    const double alpha = rz / dq;
    const int ntx2 = (g.nx + VTX - 1) / VTX;
    const int nzc = vslab_count(g.nz);
    const long long items = (long long)ntx2 * g.nty * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    double v[2] = {0.0, 0.0};
    for (long long w = w0; w < w1; ++w) {
        const VItem it_ = vitem(g, w, ntx2, nzc);
        if (!it_.valid) continue;
        const int i = it_.i, j = it_.j;
        const int iw = i == 0 ? g.nx - 1 : i - 1, ie = i + 2 >= g.nx ? 0 : i + 2;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j == g.ny - 1 ? 0 : j + 1;
        const long long col = (long long)i + (long long)g.nx * j;
        const long long ow = (long long)iw + (long long)g.nx * j - col;
        const long long oe = (long long)ie + (long long)g.nx * j - col;
        const long long os = (long long)i + (long long)g.nx * js - col;
        const long long on = (long long)i + (long long)g.nx * jn - col;
        const int zb = it_.z0 == 0 ? g.nz - 1 : it_.z0 - 1;
        double2 xb = ld2(d, col + plane * zb);
        double2 xc = ld2(d, col + plane * it_.z0);
        for (int k = it_.z0; k < it_.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = col + plane * k;
            const double2 xt = ld2(d, col + plane * zt);
            const double2 xs = ld2(d, c + os), xn = ld2(d, c + on);
            const double xw = d[c + ow], xe = d[c + oe];
            const uint8_t pc0 = pcode[c], pc1 = pcode[c + 1];
            const double q0 = -lap_code(pc0, xc.x, xw, xc.y, xs.x, xn.x, xb.x, xt.x, idx2);
            const double q1 = -lap_code(pc1, xc.y, xc.x, xe, xs.y, xn.y, xb.y, xt.y, idx2);
            const double2 rr = ld2(r, c);
            const double rn0 = (double)(T)(rr.x - alpha * q0), rn1 = (double)(T)(rr.y - alpha * q1);
            const double z0 = (double)(T)(inv[jcount(pc0)] * rn0), z1 = (double)(T)(inv[jcount(pc1)] * rn1);
            st2nt(r, c, rn0, rn1);
            st2nt(zz, c, z0, z1);
            v[0] += rn0 * rn0 + rn1 * rn1;
            v[1] += rn0 * z0 + rn1 * z1;
            xb = xc;
            xc = xt;
        }
    }
    block_reduce<2>(v, sh);
    if (threadIdx.x == 0) {
        partials[slot_rr(it + 1) * MAX_BLOCKS + blockIdx.x] = v[0];
        partials[slot_rz(it + 1) * MAX_BLOCKS + blockIdx.x] = v[1];
    }
}

// ------------------------------------------------------------- FP32 sweeps
//
// The correction solve of the mixed path stores and computes in FP32.  Four cells per
// lane (16-byte loads and stores): a block owns a 256x4 column tile and marches a slab
// of about 16 planes; pass A shares the new direction of the plane through a
// double-buffered LDS tile of floats.  Dot products are accumulated in double.
// Requires nx % 4 == 0 and 16-byte aligned vectors.

constexpr int FTX = 256;               // cells of a tile row (64 lanes x 4)
constexpr int FW = FTX + 8;            // LDS row: west halo at 3, cells from 4, east halo at FTX + 4

__host__ __device__ inline int fslab_count(int nz) {
    int want = (nz + 15) / 16;               // about 16 planes per slab
    want = ((want + 7) / 8) * 8;             // multiple of the XCD count
    if (want > nz) want = nz;
    return want < 1 ? 1 : want;
}

__device__ inline VItem fitem(const Geo& g, long long w, int ntx4, int nzc) {
    const long long tiles = (long long)ntx4 * g.nty;
    VItem v;
    const int zc = (int)(w / tiles);
    const long long t = w % tiles;
    v.i0 = (int)(t % ntx4) * FTX;
    v.j0 = (int)(t / ntx4) * TY;
    v.i = v.i0 + 4 * (threadIdx.x % 64);
    v.j = v.j0 + (int)(threadIdx.x / 64);
    v.z0 = (int)((long long)g.nz * zc / nzc);
    v.z1 = (int)((long long)g.nz * (zc + 1) / nzc);
    v.valid = v.i < g.nx && v.j < g.ny;
    return v;
}

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline f4 ld4(const float* __restrict__ p, long long c) { return *reinterpret_cast<const f4*>(p + c); }
__device__ inline void st4nt(float* __restrict__ p, long long c, f4 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<f4*>(p + c));
}
// a * x + y per component, one rounding each
__device__ inline f4 fma4(float a, f4 x, f4 y) {
    f4 r;
    r.x = fmaf(a, x.x, y.x);
    r.y = fmaf(a, x.y, y.y);
    r.z = fmaf(a, x.z, y.z);
    r.w = fmaf(a, x.w, y.w);
    return r;
}
__device__ inline float dot4(f4 a, f4 b) { return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w; }

// (A x)_c = -(L x)_c in float from the code byte
__device__ inline float aq(unsigned pc, float xc, float xw, float xe, float xs, float xn, float xb, float xt,
                           float idx2) {
    float acc = (float)(__builtin_popcount(pc & 0x3Fu) + 2 * (pc >> 6)) * xc;
    acc -= (pc & 1) ? xw : 0.0f;
    acc -= (pc & 2) ? xe : 0.0f;
    acc -= (pc & 4) ? xs : 0.0f;
    acc -= (pc & 8) ? xn : 0.0f;
    acc -= (pc & 16) ? xb : 0.0f;
    acc -= (pc & 32) ? xt : 0.0f;
    return acc * idx2;
}

__device__ inline f4 aq4(unsigned pc4, f4 c, float w, float e, f4 s, f4 n, f4 b, f4 t, float idx2) {
    f4 q;
    q.x = aq(pc4 & 0xFFu, c.x, w, c.y, s.x, n.x, b.x, t.x, idx2);
    q.y = aq((pc4 >> 8) & 0xFFu, c.y, c.x, c.z, s.y, n.y, b.y, t.y, idx2);
    q.z = aq((pc4 >> 16) & 0xFFu, c.z, c.y, c.w, s.z, n.z, b.z, t.z, idx2);
    q.w = aq(pc4 >> 24, c.w, c.z, e, s.w, n.w, b.w, t.w, idx2);
    return q;
}

// Pass A in FP32 (see k_pcg_a for the mathematics).  skip_x: the x update of this pass
// was already folded into the FP64 solution by a residual replacement.  FLEX: flexible
// CG, beta = (<z,r> - <z,r_prev>) / <z_prev,r_prev> with <z,r_prev> in slot FCG_ZRP.
template <bool FIRST, bool FLEX = false>
__global__ void __launch_bounds__(NT) k_pcg_a_f4(Geo g, const uint8_t* __restrict__ pcode,
                                                 const float* __restrict__ zz, const float* __restrict__ dold,
                                                 float* __restrict__ dnew, float* __restrict__ x,
                                                 double* __restrict__ partials, int nparts, int it, int skip_x,
                                                 Solver* sv) {
    if (stopped_before(sv, it)) return;
    __shared__ double sh[NT];
    __shared__ __attribute__((aligned(16))) float pln[2][(TY + 2) * FW];
    const float idx2 = (float)(1.0 / (g.dx * g.dx));
    double alpha = 0.0, beta = 0.0;
    const long long N = (long long)g.nx * g.ny * g.nz;
    if (!FIRST) {
        double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (FLEX) {
            const int sl[5] = {slot_rr(it), slot_rz(it), slot_rz(it - 1), slot_dq(it - 1), FCG_ZRP};
            sum_slots<5>(partials, sl, nparts, sh, tot);
        } else {
            const int sl[4] = {slot_rr(it), slot_rz(it), slot_rz(it - 1), slot_dq(it - 1)};
            double t4[4];
            sum_slots<4>(partials, sl, nparts, sh, t4);
            for (int q = 0; q < 4; ++q) tot[q] = t4[q];
        }
        const double rr = tot[0], rz = tot[1], rzp = tot[2], dq = tot[3];
        alpha = skip_x ? 0.0 : rzp / dq;
        beta = FLEX ? (rz - tot[4]) / rzp : rz / rzp;
        if (!(rr == rr)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sv->nan_seen = 1;
                sv->converged = 3;
                sv->iters = it;
                sv->stop_it = it;
            }
            return;
        }
        const bool stop = rr <= sv->tol2;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sv->rr = rr;
            sv->iters = it;
            if (stop) {
                sv->converged = 1;
                sv->stop_it = it;
            }
        }
        if (stop) {
            if (!skip_x) {
                const float af = (float)alpha;
                for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
                     c += (long long)gridDim.x * blockDim.x)
                    x[c] = fmaf(af, dold[c], x[c]);
            }
            return;
        }
    }
    const float af = (float)alpha, bf = (float)beta;
    const bool upd_x = !FIRST && !skip_x;
    auto dn1 = [&](long long c) -> float { return FIRST ? zz[c] : fmaf(bf, dold[c], zz[c]); };
    auto dn4 = [&](long long c) -> f4 { return FIRST ? ld4(zz, c) : fma4(bf, ld4(dold, c), ld4(zz, c)); };
    const int ntx4 = (g.nx + FTX - 1) / FTX;
    const int nzc = fslab_count(g.nz);
    const long long items = (long long)ntx4 * g.nty * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    const int lane = threadIdx.x % 64, lj = threadIdx.x / 64;
    const int li = 4 * lane;
    double v = 0.0;
    int buf = 0;
    const f4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
    for (long long w = w0; w < w1; ++w) {
        const VItem it_ = fitem(g, w, ntx4, nzc);
        const int i = it_.i, j = it_.j;
        // last valid lane and row of the tile own the east / north halo
        const int lane_max = min(63, (g.nx - it_.i0) / 4 - 1);
        const int row_max = min(TY - 1, g.ny - it_.j0 - 1);
        const int iw = it_.i0 == 0 ? g.nx - 1 : it_.i0 - 1;
        const int ie = i + 4 >= g.nx ? 0 : i + 4;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j >= g.ny - 1 ? 0 : j + 1;
        const long long col = it_.valid ? (long long)i + (long long)g.nx * j : 0;
        const int zb = it_.z0 == 0 ? g.nz - 1 : it_.z0 - 1;
        f4 db = zero4, dc = zero4, oc = zero4;
        if (it_.valid) {
            db = dn4(col + plane * zb);
            const f4 zc4 = ld4(zz, col + plane * it_.z0);
            if (!FIRST) oc = ld4(dold, col + plane * it_.z0);
            dc = FIRST ? zc4 : fma4(bf, oc, zc4);
        }
        for (int k = it_.z0; k < it_.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            float* P = pln[buf];
            f4 dt = zero4, ot = zero4;
            if (it_.valid) {
                const long long ct = col + plane * zt;
                const f4 zt4 = ld4(zz, ct);
                if (!FIRST) ot = ld4(dold, ct);
                dt = FIRST ? zt4 : fma4(bf, ot, zt4);
                *reinterpret_cast<f4*>(&P[(lj + 1) * FW + 4 + li]) = dc;
                const long long pk = plane * k;
                if (lane == 0) P[(lj + 1) * FW + 3] = dn1((long long)iw + (long long)g.nx * j + pk);
                if (lane == lane_max) P[(lj + 1) * FW + 8 + li] = dn1((long long)ie + (long long)g.nx * j + pk);
                if (lj == 0) *reinterpret_cast<f4*>(&P[4 + li]) = dn4((long long)i + (long long)g.nx * js + pk);
                if (lj == row_max)
                    *reinterpret_cast<f4*>(&P[(lj + 2) * FW + 4 + li]) =
                        dn4((long long)i + (long long)g.nx * jn + pk);
            }
            __syncthreads();
            if (it_.valid) {
                const long long c = col + plane * k;
                const float w_ = P[(lj + 1) * FW + 3 + li], e_ = P[(lj + 1) * FW + 8 + li];
                const f4 s4 = *reinterpret_cast<const f4*>(&P[lj * FW + 4 + li]);
                const f4 n4 = *reinterpret_cast<const f4*>(&P[(lj + 2) * FW + 4 + li]);
                const unsigned pc4 = *reinterpret_cast<const unsigned*>(pcode + c);
                const f4 q = aq4(pc4, dc, w_, e_, s4, n4, db, dt, idx2);
                if (upd_x) st4nt(x, c, fma4(af, oc, ld4(x, c)));
                st4nt(dnew, c, dc);
                v += (double)dot4(dc, q);
            }
            db = dc;
            dc = dt;
            oc = ot;
            buf ^= 1;
        }
    }
    double vv[1] = {v};
    block_reduce<1>(vv, sh);
    if (threadIdx.x == 0) partials[slot_dq(it) * MAX_BLOCKS + blockIdx.x] = vv[0];
}

// Pass B in FP32: r_{it+1} = r_it - alpha A d_it into rout (may be r), and with JZ the
// Jacobi z = M^-1 r; partials <r,r> (and <r,z>).  Without JZ the preconditioner is
// applied by a separate step (the learned one) and <r,z> comes from there.
template <bool JZ = true>
__global__ void __launch_bounds__(NT) k_pcg_b_f4(Geo g, const uint8_t* __restrict__ pcode,
                                                 const float* __restrict__ d, const float* r, float* rout,
                                                 float* __restrict__ zz, double* __restrict__ partials, int nparts,
                                                 int it, const Solver* sv) {
    if (stopped_before(sv, it + 1)) return;
    __shared__ double sh[2 * NT];
    __shared__ float invf[16];
    const double dx2 = g.dx * g.dx;
    const float idx2 = (float)(1.0 / dx2);
    if (threadIdx.x < 16) invf[threadIdx.x] = threadIdx.x ? (float)(dx2 / (double)threadIdx.x) : 0.0f;
    __syncthreads();
    const int sl[2] = {slot_rz(it), slot_dq(it)};
    double tot[2];
    sum_slots<2>(partials, sl, nparts, sh, tot);
    const double rz = tot[0], dq = tot[1];
    const float af = (float)(rz / dq);
    const int ntx4 = (g.nx + FTX - 1) / FTX;
    const int nzc = fslab_count(g.nz);
    const long long items = (long long)ntx4 * g.nty * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    double v[2] = {0.0, 0.0};
    for (long long w = w0; w < w1; ++w) {
        const VItem it_ = fitem(g, w, ntx4, nzc);
        if (!it_.valid) continue;
        const int i = it_.i, j = it_.j;
        const int iw = i == 0 ? g.nx - 1 : i - 1, ie = i + 4 >= g.nx ? 0 : i + 4;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j == g.ny - 1 ? 0 : j + 1;
        const long long col = (long long)i + (long long)g.nx * j;
        const long long ow = (long long)iw + (long long)g.nx * j - col;
        const long long oe = (long long)ie + (long long)g.nx * j - col;
        const long long os = (long long)i + (long long)g.nx * js - col;
        const long long on = (long long)i + (long long)g.nx * jn - col;
        const int zb = it_.z0 == 0 ? g.nz - 1 : it_.z0 - 1;
        f4 xb = ld4(d, col + plane * zb);
        f4 xc = ld4(d, col + plane * it_.z0);
        for (int k = it_.z0; k < it_.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = col + plane * k;
            const f4 xt = ld4(d, col + plane * zt);
            const f4 xs = ld4(d, c + os), xn = ld4(d, c + on);
            const float xw = d[c + ow], xe = d[c + oe];
            const unsigned pc4 = *reinterpret_cast<const unsigned*>(pcode + c);
            const f4 q = aq4(pc4, xc, xw, xe, xs, xn, xb, xt, idx2);
            const f4 rn = fma4(-af, q, ld4(r, c));
            st4nt(rout, c, rn);
            v[0] += (double)dot4(rn, rn);
            if (JZ) {
                f4 z;
                z.x = invf[jcount((uint8_t)(pc4 & 0xFFu))] * rn.x;
                z.y = invf[jcount((uint8_t)((pc4 >> 8) & 0xFFu))] * rn.y;
                z.z = invf[jcount((uint8_t)((pc4 >> 16) & 0xFFu))] * rn.z;
                z.w = invf[jcount((uint8_t)(pc4 >> 24))] * rn.w;
                st4nt(zz, c, z);
                v[1] += (double)dot4(rn, z);
            }
            xb = xc;
            xc = xt;
        }
    }
    block_reduce<2>(v, sh);
    if (threadIdx.x == 0) {
        partials[slot_rr(it + 1) * MAX_BLOCKS + blockIdx.x] = v[0];
        if (JZ) partials[slot_rz(it + 1) * MAX_BLOCKS + blockIdx.x] = v[1];
    }
}

// ------------------------------------------- smoothing steps of the learned preconditioner
//
// The two-level form of the learned preconditioner puts one damped Jacobi step
// S = omega D^-1 before and after the network map M:
//     z1 = S r,  r1 = r - A z1,  z2 = z1 + M(r1),  z = z2 + S (r - A z2).
// Both smoothing steps are FP32 stencil passes over the (256 x 4 tile, z-slab) items of
// the CG passes, four cells per lane.  The pre-smoothing pass applies A to S r, formed
// once per cell from r and the cell's code and shared through an LDS tile (as pass A
// shares its direction); the post-smoothing pass applies A to the stored z2 with the x
// and y neighbours from plain loads served by the L2 (as pass B).

// omega dx^2 / (Jacobi count) per code count, 0 for cells without open faces
__device__ inline void fill_sinv(float* sinv, double omega, double dx2) {
    if (threadIdx.x < 16) sinv[threadIdx.x] = threadIdx.x ? (float)(omega * dx2 / (double)threadIdx.x) : 0.0f;
    __syncthreads();
}

// S x for four cells with the codes packed in pc4
__device__ inline f4 smul4(const float* sinv, unsigned pc4, f4 x) {
    f4 w;
    w.x = sinv[jcount((uint8_t)(pc4 & 0xFFu))] * x.x;
    w.y = sinv[jcount((uint8_t)((pc4 >> 8) & 0xFFu))] * x.y;
    w.z = sinv[jcount((uint8_t)((pc4 >> 16) & 0xFFu))] * x.z;
    w.w = sinv[jcount((uint8_t)(pc4 >> 24))] * x.w;
    return w;
}

__device__ inline unsigned ldc4(const uint8_t* __restrict__ pcode, long long c) {
    return *reinterpret_cast<const unsigned*>(pcode + c);
}

// Pre-smoothing: r1 = r - A (S r), partials <r1,r1> into slot r1_slot.  With check the
// pass first makes the solve's stop test on the <r,r> partials of slot rr_slot (as the
// network's input step does without smoothing): the solve stops at iteration it once
// <r,r> <= tol2, and then no block writes anything.  S r of the plane is shared through a
// double-buffered LDS tile, as pass A shares its direction: each lane forms it for its
// own four cells, the edge lanes and rows for the tile's halo.
__global__ void __launch_bounds__(NT) k_smooth_pre_f4(Geo g, const uint8_t* __restrict__ pcode,
                                                      const float* __restrict__ r, float* __restrict__ r1,
                                                      double omega, double* __restrict__ partials, int nparts,
                                                      int r1_slot, int rr_slot, Solver* sv, int it, int check) {
    if (sv && stopped_before(sv, it)) return;
    __shared__ double sh[NT];
    __shared__ float sinv[16];
    __shared__ __attribute__((aligned(16))) float pln[2][(TY + 2) * FW];
    if (sv && check) {
        const double rr = sum_slot(partials, rr_slot, nparts, sh);
        if (!(rr == rr)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sv->nan_seen = 1;
                sv->converged = 3;
                sv->iters = it;
                sv->stop_it = it;
            }
            return;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sv->rr = rr;
            sv->iters = it;
        }
        if (rr <= sv->tol2) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sv->converged = 1;
                sv->stop_it = it;
            }
            return;
        }
    }
    const double dx2 = g.dx * g.dx;
    const float idx2 = (float)(1.0 / dx2);
    fill_sinv(sinv, omega, dx2);
    auto sr4 = [&](long long c) -> f4 { return smul4(sinv, ldc4(pcode, c), ld4(r, c)); };
    auto sr1 = [&](long long c) -> float { return sinv[jcount(pcode[c])] * r[c]; };
    const int ntx4 = (g.nx + FTX - 1) / FTX;
    const int nzc = fslab_count(g.nz);
    const long long items = (long long)ntx4 * g.nty * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    const int lane = threadIdx.x % 64, lj = threadIdx.x / 64;
    const int li = 4 * lane;
    const f4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
    double v[1] = {0.0};
    int buf = 0;
    for (long long w = w0; w < w1; ++w) {
        const VItem it_ = fitem(g, w, ntx4, nzc);
        const int i = it_.i, j = it_.j;
        // last valid lane and row of the tile own the east / north halo
        const int lane_max = min(63, (g.nx - it_.i0) / 4 - 1);
        const int row_max = min(TY - 1, g.ny - it_.j0 - 1);
        const int iw = it_.i0 == 0 ? g.nx - 1 : it_.i0 - 1;
        const int ie = i + 4 >= g.nx ? 0 : i + 4;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j >= g.ny - 1 ? 0 : j + 1;
        const long long col = it_.valid ? (long long)i + (long long)g.nx * j : 0;
        const int zb = it_.z0 == 0 ? g.nz - 1 : it_.z0 - 1;
        f4 wb = zero4, wc = zero4, rc = zero4;
        unsigned pcc = 0u;
        if (it_.valid) {
            wb = sr4(col + plane * zb);
            const long long c0 = col + plane * it_.z0;
            rc = ld4(r, c0);
            pcc = ldc4(pcode, c0);
            wc = smul4(sinv, pcc, rc);
        }
        for (int k = it_.z0; k < it_.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            float* P = pln[buf];
            f4 rt = zero4, wt = zero4;
            unsigned pct = 0u;
            if (it_.valid) {
                const long long ct = col + plane * zt;
                rt = ld4(r, ct);
                pct = ldc4(pcode, ct);
                wt = smul4(sinv, pct, rt);
                *reinterpret_cast<f4*>(&P[(lj + 1) * FW + 4 + li]) = wc;
                const long long pk = plane * k;
                if (lane == 0) P[(lj + 1) * FW + 3] = sr1((long long)iw + (long long)g.nx * j + pk);
                if (lane == lane_max) P[(lj + 1) * FW + 8 + li] = sr1((long long)ie + (long long)g.nx * j + pk);
                if (lj == 0) *reinterpret_cast<f4*>(&P[4 + li]) = sr4((long long)i + (long long)g.nx * js + pk);
                if (lj == row_max)
                    *reinterpret_cast<f4*>(&P[(lj + 2) * FW + 4 + li]) = sr4((long long)i + (long long)g.nx * jn + pk);
            }
            __syncthreads();
            if (it_.valid) {
                const long long c = col + plane * k;
                const float w_ = P[(lj + 1) * FW + 3 + li], e_ = P[(lj + 1) * FW + 8 + li];
                const f4 s4 = *reinterpret_cast<const f4*>(&P[lj * FW + 4 + li]);
                const f4 n4 = *reinterpret_cast<const f4*>(&P[(lj + 2) * FW + 4 + li]);
                const f4 q = aq4(pcc, wc, w_, e_, s4, n4, wb, wt, idx2);
                const f4 rn = rc - q;
                st4nt(r1, c, rn);
                v[0] += (double)dot4(rn, rn);
            }
            wb = wc;
            wc = wt;
            rc = rt;
            pcc = pct;
            buf ^= 1;
        }
    }
    block_reduce<1>(v, sh);
    if (threadIdx.x == 0) partials[r1_slot * MAX_BLOCKS + blockIdx.x] = v[0];
}

// Post-smoothing: z = z2 + S (r - A z2), partials <z,r> into slot zr_slot and, when rp
// is given, <z,rp> into slot zrp_slot.
__global__ void __launch_bounds__(NT) k_smooth_post_f4(Geo g, const uint8_t* __restrict__ pcode,
                                                       const float* __restrict__ z2, const float* __restrict__ r,
                                                       const float* __restrict__ rp, float* __restrict__ z,
                                                       double omega, double* __restrict__ partials, int nparts,
                                                       int zr_slot, int zrp_slot, const Solver* sv, int gate) {
    if (sv && stopped_before(sv, gate)) return;
    __shared__ double sh[2 * NT];
    __shared__ float sinv[16];
    const double dx2 = g.dx * g.dx;
    const float idx2 = (float)(1.0 / dx2);
    fill_sinv(sinv, omega, dx2);
    const int ntx4 = (g.nx + FTX - 1) / FTX;
    const int nzc = fslab_count(g.nz);
    const long long items = (long long)ntx4 * g.nty * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    double v[2] = {0.0, 0.0};
    for (long long w = w0; w < w1; ++w) {
        const VItem it_ = fitem(g, w, ntx4, nzc);
        if (!it_.valid) continue;
        const int i = it_.i, j = it_.j;
        const int iw = i == 0 ? g.nx - 1 : i - 1, ie = i + 4 >= g.nx ? 0 : i + 4;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j == g.ny - 1 ? 0 : j + 1;
        const long long col = (long long)i + (long long)g.nx * j;
        const long long ow = (long long)iw + (long long)g.nx * j - col;
        const long long oe = (long long)ie + (long long)g.nx * j - col;
        const long long os = (long long)i + (long long)g.nx * js - col;
        const long long on = (long long)i + (long long)g.nx * jn - col;
        const int zb = it_.z0 == 0 ? g.nz - 1 : it_.z0 - 1;
        f4 xb = ld4(z2, col + plane * zb);
        f4 xc = ld4(z2, col + plane * it_.z0);
        for (int k = it_.z0; k < it_.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = col + plane * k;
            const f4 xt = ld4(z2, col + plane * zt);
            const f4 xs = ld4(z2, c + os), xn = ld4(z2, c + on);
            const float xw = z2[c + ow], xe = z2[c + oe];
            const unsigned pc4 = ldc4(pcode, c);
            const f4 q = aq4(pc4, xc, xw, xe, xs, xn, xb, xt, idx2);
            const f4 rc = ld4(r, c);
            const f4 zn = xc + smul4(sinv, pc4, rc - q);
            st4nt(z, c, zn);
            v[0] += (double)dot4(zn, rc);
            if (rp) v[1] += (double)dot4(zn, ld4(rp, c));
            xb = xc;
            xc = xt;
        }
    }
    block_reduce<2>(v, sh);
    if (threadIdx.x == 0) {
        partials[zr_slot * MAX_BLOCKS + blockIdx.x] = v[0];
        if (rp) partials[zrp_slot * MAX_BLOCKS + blockIdx.x] = v[1];
    }
}

// One block: totals after a residual replacement (an init sweep with parity it) ->
// solver state of the next FP32 segment, which stops once its recursive <r,r> falls
// below max(delta^2 <r,r>, (eta_tol)^2 <b,b>).  The host checks the FP64 residual.
__global__ void __launch_bounds__(NT) k_seg_start(const double* partials, int nparts, Solver* sv, int it,
                                                  double delta, double eta_tol) {
    __shared__ double sh[4 * NT];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) {
        v[0] += partials[SLOT_B2 * MAX_BLOCKS + b];
        v[1] += partials[SLOT_R2D * MAX_BLOCKS + b];
        v[2] += partials[slot_rr(it) * MAX_BLOCKS + b];
        v[3] += partials[slot_rz(it) * MAX_BLOCKS + b];
    }
    block_reduce<4>(v, sh);
    if (threadIdx.x == 0) {
        sv->bnorm2 = v[0];
        sv->r64norm2 = v[1];
        sv->fnorm2 = v[1];
        sv->rr = v[2];
        sv->rz = v[3];
        sv->iters = it;
        sv->nan_seen = 0;
        sv->tol2 = fmax(delta * delta * v[2], eta_tol * eta_tol * v[0]);
        if (!(v[0] == v[0]) || !(v[1] == v[1]) || !(v[2] == v[2]) || !(v[3] == v[3])) {
            sv->nan_seen = 1;
            sv->converged = 3;
        } else {
            sv->converged = v[0] == 0.0 ? 2 : 0;
        }
        sv->stop_it = sv->converged ? it - 1 : STOP_NONE;
    }
}

// x += e (FP64 += FP32), e = 0
__global__ void k_accum_zero(long long n, double* __restrict__ x, float* __restrict__ e) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        x[i] = x[i] + (double)e[i];
        e[i] = 0.0f;
    }
}

// partials of ||b - L x||^2 and ||b||^2
__global__ void __launch_bounds__(NT) k_resid(Geo g, const uint8_t* __restrict__ pcode, const double* __restrict__ b, const double* __restrict__ x,
                                              double* __restrict__ partials) {
    __shared__ double sh[2 * NT];
    const double idx2 = 1.0 / (g.dx * g.dx);
    double v[2] = {0.0, 0.0};
    march(g, pcode, x, [&](long long c, uint8_t pc, double xc, double xw, double xe, double xs, double xn,
                           double xb, double xt) {
        double res = b[c] - lap_code(pc, xc, xw, xe, xs, xn, xb, xt, idx2);
        v[0] += res * res;
        v[1] += b[c] * b[c];
    });
    block_reduce<2>(v, sh);
    if (threadIdx.x == 0) {
        partials[SLOT_RES0 * MAX_BLOCKS + blockIdx.x] = v[0];
        partials[SLOT_RES1 * MAX_BLOCKS + blockIdx.x] = v[1];
    }
}

__global__ void __launch_bounds__(NT) k_sum2(const double* partials, int nparts, int s0, int s1, double* out) {
    __shared__ double sh[2 * NT];
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) {
        v[0] += partials[s0 * MAX_BLOCKS + b];
        v[1] += partials[s1 * MAX_BLOCKS + b];
    }
    block_reduce<2>(v, sh);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = v[1];
    }
}

// y = L x
__global__ void __launch_bounds__(NT) k_lap(Geo g, const uint8_t* __restrict__ pcode, const double* __restrict__ x, double* __restrict__ y) {
    const double idx2 = 1.0 / (g.dx * g.dx);
    march(g, pcode, x, [&](long long c, uint8_t pc, double xc, double xw, double xe, double xs, double xn,
                           double xb, double xt) { y[c] = lap_code(pc, xc, xw, xe, xs, xn, xb, xt, idx2); });
}

}  // namespace

// blocks of the z-marching sweeps: one per (tile, slab) item up to the partial capacity
int march_blocks(const Geo& g) {
    long long items = (long long)g.ntx * g.nty * slab_count(g.nz);
    return (int)(items < MAX_BLOCKS ? items : MAX_BLOCKS);
}

// The smoothing passes of the two-level learned preconditioner, nparts blocks each (one
// partial per block).  They need nx % 4 == 0 and 16-byte aligned vectors.
int smooth_pre(ibm_ctx* c, const float* r, float* r1, double omega, double* partials, int nparts, int r1_slot,
               int rr_slot, Solver* sv, int it, int check, hipStream_t s) {
    k_smooth_pre_f4<<<nparts, NT, 0, s>>>(c->geo, c->pcode, r, r1, omega, partials, nparts, r1_slot, rr_slot, sv, it,
                                          check);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int smooth_post(ibm_ctx* c, const float* z2, const float* r, const float* rp, float* z, double omega,
                double* partials, int nparts, int zr_slot, int zrp_slot, const Solver* sv, int gate, hipStream_t s) {
    k_smooth_post_f4<<<nparts, NT, 0, s>>>(c->geo, c->pcode, z2, r, zrp_slot >= 0 ? rp : nullptr, z, omega, partials,
                                           nparts, zr_slot, zrp_slot, sv, gate);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

static int fmarch_blocks(const Geo& g) {
    long long items = (long long)((g.nx + FTX - 1) / FTX) * g.nty * fslab_count(g.nz);
    return (int)(items < MAX_BLOCKS ? items : MAX_BLOCKS);
}

static int vmarch_blocks(const Geo& g) {
    long long items = (long long)((g.nx + VTX - 1) / VTX) * g.nty * vslab_count(g.nz);
    return (int)(items < MAX_BLOCKS ? items : MAX_BLOCKS);
}

// Event pairs around the timed sweeps, recorded on the launch stream; collected
// after the solve's final host synchronisation.
void timing_begin(ibm_ctx* c, int k, hipStream_t s) {
    if (!c->timing_on || c->ev_used[k] >= c->ev_cap) return;
    (void)hipEventRecord(c->ev[k][2 * c->ev_used[k]], s);
}

void timing_end(ibm_ctx* c, int k, hipStream_t s) {
    if (!c->timing_on || c->ev_used[k] >= c->ev_cap) return;
    (void)hipEventRecord(c->ev[k][2 * c->ev_used[k] + 1], s);
    c->ev_used[k] += 1;
}

void timing_collect(ibm_ctx* c) {
    if (!c->timing_on) return;
    for (int k = 0; k < TK_SLOTS_MAX; ++k) {
        for (int e = 0; e < c->ev_used[k]; ++e) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev[k][2 * e], c->ev[k][2 * e + 1]) == hipSuccess) {
                c->t_ms[k] += ms;
                c->t_launches[k] += 1;
            }
        }
        c->ev_used[k] = 0;
    }
}

// ---------------------------------------------------------- initial guess of a step
// A step's solve starts from p^n or from g = 2 p^n - p^{n-1}, whichever leaves the
// smaller residual ||b - L x||: the extrapolation pays once the flow is developed and
// overshoots while an impulsive start still changes the pressure quickly.  Partials of
// ||b - L p||^2 go to SLOT_RES0 and of ||b - L g||^2 to SLOT_RES1; every block of the
// picking kernel sums them in block order, so all blocks take the same decision.

__global__ void __launch_bounds__(NT) k_guess_fill(long long n, const double* __restrict__ p,
                                                   const double* __restrict__ pp, double* __restrict__ g) {
    for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < n; c += (long long)gridDim.x * NT)
        g[c] = 2.0 * p[c] - pp[c];
}

__global__ void __launch_bounds__(NT) k_guess_res(Geo g, const uint8_t* __restrict__ pcode,
                                                  const double* __restrict__ b, const double* __restrict__ x,
                                                  double* __restrict__ partials, int slot) {
    __shared__ double sh[NT];
    const double idx2 = 1.0 / (g.dx * g.dx);
    double v[1] = {0.0};
    march(g, pcode, x, [&](long long c, uint8_t pc, double xc, double xw, double xe, double xs, double xn,
                           double xb, double xt) {
        const double res = b[c] - lap_code(pc, xc, xw, xe, xs, xn, xb, xt, idx2);
        v[0] += res * res;
    });
    block_reduce<1>(v, sh);
    if (threadIdx.x == 0) partials[slot * MAX_BLOCKS + blockIdx.x] = v[0];
}

// p <- g where g leaves the smaller residual; p_prev <- p (old)
__global__ void __launch_bounds__(NT) k_guess_pick(long long n, const double* __restrict__ partials, int nparts,
                                                   double* __restrict__ p, double* __restrict__ pp,
                                                   const double* __restrict__ g) {
    __shared__ double sh[2 * NT];
    double v[2] = {0.0, 0.0};
    for (int q = threadIdx.x; q < nparts; q += NT) {
        v[0] += partials[SLOT_RES0 * MAX_BLOCKS + q];
        v[1] += partials[SLOT_RES1 * MAX_BLOCKS + q];
    }
    block_reduce<2>(v, sh);
    const bool use = v[1] < v[0];
    for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < n; c += (long long)gridDim.x * NT) {
        const double t = p[c];
        if (use) p[c] = g[c];
        pp[c] = t;
    }
}

int step_initial_guess(ibm_ctx* c, const double* b, double* p, double* p_prev, hipStream_t s) {
    const Geo& g = c->geo;
    const long long N = c->N;
    const int nb = march_blocks(g);
    const int ne = (int)std::min<long long>((N + NT - 1) / NT, 4096);
    double* gbuf = c->zbuf;   // free before the solve, which initialises it
    k_guess_fill<<<ne, NT, 0, s>>>(N, p, p_prev, gbuf);
    k_guess_res<<<nb, NT, 0, s>>>(g, c->pcode, b, p, c->partials, SLOT_RES0);
    k_guess_res<<<nb, NT, 0, s>>>(g, c->pcode, b, gbuf, c->partials, SLOT_RES1);
    k_guess_pick<<<ne, NT, 0, s>>>(N, c->partials, nb, p, p_prev, gbuf);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int laplacian_run(ibm_ctx* c, const double* x, double* y, hipStream_t s) {
    k_lap<<<march_blocks(c->geo), NT, 0, s>>>(c->geo, c->pcode, x, y);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int true_residual(ibm_ctx* c, const double* b, const double* x, double* rel, hipStream_t s) {
    const int nb = march_blocks(c->geo);
    k_resid<<<nb, NT, 0, s>>>(c->geo, c->pcode, b, x, c->partials);
    k_sum2<<<1, NT, 0, s>>>(c->partials, nb, SLOT_RES0, SLOT_RES1, c->red);
    IBM_HIP(hipGetLastError());
    IBM_HIP(hipMemcpyAsync(c->h_red, c->red, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    *rel = c->h_red[1] > 0.0 ? sqrt(c->h_red[0] / c->h_red[1]) : 0.0;
    return IBM_OK;
}

// Conjugate-gradient iterations from iteration start_it (0: after an init + start
// pair; otherwise after a residual replacement, whose first pass A skips the x update);
// vectors of type T.  path: 0 scalar sweeps, 1 pairs of cells per lane, 2 (float
// only) four cells per lane.  Sets *done to the iterations made.  Returns the device
// flag (0 not converged at the cap, 1 converged, 2 trivial, 3 NaN).
template <class T>
static int cg_loop(ibm_ctx* c, T* x, T* r, T* z, T* d0, T* d1, int path, int nred, int start_it, int max_iter,
                   int check_every, int* last_iters, int* done, hipStream_t s, bool fresh = false) {
    const Geo& g = c->geo;
    T* dbuf[2] = {d0, d1};
    // the first pass A of a fresh start takes d = z (no previous direction, no x update)
    auto first_pass = [&](int it) { return it == 0 || (fresh && it == start_it); };
    auto pass_a = [&](int it) {
        T* dnew = dbuf[it & 1];
        T* dold = dbuf[(it + 1) & 1];
        const int skip = (start_it > 0 && it == start_it) ? 1 : 0;
        const int K = TK_SPMV;
        if constexpr (std::is_same<T, float>::value) {
            if (path == 2) {
                if (first_pass(it))
                    launch_timed(c, K, k_pcg_a_f4<true>, nred, s, g, (const uint8_t*)c->pcode, (const float*)z,
                                 (const float*)dold, dnew, x, c->partials, nred, it, 0, c->solver);
                else
                    launch_timed(c, K, k_pcg_a_f4<false>, nred, s, g, (const uint8_t*)c->pcode, (const float*)z,
                                 (const float*)dold, dnew, x, c->partials, nred, it, skip, c->solver);
                return;
            }
        }
        if (path == 1) {
            if (first_pass(it))
                launch_timed(c, K, k_pcg_a_v<T, true>, nred, s, g, (const uint8_t*)c->pcode, (const T*)z,
                             (const T*)dold, dnew, x, c->partials, nred, it, 0, c->solver);
            else
                launch_timed(c, K, k_pcg_a_v<T, false>, nred, s, g, (const uint8_t*)c->pcode, (const T*)z,
                             (const T*)dold, dnew, x, c->partials, nred, it, skip, c->solver);
        } else {
            launch_timed(c, K, k_pcg_a<T>, nred, s, g, (const uint8_t*)c->pcode, (const T*)z, (const T*)dold, dnew, x,
                         c->partials, nred, it, 0, skip, (fresh && it == start_it) ? 1 : 0, c->solver);
        }
    };
    auto pass_b = [&](int it) {
        T* dnew = dbuf[it & 1];
        const int K = TK_UPDATE;
        if constexpr (std::is_same<T, float>::value) {
            if (path == 2) {
                launch_timed(c, K, k_pcg_b_f4<true>, nred, s, g, (const uint8_t*)c->pcode, (const float*)dnew,
                             (const float*)r, r, z, c->partials, nred, it, (const Solver*)c->solver);
                return;
            }
        }
        if (path == 1)
            launch_timed(c, K, k_pcg_b_v<T>, nred, s, g, (const uint8_t*)c->pcode, (const T*)dnew, r, z, c->partials,
                         nred, it, (const Solver*)c->solver);
        else
            launch_timed(c, K, k_pcg_b<T>, nred, s, g, (const uint8_t*)c->pcode, (const T*)dnew, r, z, c->partials,
                         nred, it, (const Solver*)c->solver);
    };
    if (check_every <= 0) check_every = 16;
    int batch = *last_iters > 0 ? *last_iters + 2 : check_every;
    if (batch > max_iter) batch = max_iter;
    int total = 0;
    while (true) {
        int n = batch;
        if (n > max_iter - total) n = max_iter - total;
        for (int k = 0; k < n; ++k) {
            const int it = start_it + total + k;
            pass_a(it);
            pass_b(it);
        }
        IBM_HIP(hipGetLastError());
        total += n;
        if (total >= max_iter) {
            // at the cap, one more pass A tests r and applies the last x update (when not
            // converged it also starts a direction that a later segment recomputes)
            pass_a(start_it + total);
            IBM_HIP(hipGetLastError());
        }
        // otherwise a residual that converged in the last pass B is detected by the
        // first pass A of the next batch, which then only applies the last x update
        IBM_HIP(hipMemcpyAsync(c->h_solver, c->solver, sizeof(Solver), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (c->progress) c->progress(c->progress_user, c->progress_iters + total, c->h_solver->rr);
        if (c->h_solver->converged || total >= max_iter) break;
        batch = check_every;
    }
    int made = c->h_solver->iters - start_it;
    if (made < 0) made = 0;
    *done = made;
    *last_iters = made;
    timing_collect(c);
    if (c->timing_on) c->t_real_iters += made;
    return c->h_solver->converged;
}

static bool vec_ok(const Geo& g, const void* p, size_t align) {
    return (g.nx % 2) == 0 && ((uintptr_t)p % align) == 0;
}

// FP64 Jacobi PCG on L x = b (b already compatible); x in/out.  Sets *iters.
int pcg64(ibm_ctx* c, const double* b, double* x, double tol, int max_iter, int check_every, int* iters,
          hipStream_t s) {
    const Geo& g = c->geo;
    // even nx: the double2 passes; every reduction of the solve is then written by nred
    // blocks (the init sweep runs with the same count), so all partial sums agree
    const bool vec = vec_ok(g, x, 16);
    const int nred = vec ? vmarch_blocks(g) : march_blocks(g);
    k_pcg_init<double><<<nred, NT, 0, s>>>(g, c->pcode, b, x, c->r, c->zbuf, c->partials, 0);
    k_pcg_start<<<1, NT, 0, s>>>(c->partials, nred, c->solver, tol, SLOT_B2);
    k_zero_if_trivial<<<1024, 256, 0, s>>>(c->N, x, c->solver);
    IBM_HIP(hipGetLastError());
    int flag = cg_loop<double>(c, x, c->r, c->zbuf, c->d, c->q, vec ? 1 : 0, nred, 0, max_iter, check_every,
                               &c->last_iters, iters, s);
    if (flag < 0) return flag;
    if (flag == 3) {
        set_error("pressure solve: non-finite residual");
        return IBM_ERR_NAN;
    }
    return flag ? IBM_OK : IBM_NOT_CONVERGED;
}

__global__ void k_zero_f32(long long n, float* __restrict__ e) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        e[i] = 0.0f;
}

__global__ void k_zero_f64(long long n, double* __restrict__ x) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

// ------------------------------------------------------------- flexible CG
//
// FCG(1) in FP32 with the learned preconditioner (cnn.hip) on the correction equation:
//   z = M(r);  beta = <z, r - r_prev> / <z_prev, r_prev> (0 at a restart);  d = z + beta d;
//   q = A d;  alpha = <z, r> / <d, q>;  e += alpha d;  r_prev = r;  r -= alpha q.
// Slots of the partial sums: <r,r> of the update in FCG_RR (the first iteration of a
// segment reads the init sweep's RR slot), <z,r> ping-pong in FCG_ZR + parity,
// <z, r_prev> in FCG_ZRP, <d,q> in FCG_DQ.  Every kernel exits at once after the
// segment has converged (the preconditioner's input kernel makes that test).
// d = z + beta d (beta = 0 when first); stops the segment when <z,r> is not positive
// (the preconditioner is then not a descent direction) or not finite.
__global__ void __launch_bounds__(NT) k_fcg_dir(long long n, const float* __restrict__ z, float* __restrict__ d,
                                                const double* __restrict__ partials, int nparts, int zr_slot,
                                                int zrprev_slot, int first, int it, Solver* sv) {
    if (stopped_before(sv, it + 1)) return;
    __shared__ double sh[12];
    const int sl[3] = {zr_slot, FCG_ZRP, zrprev_slot};
    double tot[3];
    sum_slots<3>(partials, sl, nparts, sh, tot);
    const double zr = tot[0];
    if (!(zr > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (zr == zr) {
                sv->converged = 1;   // no descent: end the segment, the FP64 check decides
            } else {
                sv->nan_seen = 1;
                sv->converged = 3;
            }
            sv->stop_it = it;
        }
        return;
    }
    const float beta = first ? 0.0f : (float)((zr - tot[1]) / tot[2]);
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
        d[i] = first ? z[i] : fmaf(beta, d[i], z[i]);
}

// q = A d (FP32), partial <d,q>
__global__ void __launch_bounds__(NT) k_fcg_q(Geo g, const uint8_t* __restrict__ pcode, const float* __restrict__ d,
                                              float* __restrict__ q, double* __restrict__ partials, int it,
                                              Solver* sv) {
    if (stopped_before(sv, it + 1)) return;
    __shared__ double sh[4];
    const float idx2 = (float)(1.0 / (g.dx * g.dx));
    const long long n = (long long)g.nx * g.ny * g.nz;
    double v[1] = {0.0};
    for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < n; c += (long long)gridDim.x * NT) {
        const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / ((long long)g.nx * g.ny));
        const uint8_t pc = pcode[c];
        const float dc = d[c];
        float acc = (float)jcount(pc) * dc;
        for (int dd = 0; dd < 6; ++dd) {
            if (pc & (1 << dd)) {
                bool bnd;
                acc -= d[nb_index(g, i, j, k, dd, bnd)];
            }
        }
        const float qc = acc * idx2;
        q[c] = qc;
        v[0] += (double)dc * (double)qc;
    }
    block_reduce<1>(v, sh);
    if (threadIdx.x == 0) partials[FCG_DQ * MAX_BLOCKS + blockIdx.x] = v[0];
}

// e += alpha d; r_new = r - alpha q; partial <r_new, r_new>
__global__ void __launch_bounds__(NT) k_fcg_upd(long long n, float* __restrict__ e, const float* __restrict__ d,
                                                const float* __restrict__ q, const float* __restrict__ r,
                                                float* __restrict__ rnew, double* __restrict__ partials, int nparts,
                                                int zr_slot, int it, Solver* sv) {
    if (stopped_before(sv, it + 1)) return;
    __shared__ double sh[8];
    const int sl[2] = {zr_slot, FCG_DQ};
    double tot[2];
    sum_slots<2>(partials, sl, nparts, sh, tot);
    const float alpha = (float)(tot[0] / tot[1]);
    double v[1] = {0.0};
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
        e[i] = fmaf(alpha, d[i], e[i]);
        const float rn = fmaf(-alpha, q[i], r[i]);
        rnew[i] = rn;
        v[0] += (double)rn * (double)rn;
    }
    block_reduce<1>(v, sh);
    if (threadIdx.x == 0) partials[FCG_RR * MAX_BLOCKS + blockIdx.x] = v[0];
}

// One FCG segment on the fused FP32 passes (nx % 4 == 0), from a residual replacement
// whose init sweep wrote the RR slot of parity it0 (r in c->r32, e = 0).  Iteration it:
// the network gives z_it = M(r_it) with <z,r> in RZ(it) and <z, r_{it-1}> in FCG_ZRP;
// pass A (flexible beta) applies the lagging x update, forms d_it and <d, A d>; pass B
// writes r_{it+1} into the other residual buffer with <r,r>.  Convergence is tested by
// pass A, as in cg_loop.  Sets *made; returns the device flag.
static int fcg_segment_fused(ibm_ctx* c, int nred, int it0, int max_iter, int check_every, double omega, int* made,
                             hipStream_t s) {
    const Geo& g = c->geo;
    float* rb[2] = {c->r32, c->zprev32};
    float* dbuf[2] = {c->d32, c->q32};
    int cur = 0;
    if (check_every <= 0) check_every = 8;
    int total = 0;
    int batch = c->last_iters_inner > 0 ? c->last_iters_inner + 1 : check_every;
    auto pass_a = [&](int it, int k) {
        float* dnew = dbuf[it & 1];
        float* dold = dbuf[(it + 1) & 1];
        if (k == 0)
            k_pcg_a_f4<true><<<nred, NT, 0, s>>>(g, c->pcode, c->z32, dold, dnew, c->e32, c->partials, nred, it, 0,
                                                 c->solver);
        else
            k_pcg_a_f4<false, true><<<nred, NT, 0, s>>>(g, c->pcode, c->z32, dold, dnew, c->e32, c->partials, nred,
                                                        it, 0, c->solver);
    };
    while (true) {
        int nb = batch;
        if (nb > max_iter - total) nb = max_iter - total;
        for (int k = total; k < total + nb; ++k) {
            const int it = it0 + k;
            timing_begin(c, TK_SPMV, s);
            int rc = cnn_precondition_solver(c->cnn, c, rb[cur], k ? rb[cur ^ 1] : nullptr, c->z32, c->partials, nred,
                                             slot_rr_host(it), slot_rz_host(it), k ? FCG_ZRP : -1, FCG_R1, omega,
                                             c->solver, it, 0, s);
            timing_end(c, TK_SPMV, s);
            if (rc) return rc;
            timing_begin(c, TK_UPDATE, s);
            pass_a(it, k);
            k_pcg_b_f4<false><<<nred, NT, 0, s>>>(g, c->pcode, dbuf[it & 1], rb[cur], rb[cur ^ 1], nullptr, c->partials,
                                                  nred, it, c->solver);
            timing_end(c, TK_UPDATE, s);
            cur ^= 1;
        }
        IBM_HIP(hipGetLastError());
        total += nb;
        if (total >= max_iter) {
            pass_a(it0 + total, total);   // tests r and applies the last x update
            IBM_HIP(hipGetLastError());
        }
        IBM_HIP(hipMemcpyAsync(c->h_solver, c->solver, sizeof(Solver), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (c->progress) c->progress(c->progress_user, c->progress_iters + total, c->h_solver->rr);
        if (c->h_solver->converged || total >= max_iter) break;
        batch = check_every;
    }
    int m = c->h_solver->iters - it0;
    if (m < 0) m = 0;
    *made = m;
    c->last_iters_inner = m;
    timing_collect(c);
    if (c->timing_on) c->t_real_iters += m;
    return c->h_solver->converged;
}

// One FCG segment from a residual replacement whose init sweep wrote the RR slot of
// parity it0 (r in c->r32, e = 0).  Sets *made to the iterations made; returns the
// device flag as cg_loop does.
static int fcg_segment(ibm_ctx* c, int nred, int it0, int max_iter, int check_every, double omega, int* made,
                       hipStream_t s) {
    const Geo& g = c->geo;
    float* rb[2] = {c->r32, c->zprev32};
    int cur = 0;
    if (check_every <= 0) check_every = 8;
    int total = 0;
    int batch = c->last_iters_inner > 0 ? c->last_iters_inner + 1 : check_every;
    while (true) {
        int nb = batch;
        if (nb > max_iter - total) nb = max_iter - total;
        for (int k = total; k < total + nb; ++k) {
            const int it = it0 + k;
            const int zr = FCG_ZR + (k & 1), zrprev = FCG_ZR + ((k + 1) & 1);
            timing_begin(c, TK_SPMV, s);
            int rc = cnn_precondition_solver(c->cnn, c, rb[cur], k ? rb[cur ^ 1] : nullptr, c->z32, c->partials, nred,
                                             k ? FCG_RR : slot_rr_host(it0), zr, k ? FCG_ZRP : -1, FCG_R1, omega,
                                             c->solver, it, 1, s);
            timing_end(c, TK_SPMV, s);
            if (rc) return rc;
            timing_begin(c, TK_UPDATE, s);
            k_fcg_dir<<<nred, NT, 0, s>>>(c->N, c->z32, c->d32, c->partials, nred, zr, zrprev, k == 0 ? 1 : 0, it,
                                          c->solver);
            k_fcg_q<<<nred, NT, 0, s>>>(g, c->pcode, c->d32, c->q32, c->partials, it, c->solver);
            k_fcg_upd<<<nred, NT, 0, s>>>(c->N, c->e32, c->d32, c->q32, rb[cur], rb[cur ^ 1], c->partials, nred, zr,
                                          it, c->solver);
            timing_end(c, TK_UPDATE, s);
            cur ^= 1;
        }
        IBM_HIP(hipGetLastError());
        total += nb;
        IBM_HIP(hipMemcpyAsync(c->h_solver, c->solver, sizeof(Solver), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (c->progress) c->progress(c->progress_user, c->progress_iters + total, c->h_solver->rr);
        if (c->h_solver->converged || total >= max_iter) break;
        batch = check_every;
    }
    int m = c->h_solver->converged ? c->h_solver->iters - it0 : total;
    if (m < 0) m = 0;
    *made = m;
    c->last_iters_inner = m;
    timing_collect(c);
    if (c->timing_on) c->t_real_iters += m;
    return c->h_solver->converged;
}

// FP64 iterative refinement with residual replacement around FP32 segments.  The FP64
// residual r64 = b - L x (the convergence check) is rounded to FP32 and a segment works on
// A e = -r64 until its recursive residual has fallen by inner_tol (or below
// eta tol ||b||); then x += e in FP64, e = 0, and r64 is recomputed and replaces the
// FP32 residual.  Stops when ||r64|| <= tol ||b||.  A segment that shrinks ||r64|| by
// less than stall_factor, a non-finite value, too many segments, or the force_stall
// hook hand the solve to FP64 PCG from the current x.
// seg(it, &made) runs one segment from global iteration it and returns its flag.
template <class Seg>
static int refine_solve(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st, int nred,
                        bool can_retry, Seg&& seg, hipStream_t s) {
    const Geo& g = c->geo;
    const long long N = c->N;
    const double delta = (o->inner_tol > 0.0 && o->inner_tol < 1.0) ? o->inner_tol : 0.1;
    const double stall = o->stall_factor > 1.0 ? o->stall_factor : 2.0;
    const double eta_tol = 0.25 * o->tol;   // last segment aims below tol, leaving room for FP32 drift
    const int max_sweeps = 200;
    int total_inner = 0, sweeps = 0, it = 0;
    double prev_rel = -1.0;
    bool fallback = false;
    // a stalled segment is retried from a fresh direction (when the segments keep theirs)
    // up to max_retries times before the FP64 fallback
    const int max_retries = 3;
    int retries = 0;
    bool fresh = false, last_fresh = false;
    int rc = IBM_OK;
    c->progress_iters = 0;
    k_zero_f32<<<2048, 256, 0, s>>>(N, c->e32);
    k_pcg_init<float><<<nred, NT, 0, s>>>(g, c->pcode, b, x, c->r32, c->z32, c->partials, 0);
    k_seg_start<<<1, NT, 0, s>>>(c->partials, nred, c->solver, 0, delta, eta_tol);
    IBM_HIP(hipGetLastError());
    while (true) {
        IBM_HIP(hipMemcpyAsync(c->h_solver, c->solver, sizeof(Solver), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        const double bn2 = c->h_solver->bnorm2, rn2 = c->h_solver->r64norm2;
        if (bn2 == 0.0 && c->h_solver->converged != 3) {
            k_zero_f64<<<2048, 256, 0, s>>>(N, x);   // b = 0: x = 0 (zero mean on enclosed components)
            IBM_HIP(hipGetLastError());
            break;
        }
        const double rel = sqrt(rn2 / bn2);
        if (c->progress) c->progress(c->progress_user, total_inner, -rel);
        if (!(rel == rel) || c->h_solver->converged == 3) {
            fallback = true;
            break;
        }
        if (rel <= o->tol) break;
        fresh = false;
        if (prev_rel >= 0.0 && (rel * stall > prev_rel || (o->force_stall && sweeps == 1))) {
            // a segment that kept the previous Krylov direction gets one retry from a
            // fresh one; a fresh segment that stalls (or the test hook) falls back
            if (!can_retry || last_fresh || retries >= max_retries || o->force_stall == 1) {
                fallback = true;
                break;
            }
            ++retries;
            fresh = true;
        }
        if (sweeps >= max_sweeps || total_inner >= o->max_iter) {
            fallback = true;
            break;
        }
        prev_rel = rel;
        int made = 0;
        c->progress_iters = total_inner;
        int flag = seg(it, fresh, &made);
        last_fresh = fresh;
        if (flag < 0) return flag;
        total_inner += made;
        it += made;
        sweeps += 1;
        if (flag == 3) {
            fallback = true;
            break;
        }
        k_accum_zero<<<2048, 256, 0, s>>>(N, x, c->e32);
        k_pcg_init<float><<<nred, NT, 0, s>>>(g, c->pcode, b, x, c->r32, c->z32, c->partials, it);
        k_seg_start<<<1, NT, 0, s>>>(c->partials, nred, c->solver, it, delta, eta_tol);
        IBM_HIP(hipGetLastError());
    }
    int fb_iters = 0;
    if (fallback) {
        c->progress_iters = total_inner;
        rc = pcg64(c, b, x, o->tol, o->max_iter, o->check_every, &fb_iters, s);
        if (rc < 0) return rc;
    }
    if (st) {
        st->iters_inner = total_inner + fb_iters;
        st->iters_outer = sweeps;
        st->fallback_used = fallback ? 1 : 0;
        st->iters_fallback = fb_iters;
    }
    return rc;
}

// Mixed precision with Jacobi: FP32 CG segments that keep their search direction across
// the residual replacements (the Krylov information of earlier segments is kept).
int mixed_solve(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st, hipStream_t s) {
    const Geo& g = c->geo;
    const bool quad = (g.nx % 4) == 0 && ((uintptr_t)c->r32 % 16) == 0 && ((uintptr_t)c->z32 % 16) == 0 &&
                      ((uintptr_t)c->e32 % 16) == 0 && ((uintptr_t)c->d32 % 16) == 0 &&
                      ((uintptr_t)c->q32 % 16) == 0;
    const bool pair = vec_ok(g, c->r32, 8);
    const int path = quad ? 2 : (pair ? 1 : 0);
    const int nred = quad ? fmarch_blocks(g) : (pair ? vmarch_blocks(g) : march_blocks(g));
    const int inner_max = o->inner_max_iter > 0 ? o->inner_max_iter : 1000;
    return refine_solve(
        c, b, x, o, st, nred, o->inner_restart == 0,
        [&](int it, bool fresh, int* made) {
            return cg_loop<float>(c, c->e32, c->r32, c->z32, c->d32, c->q32, path, nred, it, inner_max,
                                  o->check_every, &c->last_iters_inner, made, s, fresh || o->inner_restart != 0);
        },
        s);
}

// Mixed precision with the learned preconditioner: FCG(1) segments, restarted at every
// residual replacement (the BF16 preconditioner is only nearly symmetric, so the
// flexible beta is used and no Krylov space is carried across replacements).
int cnn_fcg_solve(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st, hipStream_t s) {
    if (!c->cnn) {
        set_error("IBM_SOLVER_FCG_CNN: no network attached to the context");
        return IBM_ERR_ARG;
    }
    if (!cnn_covers(c->cnn, c->N)) {
        set_error("IBM_SOLVER_FCG_CNN: network workspace smaller than the grid");
        return IBM_ERR_ARG;
    }
    const Geo& g = c->geo;
    const bool quad = (g.nx % 4) == 0 && ((uintptr_t)c->r32 % 16) == 0 && ((uintptr_t)c->zprev32 % 16) == 0 &&
                      ((uintptr_t)c->z32 % 16) == 0 && ((uintptr_t)c->e32 % 16) == 0 &&
                      ((uintptr_t)c->d32 % 16) == 0 && ((uintptr_t)c->q32 % 16) == 0;
    const int nred = quad ? fmarch_blocks(g) : march_blocks(g);
    const int inner_max = o->inner_max_iter > 0 ? o->inner_max_iter : 1000;
    // damped Jacobi weight of the smoothing steps around the network (0: additive form)
    const double omega = o->omega > 0.0 ? o->omega : 0.0;
    if (omega > 1.0 || (omega > 0.0 && !quad)) {
        set_error("IBM_SOLVER_FCG_CNN: smoothing weight omega must lie in (0, 1] and needs nx % 4 == 0");
        return IBM_ERR_ARG;
    }
    int rc = cnn_prepare_geometry(c->cnn, c, s);
    if (rc) return rc;
    return refine_solve(
        c, b, x, o, st, nred, false,
        [&](int it, bool, int* made) {
            return quad ? fcg_segment_fused(c, nred, it, inner_max, o->check_every, omega, made, s)
                        : fcg_segment(c, nred, it, inner_max, o->check_every, omega, made, s);
        },
        s);
}

// ------------------------------------------------------------- red-black SOR

// One half sweep of red-black successive over-relaxation on L x = b (Sec. 2.1): every
// cell of the given colour (parity of i + j + k) with L_cc != 0 gets
// x_c += omega (b_c - (L x)_c) / L_cc.  All neighbours of such a cell have the other
// colour (periodic axes have even counts, checked by the host), so the cells of one
// half sweep read only values that it does not write.  Columns of (tile, z-slab) items
// as in the conjugate-gradient passes.
__global__ void __launch_bounds__(NT) k_sor(Geo g, const uint8_t* __restrict__ pcode, const double* __restrict__ b,
                                            double* __restrict__ x, int colour, double omega) {
    const double idx2 = 1.0 / (g.dx * g.dx);
    const int nzc = slab_count(g.nz);
    const long long tiles = (long long)g.ntx * g.nty;
    const long long items = tiles * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    const long long w0 = items * ch / nb, w1 = items * (ch + 1) / nb;
    const long long plane = (long long)g.nx * g.ny;
    for (long long w = w0; w < w1; ++w) {
        const int zc = (int)(w / tiles);
        const long long t = w % tiles;
        const int i = (int)(t % g.ntx) * TX + (threadIdx.x % TX);
        const int j = (int)(t / g.ntx) * TY + (threadIdx.x / TX);
        const int z0 = (int)((long long)g.nz * zc / nzc), z1 = (int)((long long)g.nz * (zc + 1) / nzc);
        if (i >= g.nx || j >= g.ny) continue;
        const int iw = i == 0 ? g.nx - 1 : i - 1, ie = i == g.nx - 1 ? 0 : i + 1;
        const int js = j == 0 ? g.ny - 1 : j - 1, jn = j == g.ny - 1 ? 0 : j + 1;
        const long long col = (long long)i + (long long)g.nx * j;
        const long long ow = (long long)iw + (long long)g.nx * j - col;
        const long long oe = (long long)ie + (long long)g.nx * j - col;
        const long long os = (long long)i + (long long)g.nx * js - col;
        const long long on = (long long)i + (long long)g.nx * jn - col;
        // first plane of the slab with the wanted colour, then every second plane
        const int k0 = z0 + (((i + j + z0) & 1) != colour ? 1 : 0);
        for (int k = k0; k < z1; k += 2) {
            const long long c = col + plane * k;
            const uint8_t pc = pcode[c];
            const double cnt = jacobi_count(pc);
            if (cnt == 0.0) continue;
            const int zb = k == 0 ? g.nz - 1 : k - 1, zt = k == g.nz - 1 ? 0 : k + 1;
            const double xc = x[c];
            const double lx = lap_code(pc, xc, x[c + ow], x[c + oe], x[c + os], x[c + on], x[col + plane * zb],
                                       x[col + plane * zt], idx2);
            x[c] = xc + omega * (b[c] - lx) / (-cnt * idx2);
        }
    }
}

// Red-black SOR on L x = b (b already compatible); x in/out.  The true residual is
// tested every check_every sweeps (and at the cap); sets *sweeps.
static int rbsor64(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, int* sweeps, hipStream_t s) {
    const Geo& g = c->geo;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k)
        if (g.bc[2 * k] == IBM_BC_PERIODIC && (n[k] & 1)) {
            set_error("red-black SOR: periodic axes need an even number of cells");
            return IBM_ERR_ARG;
        }
    const int nmax = n[0] > n[1] ? (n[0] > n[2] ? n[0] : n[2]) : (n[1] > n[2] ? n[1] : n[2]);
    const double omega = o->omega > 0.0 ? o->omega : 2.0 / (1.0 + sin(M_PI / (double)nmax));
    if (!(omega > 0.0 && omega < 2.0)) {
        set_error("red-black SOR: need 0 < omega < 2");
        return IBM_ERR_ARG;
    }
    const int check = o->check_every > 0 ? o->check_every : 16;
    const int nb = march_blocks(g);
    int it = 0;
    *sweeps = 0;
    while (true) {
        double rel = 0.0;
        if (int rc = true_residual(c, b, x, &rel, s)) return rc;
        if (c->h_red[1] == 0.0) {   // b = 0: x = 0
            k_zero_f64<<<1024, 256, 0, s>>>(c->N, x);
            IBM_HIP(hipGetLastError());
            break;
        }
        if (!(rel == rel)) {
            set_error("red-black SOR: non-finite residual");
            return IBM_ERR_NAN;
        }
        if (c->progress) c->progress(c->progress_user, it, rel * rel * c->h_red[1]);
        if (rel <= o->tol) break;
        if (it >= o->max_iter) {
            *sweeps = it;
            timing_collect(c);
            return IBM_NOT_CONVERGED;
        }
        const int todo = check < o->max_iter - it ? check : o->max_iter - it;
        for (int q = 0; q < todo; ++q) {
            launch_timed(c, TK_SPMV, k_sor, nb, s, g, (const uint8_t*)c->pcode, b, x, 0, omega);
            launch_timed(c, TK_SPMV, k_sor, nb, s, g, (const uint8_t*)c->pcode, b, x, 1, omega);
        }
        IBM_HIP(hipGetLastError());
        it += todo;
    }
    *sweeps = it;
    timing_collect(c);
    if (c->timing_on) c->t_real_iters += it;
    return IBM_OK;
}

int poisson_run(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st, hipStream_t s) {
    int iters = 0;
    int rc;
    ibm_stats local;
    if (o->kind == IBM_SOLVER_FCG_JACOBI) {
        rc = mixed_solve(c, b, x, o, &local, s);
        iters = local.iters_inner;
    } else if (o->kind == IBM_SOLVER_PCG_JACOBI) {
        c->progress_iters = 0;
        rc = pcg64(c, b, x, o->tol, o->max_iter, o->check_every, &iters, s);
        local.iters_outer = 0;
        local.fallback_used = 0;
        local.iters_fallback = 0;
    } else if (o->kind == IBM_SOLVER_FCG_CNN) {
        rc = cnn_fcg_solve(c, b, x, o, &local, s);
        iters = local.iters_inner;
    } else if (o->kind == IBM_SOLVER_RBSOR) {
        rc = rbsor64(c, b, x, o, &iters, s);
        local.iters_outer = 0;
        local.fallback_used = 0;
        local.iters_fallback = 0;
    } else {
        set_error("unknown solver kind");
        return IBM_ERR_ARG;
    }
    if (rc < 0) return rc;
    int rc2 = remove_means(c, x, s);
    if (rc2) return rc2;
    if (st) {
        st->iters_inner = iters;
        st->iters_outer = local.iters_outer;
        st->fallback_used = local.fallback_used;
        st->iters_fallback = local.iters_fallback;
        st->status = rc;
        int rc3 = true_residual(c, b, x, &st->rel_residual, s);
        if (rc3) return rc3;
    }
    return rc;
}

}  // namespace ibm
