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

#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "common.h"

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

}  // extern "C"
