// Near-field surface pressure and force by Shepard interpolation (eq. (force)): the
// cell-centre pressure is averaged at every triangle vertex X with weights
// 1 / |X - x_k|^2 over the eight cell centres x_k that span the dual cell containing X,
// separately for the points in front of the triangle (n . (x_k - X) > 0) and behind it
// (< 0); points in its plane count for neither side.  A triangle's side value is the
// mean over its vertices that have one; its force is A n (p_back - p_front), a side
// without points contributing nothing.  Triangles of zero, overflowing or non-finite
// area have no values and no force.
//
// One thread per triangle, 24 gathers of the pressure.  The source is compiled without
// FMA contraction and every sum is written out left to right, so that each triangle's
// values (and the front/back decision of every point) are one fixed FP64 computation.
// The force is summed over the triangles through per-block partials in block order.
//
// Thin-plate filter Z of eq. (force_filter), optional: a point is left out at a vertex
// when the segment from the vertex to it crosses a triangle of the surface at a
// parameter t in (T_MIN, 1] (Moller-Trumbore, edges inclusive), i.e. when the point lies
// behind another face, as the far side of a plate thinner than a cell does.  Candidate
// triangles come from uniform bins of 2x2x2 cells (counted with global atomics, an
// exclusive scan, filled with global atomics); the order inside a bin does not matter,
// since only whether some triangle is crossed counts.  The crossing flags of all
// (triangle, vertex, corner) triples are computed first, one thread each.

#include <cfloat>
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace ibm {
namespace {

constexpr double T_MIN = 1e-6;
constexpr int BIN_CELLS = 2;

struct Bins {
    int nbx, nby, nbz;
    double bdx, ox, oy, oz;
    const long long* off;   // nbins + 1 offsets into ids
    const int* ids;   // triangle ids per bin
};

__device__ inline int bin_of(double v, double o, double bdx, int nb) {
    const double f = floor((v - o) / bdx);
    if (!(f >= 0.0)) return 0;
    if (f > (double)(nb - 1)) return nb - 1;
    return (int)f;
}

// whether the segment P + t (Q - P) meets triangle v at some t in (T_MIN, 1]
__device__ inline bool seg_hits(double px, double py, double pz, double dx_, double dy, double dz,
                                const double* __restrict__ v) {
    const double e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
    const double e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
    const double pvx = dy * e2z - dz * e2y, pvy = dz * e2x - dx_ * e2z, pvz = dx_ * e2y - dy * e2x;
    const double det = e1x * pvx + e1y * pvy + e1z * pvz;
    if (det == 0.0) return false;
    const double inv = 1.0 / det;
    const double tx = px - v[0], ty = py - v[1], tz = pz - v[2];
    const double u = (tx * pvx + ty * pvy + tz * pvz) * inv;
    const double qx = ty * e1z - tz * e1y, qy = tz * e1x - tx * e1z, qz = tx * e1y - ty * e1x;
    const double w = (dx_ * qx + dy * qy + dz * qz) * inv;
    const double t = (e2x * qx + e2y * qy + e2z * qz) * inv;
    return u >= 0.0 && u <= 1.0 && w >= 0.0 && u + w <= 1.0 && t > T_MIN && t <= 1.0;
}

__device__ inline bool occluded(const Bins& B, const double* __restrict__ tri, double px, double py, double pz,
                                double qx, double qy, double qz) {
    const int x0 = bin_of(fmin(px, qx), B.ox, B.bdx, B.nbx), x1 = bin_of(fmax(px, qx), B.ox, B.bdx, B.nbx);
    const int y0 = bin_of(fmin(py, qy), B.oy, B.bdx, B.nby), y1 = bin_of(fmax(py, qy), B.oy, B.bdx, B.nby);
    const int z0 = bin_of(fmin(pz, qz), B.oz, B.bdx, B.nbz), z1 = bin_of(fmax(pz, qz), B.oz, B.bdx, B.nbz);
    const double dx_ = qx - px, dy = qy - py, dz = qz - pz;
    for (int bz = z0; bz <= z1; ++bz)
        for (int by = y0; by <= y1; ++by)
            for (int bx = x0; bx <= x1; ++bx) {
                const long long b = bx + (long long)B.nbx * (by + (long long)B.nby * bz);
                for (long long e = B.off[b]; e < B.off[b + 1]; ++e)
                    if (seg_hits(px, py, pz, dx_, dy, dz, tri + 9 * (long long)B.ids[e])) return true;
            }
    return false;
}

// bin range of triangle t's bounding box; false for a non-finite triangle
__device__ inline bool tri_bins(const Bins& B, const double* __restrict__ v, int (&lo)[3], int (&hi)[3]) {
    const double o[3] = {B.ox, B.oy, B.oz};
    const int nb[3] = {B.nbx, B.nby, B.nbz};
    for (int a = 0; a < 3; ++a) {
        const double c0 = v[a], c1 = v[3 + a], c2 = v[6 + a];
        if (!(c0 - c0 == 0.0 && c1 - c1 == 0.0 && c2 - c2 == 0.0)) return false;
        lo[a] = bin_of(fmin(c0, fmin(c1, c2)), o[a], B.bdx, nb[a]);
        hi[a] = bin_of(fmax(c0, fmax(c1, c2)), o[a], B.bdx, nb[a]);
    }
    return true;
}

// One wavefront per triangle: its lanes walk the triangle's bin range together (a plate
// triangle can span thousands of bins; one thread per triangle serialised those).
__global__ void __launch_bounds__(NT) k_bin_count(Bins B, const double* __restrict__ tri, long long ntri,
                                                  long long* __restrict__ count) {
    const int lane = threadIdx.x & 63;
    const long long waves = (long long)gridDim.x * (NT / 64);
    for (long long t = (long long)blockIdx.x * (NT / 64) + (threadIdx.x >> 6); t < ntri; t += waves) {
        int lo[3], hi[3];
        if (!tri_bins(B, tri + 9 * t, lo, hi)) continue;
        const long long ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1;
        const long long nbt = ex * ey * (hi[2] - lo[2] + 1);
        for (long long e = lane; e < nbt; e += 64) {
            const int bx = lo[0] + (int)(e % ex), by = lo[1] + (int)((e / ex) % ey), bz = lo[2] + (int)(e / (ex * ey));
            atomicAdd((unsigned long long*)&count[bx + (long long)B.nbx * (by + (long long)B.nby * bz)], 1ULL);
        }
    }
}

__global__ void __launch_bounds__(NT) k_bin_fill(Bins B, const double* __restrict__ tri, long long ntri,
                                                 long long* __restrict__ cursor, int* __restrict__ ids) {
    const int lane = threadIdx.x & 63;
    const long long waves = (long long)gridDim.x * (NT / 64);
    for (long long t = (long long)blockIdx.x * (NT / 64) + (threadIdx.x >> 6); t < ntri; t += waves) {
        int lo[3], hi[3];
        if (!tri_bins(B, tri + 9 * t, lo, hi)) continue;
        const long long ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1;
        const long long nbt = ex * ey * (hi[2] - lo[2] + 1);
        for (long long e = lane; e < nbt; e += 64) {
            const int bx = lo[0] + (int)(e % ex), by = lo[1] + (int)((e / ex) % ey), bz = lo[2] + (int)(e / (ex * ey));
            const long long b = bx + (long long)B.nbx * (by + (long long)B.nby * bz);
            const long long pos = (long long)atomicAdd((unsigned long long*)&cursor[b], 1ULL);
            ids[B.off[b] + pos] = (int)t;
        }
    }
}

__global__ void k_fill_ll(long long* __restrict__ a, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = 0;
}

// Filter flag of every (triangle, vertex, dual-cell corner) in the corner order of
// k_shepard (a + 2 b + 4 c): whether the segment from the vertex to that cell centre
// crosses a triangle.  One thread per flag, so the long candidate loops spread over 24
// threads per triangle; k_shepard decides everything else as without the filter.
__global__ void __launch_bounds__(NT) k_occlude(Geo g, const double* __restrict__ tri, long long ntri, Bins B,
                                                uint8_t* __restrict__ occ) {
    for (long long w = (long long)blockIdx.x * NT + threadIdx.x; w < 24 * ntri; w += (long long)gridDim.x * NT) {
        const long long t = w / 24;
        const int r = (int)(w - 24 * t), q = r >> 3, corner = r & 7;
        const double* v = tri + 9 * t + 3 * q;
        const double X = v[0], Y = v[1], Z = v[2];
        uint8_t hit = 0;
        const double fi = floor((X - g.ox) / g.dx - 0.5), fj = floor((Y - g.oy) / g.dx - 0.5),
                     fk = floor((Z - g.oz) / g.dx - 0.5);
        if (fi >= -2.0 && fi <= g.nx + 1.0 && fj >= -2.0 && fj <= g.ny + 1.0 && fk >= -2.0 && fk <= g.nz + 1.0) {
            const long long i = (long long)fi + (corner & 1), j = (long long)fj + ((corner >> 1) & 1),
                            k = (long long)fk + (corner >> 2);
            if (i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz) {
                const double xc = g.ox + ((double)i + 0.5) * g.dx;
                const double yc = g.oy + ((double)j + 0.5) * g.dx;
                const double zc = g.oz + ((double)k + 0.5) * g.dx;
                hit = occluded(B, tri, X, Y, Z, xc, yc, zc) ? 1 : 0;
            }
        }
        occ[w] = hit;
    }
}

__global__ void __launch_bounds__(NT) k_shepard(Geo g, const double* __restrict__ tri, long long ntri,
                                                const double* __restrict__ p, double* __restrict__ side,
                                                double* __restrict__ part, const uint8_t* __restrict__ occ,
                                                int filter) {
    __shared__ double sh[3 * (NT / 64)];
    double f[3] = {0.0, 0.0, 0.0};
    const long long cells_x = g.nx, cells_xy = (long long)g.nx * g.ny;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < ntri; t += (long long)gridDim.x * NT) {
        const double* v = tri + 9 * t;
        const double e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
        const double e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
        const double cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
        const double two_a = sqrt(cx * cx + cy * cy + cz * cz);
        double pf = NAN, pb = NAN;
        if (two_a > 0.0 && two_a <= DBL_MAX) {   // not degenerate, overflowing or non-finite
            const double nxv = cx / two_a, nyv = cy / two_a, nzv = cz / two_a;
            double sf = 0.0, sb = 0.0;
            int cf = 0, cb = 0;
            for (int q = 0; q < 3; ++q) {
                const double X = v[3 * q], Y = v[3 * q + 1], Z = v[3 * q + 2];
                const double fi = floor((X - g.ox) / g.dx - 0.5), fj = floor((Y - g.oy) / g.dx - 0.5),
                             fk = floor((Z - g.oz) / g.dx - 0.5);
                // a vertex whose dual cell lies wholly outside the grid (or a non-finite
                // coordinate) has no points on either side
                if (!(fi >= -2.0 && fi <= g.nx + 1.0 && fj >= -2.0 && fj <= g.ny + 1.0 && fk >= -2.0 &&
                      fk <= g.nz + 1.0))
                    continue;
                const long long i0 = (long long)fi, j0 = (long long)fj, k0 = (long long)fk;
                double num[2] = {0.0, 0.0}, den[2] = {0.0, 0.0};
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            const long long i = i0 + a, j = j0 + b, k = k0 + c;
                            if (i < 0 || i >= g.nx || j < 0 || j >= g.ny || k < 0 || k >= g.nz) continue;
                            const double xc = g.ox + ((double)i + 0.5) * g.dx;
                            const double yc = g.oy + ((double)j + 0.5) * g.dx;
                            const double zc = g.oz + ((double)k + 0.5) * g.dx;
                            const double rx = xc - X, ry = yc - Y, rz = zc - Z;
                            const double s = nxv * rx + nyv * ry + nzv * rz;
                            if (s == 0.0) continue;
                            if (filter && occ[24 * t + 8 * q + (a + 2 * b + 4 * c)]) continue;
                            const int sd = s > 0.0 ? 0 : 1;
                            const double d2 = rx * rx + ry * ry + rz * rz;
                            num[sd] += p[i + cells_x * j + cells_xy * k] / d2;
                            den[sd] += 1.0 / d2;
                        }
                if (den[0] > 0.0) { sf += num[0] / den[0]; ++cf; }
                if (den[1] > 0.0) { sb += num[1] / den[1]; ++cb; }
            }
            if (cf) pf = sf / cf;
            if (cb) pb = sb / cb;
            const double area = 0.5 * two_a;
            const double dp = (cb ? pb : 0.0) - (cf ? pf : 0.0);
            f[0] += (area * nxv) * dp;
            f[1] += (area * nyv) * dp;
            f[2] += (area * nzv) * dp;
        }
        if (side) {
            side[2 * t] = pf;
            side[2 * t + 1] = pb;
        }
    }
    block_reduce<3>(f, sh);
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) part[a * MAX_BLOCKS + blockIdx.x] = f[a];
}

__global__ void __launch_bounds__(NT) k_sum3(const double* __restrict__ part, int nparts, double* __restrict__ out) {
    __shared__ double sh[3 * (NT / 64)];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += NT)
        for (int a = 0; a < 3; ++a) v[a] += part[a * MAX_BLOCKS + b];
    block_reduce<3>(v, sh);
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) out[a] = v[a];
}

}  // namespace

// grow-only device buffer
template <class P>
static int grow(P** buf, long long* cap, long long need) {
    if (need <= *cap) return IBM_OK;
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (ibm::dev_malloc((void**)buf, sizeof(P) * (size_t)(need > 1 ? need : 1)) != hipSuccess) {
        (void)hipGetLastError();
        *buf = nullptr;
        set_error("near-field force: out of device memory for the triangle bins");
        return IBM_ERR_OOM;
    }
    *cap = need;
    return IBM_OK;
}

int shepard_run(ibm_ctx* c, const double* tri, long long ntri, const double* p, int filter, double* side,
                double* force, hipStream_t s) {
    for (int a = 0; a < 3; ++a) force[a] = 0.0;
    if (ntri == 0) return IBM_OK;
    const Geo& g = c->geo;
    const long long nbk = (ntri + NT - 1) / NT;
    const int nb = (int)(nbk < 2048 ? nbk : 2048);
    Bins B{};
    uint8_t* occ = nullptr;
    if (filter) {
        B.nbx = (g.nx + BIN_CELLS - 1) / BIN_CELLS;
        B.nby = (g.ny + BIN_CELLS - 1) / BIN_CELLS;
        B.nbz = (g.nz + BIN_CELLS - 1) / BIN_CELLS;
        B.bdx = BIN_CELLS * g.dx;
        B.ox = g.ox;
        B.oy = g.oy;
        B.oz = g.oz;
        const long long nbins = (long long)B.nbx * B.nby * B.nbz;
        if (int rc = grow(&c->bin_count, &c->bin_cap, 2 * (nbins + 1))) return rc;
        if (int rc = grow(&c->bin_occ, &c->bin_occ_cap, 24 * ntri)) return rc;
        long long* count = c->bin_count;
        long long* off = c->bin_count + (nbins + 1);
        const long long nbw = (ntri + NT / 64 - 1) / (NT / 64);   // one wavefront per triangle
        const int nbb = (int)(nbw < 8192 ? nbw : 8192);
        k_fill_ll<<<1024, 256, 0, s>>>(count, nbins + 1);
        k_bin_count<<<nbb, NT, 0, s>>>(B, tri, ntri, count);
        size_t tmp_bytes = 0;
        IBM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, count, off, (int)(nbins + 1), s));
        if (int rc = grow(&c->bin_tmp, &c->bin_tmp_cap, (long long)tmp_bytes)) return rc;
        IBM_HIP(hipcub::DeviceScan::ExclusiveSum(c->bin_tmp, tmp_bytes, count, off, (int)(nbins + 1), s));
        long long total = 0;
        IBM_HIP(hipMemcpyAsync(&total, off + nbins, sizeof(long long), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (total >= 0x7fffffffLL) {
            set_error("near-field force: too many triangle-bin entries for the thin-plate filter");
            return IBM_ERR_ARG;
        }
        if (int rc = grow(&c->bin_ids, &c->bin_ids_cap, total)) return rc;
        k_fill_ll<<<1024, 256, 0, s>>>(count, nbins + 1);   // reused as the fill cursor
        B.off = off;
        B.ids = c->bin_ids;
        k_bin_fill<<<nbb, NT, 0, s>>>(B, tri, ntri, count, c->bin_ids);
        const long long nbo = (24 * ntri + NT - 1) / NT;
        k_occlude<<<(int)(nbo < 16384 ? nbo : 16384), NT, 0, s>>>(c->geo, tri, ntri, B, c->bin_occ);
        occ = c->bin_occ;
        IBM_HIP(hipGetLastError());
    }
    if (c->timing_on)
        launch_timed(c, TK_OTHER, k_shepard, nb, s, c->geo, tri, ntri, p, side, c->partials, (const uint8_t*)occ,
                     filter);
    else
        k_shepard<<<nb, NT, 0, s>>>(c->geo, tri, ntri, p, side, c->partials, occ, filter);
    k_sum3<<<1, NT, 0, s>>>(c->partials, nb, c->red);
    IBM_HIP(hipGetLastError());
    IBM_HIP(hipMemcpyAsync(c->h_red, c->red, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    for (int a = 0; a < 3; ++a) force[a] = c->h_red[a];
    return IBM_OK;
}

void shepard_release(ibm_ctx* c) {
    if (c->bin_count) (void)hipFree(c->bin_count);
    if (c->bin_ids) (void)hipFree(c->bin_ids);
    if (c->bin_occ) (void)hipFree(c->bin_occ);
    if (c->bin_tmp) (void)hipFree(c->bin_tmp);
    c->bin_count = nullptr;
    c->bin_ids = nullptr;
    c->bin_occ = nullptr;
    c->bin_tmp = nullptr;
    c->bin_cap = c->bin_ids_cap = c->bin_occ_cap = c->bin_tmp_cap = 0;
}

}  // namespace ibm
