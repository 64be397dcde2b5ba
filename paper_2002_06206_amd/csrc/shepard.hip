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

#include <cfloat>
#include <cmath>

#include "common.h"

namespace ibm {
namespace {

__global__ void __launch_bounds__(NT) k_shepard(Geo g, const double* __restrict__ tri, long long ntri,
                                                const double* __restrict__ p, double* __restrict__ side,
                                                double* __restrict__ part) {
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
                            const double rx = (g.ox + ((double)i + 0.5) * g.dx) - X;
                            const double ry = (g.oy + ((double)j + 0.5) * g.dx) - Y;
                            const double rz = (g.oz + ((double)k + 0.5) * g.dx) - Z;
                            const double s = nxv * rx + nyv * ry + nzv * rz;
                            if (s == 0.0) continue;
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

int shepard_run(ibm_ctx* c, const double* tri, long long ntri, const double* p, double* side, double* force,
                hipStream_t s) {
    for (int a = 0; a < 3; ++a) force[a] = 0.0;
    if (ntri == 0) return IBM_OK;
    const long long nbk = (ntri + NT - 1) / NT;
    const int nb = (int)(nbk < 2048 ? nbk : 2048);
    if (c->timing_on)
        launch_timed(c, TK_OTHER, k_shepard, nb, s, c->geo, tri, ntri, p, side, c->partials);
    else
        k_shepard<<<nb, NT, 0, s>>>(c->geo, tri, ntri, p, side, c->partials);
    k_sum3<<<1, NT, 0, s>>>(c->partials, nb, c->red);
    IBM_HIP(hipGetLastError());
    IBM_HIP(hipMemcpyAsync(c->h_red, c->red, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    for (int a = 0; a < 3; ++a) force[a] = c->h_red[a];
    return IBM_OK;
}

}  // namespace ibm
