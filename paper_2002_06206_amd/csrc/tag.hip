// Fluid/ghost tagging of a triangle soup (Sec. 2.3.1): every closed segment between
// face-adjacent cell centres that meets a closed triangle is blocked for both cells,
// with theta = (distance from the own centre to the nearest crossing)/dx.
//
// Work decomposition: the soup is rasterised along each axis.  For (triangle, axis)
// the grid lines parallel to the axis whose (u,v) position falls in the triangle's
// projected bounding box are candidates; candidates are flattened by a prefix sum so
// one thread takes one (triangle, axis, line) no matter how large the triangle is.
// A thread decides with exact signs whether its line pierces the closed projected
// triangle, then finds the crossed segment by bisection on the exact sign of
// (x* - x_i), where x* is the crossing coordinate on the line.
//
// Exact signs: a double evaluation with a conservative forward error bound decides
// almost always; otherwise the determinant is re-evaluated exactly with
// floating-point expansions (error-free two-sum / two-product, Shewchuk 1997).
// Inputs are validated to magnitudes 0 or [2^-200, 2^200] so no product underflows.
//
// This file is compiled with -ffp-contract=off: theta must follow one fixed double
// formula bit for bit.

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace ibm {
namespace {

// ----------------------------------------------------------- expansions

__device__ inline void two_sum(double a, double b, double& x, double& y) {
    x = a + b;
    double bv = x - a;
    double av = x - bv;
    double br = b - bv;
    double ar = a - av;
    y = ar + br;
}

__device__ inline void two_diff(double a, double b, double& x, double& y) {
    x = a - b;
    double bv = a - x;
    double av = x + bv;
    double br = bv - b;
    double ar = a - av;
    y = ar + br;
}

__device__ inline void two_prod(double a, double b, double& x, double& y) {
    x = a * b;
    y = fma(a, b, -x);
}

// h = e + b (e nonoverlapping, increasing magnitude); zero components dropped.
__device__ inline int grow_expansion(int elen, const double* e, double b, double* h) {
    double q = b;
    int hn = 0;
    for (int i = 0; i < elen; ++i) {
        double qn, hh;
        two_sum(q, e[i], qn, hh);
        q = qn;
        if (hh != 0.0) h[hn++] = hh;
    }
    if (q != 0.0 || hn == 0) h[hn++] = q;
    return hn;
}

// h = e + f, by growing e with each component of f.  h must hold elen+flen terms
// and may not alias e or f; tmp is scratch of the same size.
__device__ inline int expansion_sum(int elen, const double* e, int flen, const double* f, double* h,
                                    double* tmp) {
    int n = elen;
    for (int i = 0; i < elen; ++i) h[i] = e[i];
    for (int j = 0; j < flen; ++j) {
        n = grow_expansion(n, h, f[j], tmp);
        for (int i = 0; i < n; ++i) h[i] = tmp[i];
    }
    return n;
}

// h = b * e.  h must hold 2*elen terms.
__device__ inline int scale_expansion(int elen, const double* e, double b, double* h) {
    double q, hh;
    int hn = 0;
    two_prod(e[0], b, q, hh);
    if (hh != 0.0) h[hn++] = hh;
    for (int i = 1; i < elen; ++i) {
        double t1, t0, s1, s0;
        two_prod(e[i], b, t1, t0);
        two_sum(q, t0, s1, s0);
        if (s0 != 0.0) h[hn++] = s0;
        two_sum(t1, s1, q, hh);
        if (hh != 0.0) h[hn++] = hh;
    }
    if (q != 0.0 || hn == 0) h[hn++] = q;
    return hn;
}

__device__ inline int expansion_sign(int n, const double* e) {
    double top = e[n - 1];
    return (top > 0.0) - (top < 0.0);
}

// Exact product of two 2-term expansions (a1 + a0)(b1 + b0) -> up to 8 terms.
__device__ inline int mul22(const double* a, const double* b, double* h) {
    double s0[4], s1[4], tmp[8];
    int n0 = scale_expansion(2, b, a[0], s0);
    int n1 = scale_expansion(2, b, a[1], s1);
    return expansion_sum(n0, s0, n1, s1, h, tmp);
}

// Exact expansion of (au-pu)(bv-pv) - (av-pv)(bu-pu): up to 16 terms.
__device__ inline int orient2d_exp(double pu, double pv, double au, double av, double bu, double bv,
                                   double* h) {
    double d1[2], d2[2], d3[2], d4[2];
    two_diff(au, pu, d1[1], d1[0]);
    two_diff(bv, pv, d2[1], d2[0]);
    two_diff(av, pv, d3[1], d3[0]);
    two_diff(bu, pu, d4[1], d4[0]);
    double t1[8], t2[8], tmp[16];
    int n1 = mul22(d1, d2, t1);
    int n2 = mul22(d3, d4, t2);
    for (int i = 0; i < n2; ++i) t2[i] = -t2[i];
    return expansion_sum(n1, t1, n2, t2, h, tmp);
}

// Sign of twice the signed area of (p, a, b).
__device__ inline int orient2d_sign(double pu, double pv, double au, double av, double bu, double bv) {
    double t1 = (au - pu) * (bv - pv);
    double t2 = (av - pv) * (bu - pu);
    double det = t1 - t2;
    double bound = 1e-14 * (fabs(t1) + fabs(t2));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    double h[16];
    int n = orient2d_exp(pu, pv, au, av, bu, bv, h);
    return expansion_sign(n, h);
}

struct Tri {
    double a[3], b[3], c[3];
};

// Sign of sum_m w_m (m_k - t) = W (x* - t): w_a = area(p,b,c), w_b = area(p,c,a),
// w_c = area(p,a,b) in the (u,v) projection.
__device__ int crossing_sign(double pu, double pv, double t, const Tri& T, int u, int v, int k) {
    const double* A = T.a;
    const double* B = T.b;
    const double* C = T.c;
    double wa1 = (B[u] - pu) * (C[v] - pv), wa2 = (B[v] - pv) * (C[u] - pu);
    double wb1 = (C[u] - pu) * (A[v] - pv), wb2 = (C[v] - pv) * (A[u] - pu);
    double wc1 = (A[u] - pu) * (B[v] - pv), wc2 = (A[v] - pv) * (B[u] - pu);
    double ea = A[k] - t, eb = B[k] - t, ec = C[k] - t;
    double det = (wa1 - wa2) * ea + (wb1 - wb2) * eb + (wc1 - wc2) * ec;
    double P = (fabs(wa1) + fabs(wa2)) * fabs(ea) + (fabs(wb1) + fabs(wb2)) * fabs(eb) +
               (fabs(wc1) + fabs(wc2)) * fabs(ec);
    double bound = 1e-13 * P;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    // exact: three 16-term areas times 2-term differences, summed
    double w[16], dk[2], s1[32], s2[32], prod[64], acc[192], acc2[192], tmp[192];
    int nacc = 0;
    const double* V[3] = {A, B, C};
    for (int m = 0; m < 3; ++m) {
        const double* P1 = V[(m + 1) % 3];
        const double* P2 = V[(m + 2) % 3];
        int nw = orient2d_exp(pu, pv, P1[u], P1[v], P2[u], P2[v], w);
        two_diff(V[m][k], t, dk[1], dk[0]);
        int n1 = scale_expansion(nw, w, dk[0], s1);
        int n2 = scale_expansion(nw, w, dk[1], s2);
        int np = expansion_sum(n1, s1, n2, s2, prod, tmp);
        if (nacc == 0) {
            for (int i = 0; i < np; ++i) acc[i] = prod[i];
            nacc = np;
        } else {
            nacc = expansion_sum(nacc, acc, np, prod, acc2, tmp);
            for (int i = 0; i < nacc; ++i) acc[i] = acc2[i];
        }
    }
    return expansion_sign(nacc, acc);
}

__device__ inline double centre(double o, double dx, long long i) {
    return o + ((double)i + 0.5) * dx;
}

// floor/ceil of a line coordinate, clamped in double before the integer cast
__device__ inline long long lfloor(double v, long long lo, long long hi) {
    double f = floor(v);
    f = fmax(f, (double)lo);
    f = fmin(f, (double)hi);
    return (long long)f;
}

__device__ inline bool coord_ok(double x) {
    double a = fabs(x);
    return a == 0.0 || (a >= 0x1p-200 && a <= 0x1p200);
}

struct TagArgs {
    const double* tri;
    long long ntri;
    int n[3];
    double dx;
    double o[3];
    double eps;          // bary_eps: tolerance of the ray / triangle test (0 = exact)
};

// Bounding box of a triangle along axis x, grown so that it holds the triangle grown by
// eps in barycentric terms (its corners are a + eps (2a - b - c) and the like, at most
// 2 eps times the extent beyond the box).
__device__ inline void grown_range(const double* p, int x, double eps, double& lo, double& hi) {
    lo = fmin(p[x], fmin(p[3 + x], p[6 + x]));
    hi = fmax(p[x], fmax(p[3 + x], p[6 + x]));
    const double gr = 2.0 * eps * (hi - lo);
    lo -= gr;
    hi += gr;
}

// Candidate-line count per (triangle, axis).
__global__ void k_count(TagArgs a, unsigned long long* cnt, int* bad) {
    long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id == a.ntri * 3) cnt[id] = 0;
    if (id >= a.ntri * 3) return;
    long long t = id / 3;
    int k = (int)(id % 3);
    const double* p = a.tri + 9 * t;
    bool ok = true;
    for (int q = 0; q < 9; ++q) ok = ok && coord_ok(p[q]);
    if (!ok) {
        atomicOr(bad, 1);
        cnt[id] = 0;
        return;
    }
    int u = (k + 1) % 3, v = (k + 2) % 3;
    double umin, umax, vmin, vmax;
    grown_range(p, u, a.eps, umin, umax);
    grown_range(p, v, a.eps, vmin, vmax);
    long long j0 = lfloor((umin - a.o[u]) / a.dx - 0.5 - 1.0, 0, a.n[u]);
    long long j1 = lfloor(ceil((umax - a.o[u]) / a.dx - 0.5) + 1.0, -1, a.n[u] - 1);
    long long l0 = lfloor((vmin - a.o[v]) / a.dx - 0.5 - 1.0, 0, a.n[v]);
    long long l1 = lfloor(ceil((vmax - a.o[v]) / a.dx - 0.5) + 1.0, -1, a.n[v] - 1);
    // a segment exists along k only when n[k] >= 2
    if (j1 < j0 || l1 < l0 || a.n[k] < 2) {
        cnt[id] = 0;
        return;
    }
    cnt[id] = (unsigned long long)((j1 - j0 + 1) * (l1 - l0 + 1));
}

// One thread per candidate (triangle, axis, line).  Pass 1 (list == null) sets the
// blocked bits of both cells of every crossed segment; pass 2 (the mask complete and
// coff its exclusive popcount prefix) keeps the nearest crossing of each blocked
// (cell, dir) in the compact list by an atomic minimum on the bits of the non-negative
// theta.  Both passes take the same decisions.
__global__ void k_lines(TagArgs a, const unsigned long long* off, unsigned long long total, uint32_t* maskw,
                        const uint32_t* coff, unsigned long long* list) {
    const long long ntk = a.ntri * 3;
    for (unsigned long long q = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (unsigned long long)gridDim.x * blockDim.x) {
        // (triangle, axis) owning candidate q: last tk with off[tk] <= q
        long long lo = 0, hi = ntk - 1;
        while (lo < hi) {
            long long mid = (lo + hi + 1) >> 1;
            if (off[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const long long tk = lo;
        const long long t = tk / 3;
        const int k = (int)(tk % 3);
        const int u = (k + 1) % 3, v = (k + 2) % 3;
        Tri T;
        const double* p = a.tri + 9 * t;
        for (int x = 0; x < 3; ++x) {
            T.a[x] = p[x];
            T.b[x] = p[3 + x];
            T.c[x] = p[6 + x];
        }
        double umin, umax, vmin, vmax, kmin, kmax;
        grown_range(p, u, a.eps, umin, umax);
        grown_range(p, v, a.eps, vmin, vmax);
        grown_range(p, k, a.eps, kmin, kmax);
        (void)umax;
        long long j0 = lfloor((umin - a.o[u]) / a.dx - 0.5 - 1.0, 0, a.n[u]);
        long long l0 = lfloor((vmin - a.o[v]) / a.dx - 0.5 - 1.0, 0, a.n[v]);
        long long l1 = lfloor(ceil((vmax - a.o[v]) / a.dx - 0.5) + 1.0, -1, a.n[v] - 1);
        const long long nl = l1 - l0 + 1;
        const long long local = (long long)(q - off[tk]);
        const long long j = j0 + local / nl;
        const long long l = l0 + local % nl;
        const double pu = centre(a.o[u], a.dx, j), pv = centre(a.o[v], a.dx, l);

        int sa = orient2d_sign(pu, pv, T.b[u], T.b[v], T.c[u], T.c[v]);
        int sb = orient2d_sign(pu, pv, T.c[u], T.c[v], T.a[u], T.a[v]);
        int sc = orient2d_sign(pu, pv, T.a[u], T.a[v], T.b[u], T.b[v]);
        int sW;
        if (sa >= 0 && sb >= 0 && sc >= 0 && sa + sb + sc > 0) sW = 1;
        else if (sa <= 0 && sb <= 0 && sc <= 0 && sa + sb + sc < 0) sW = -1;
        else sW = 0;

        // double crossing coordinate, fixed operation order
        double dau = T.a[u] - pu, dav = T.a[v] - pv;
        double dbu = T.b[u] - pu, dbv = T.b[v] - pv;
        double dcu = T.c[u] - pu, dcv = T.c[v] - pv;
        double wa = dbu * dcv - dbv * dcu;
        double wb = dcu * dav - dcv * dau;
        double wc = dau * dbv - dav * dbu;
        double num = (wa * T.a[k] + wb * T.b[k]) + wc * T.c[k];
        double den = (wa + wb) + wc;
        if (sW == 0) {
            // missed exactly: a hit only within the tolerance, each sub-triangle area
            // (with the exact orientation sign of the projected triangle) at least
            // -eps |w_a + w_b + w_c|
            if (!(a.eps > 0.0)) continue;
            const int sT = orient2d_sign(T.a[u], T.a[v], T.b[u], T.b[v], T.c[u], T.c[v]);
            if (sT == 0) continue;
            const double st = (double)sT, lim = -a.eps * fabs(den);
            if (!(wa * st >= lim && wb * st >= lim && wc * st >= lim)) continue;
            sW = sT;
        }
        double xs = num / den;

        // first centre index along k with x_i > x* (exact), bisection over a bracket
        const int nk = a.n[k];
        long long ilo = lfloor((kmin - a.o[k]) / a.dx - 0.5 - 1.0, 0, nk);
        long long ihi = lfloor(ceil((kmax - a.o[k]) / a.dx - 0.5) + 1.0, -1, nk - 1);
        if (ihi < ilo) continue;
        long long b0 = ilo, b1 = ihi + 1;
        while (b0 < b1) {
            long long mid = (b0 + b1) >> 1;
            int sg = crossing_sign(pu, pv, centre(a.o[k], a.dx, mid), T, u, v, k) * sW;
            if (sg < 0) b1 = mid; else b0 = mid + 1;
        }
        const long long ifirst = b0;
        for (long long sidx = ifirst - 2; sidx <= ifirst - 1; ++sidx) {
            if (sidx < 0 || sidx + 1 > nk - 1) continue;
            const double xa = centre(a.o[k], a.dx, sidx), xb = centre(a.o[k], a.dx, sidx + 1);
            int s_lo = crossing_sign(pu, pv, xa, T, u, v, k) * sW;
            int s_hi = crossing_sign(pu, pv, xb, T, u, v, k) * sW;
            if (s_lo < 0 || s_hi > 0) continue;
            double tl = (xs - xa) / a.dx, th = (xb - xs) / a.dx;
            if (tl < 0.0) tl = 0.0;
            if (tl > 1.0) tl = 1.0;
            if (th < 0.0) th = 0.0;
            if (th > 1.0) th = 1.0;
            long long idx[3];
            idx[k] = sidx;
            idx[u] = j;
            idx[v] = l;
            long long ca = idx[0] + (long long)a.n[0] * (idx[1] + (long long)a.n[1] * idx[2]);
            idx[k] = sidx + 1;
            long long cb = idx[0] + (long long)a.n[0] * (idx[1] + (long long)a.n[1] * idx[2]);
            int da = 2 * k + 1, db = 2 * k;
            if (!list) {
                atomicOr(&maskw[ca >> 2], (1u << da) << (8 * (ca & 3)));
                atomicOr(&maskw[cb >> 2], (1u << db) << (8 * (cb & 3)));
            } else {
                const uint8_t* mb = reinterpret_cast<const uint8_t*>(maskw);
                const uint32_t ia = coff[ca] + (uint32_t)__builtin_popcount((unsigned)mb[ca] & ((1u << da) - 1u));
                const uint32_t ib = coff[cb] + (uint32_t)__builtin_popcount((unsigned)mb[cb] & ((1u << db) - 1u));
                atomicMin(&list[ia], (unsigned long long)__double_as_longlong(tl));
                atomicMin(&list[ib], (unsigned long long)__double_as_longlong(th));
            }
        }
    }
}

__global__ void k_fill_u32(uint32_t* p, long long n, uint32_t v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, long long n, unsigned long long v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int* p, long long n, int v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

struct PopcountByte {
    __host__ __device__ uint32_t operator()(uint8_t m) const { return (uint32_t)__builtin_popcount((unsigned)m); }
};

// number of list entries: last offset + popcount of the last cell
__global__ void k_list_total(const uint32_t* coff, const uint8_t* mask, long long N, unsigned long long* out) {
    *out = (unsigned long long)coff[N - 1] + (unsigned long long)__builtin_popcount((unsigned)mask[N - 1]);
}

// dense theta (cells x 6, 2.0 where open) from the compact list
__global__ void k_expand(long long N, ThetaSrc t, double* theta) {
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x)
        for (int d = 0; d < 6; ++d) theta[6 * c + d] = theta_of(t, c, d);
}

__global__ void k_differs(long long N, const uint8_t* a, const uint8_t* b, int* flag) {
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x)
        if (a[c] != b[c]) *flag = 1;
}

}  // namespace

// Tagging into the context: pass 1 sets the blocked bits, an exclusive scan of their
// popcounts gives each cell's first entry of the compact theta list, pass 2 fills the
// list with the nearest crossings.  Memory: one byte and one 32-bit offset per cell and
// 8 bytes per blocked (cell, dir), instead of 48 bytes per cell for a dense theta.
int tag_run(ibm_ctx* c, const double* tri, long long ntri, double bary_eps, hipStream_t s) {
    const long long N = c->N;
    const long long nw = (N + 3) / 4;
    k_fill_u32<<<2048, 256, 0, s>>>(c->tagmask, nw, 0u);
    IBM_HIP(hipGetLastError());
    c->tagged = false;
    c->tag_ncut = 0;
    TagArgs a;
    a.tri = tri;
    a.ntri = ntri;
    a.n[0] = c->geo.nx;
    a.n[1] = c->geo.ny;
    a.n[2] = c->geo.nz;
    a.dx = c->geo.dx;
    a.o[0] = c->geo.ox;
    a.o[1] = c->geo.oy;
    a.o[2] = c->geo.oz;
    a.eps = bary_eps;
    const long long ntk = ntri * 3;
    unsigned long long *cnt = nullptr, *off = nullptr, *dtotal = nullptr;
    int* bad = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    unsigned long long total = 0;
    int rc = IBM_OK;
    if (ntri > 0) {
        IBM_HIP(ibm::dev_malloc_async((void**)&cnt, sizeof(unsigned long long) * (ntk + 1), s));
        IBM_HIP(ibm::dev_malloc_async((void**)&off, sizeof(unsigned long long) * (ntk + 1), s));
        IBM_HIP(ibm::dev_malloc_async((void**)&bad, sizeof(int), s));
        k_fill_i32<<<1, 1, 0, s>>>(bad, 1, 0);
        // cnt[ntk] = 0, so the exclusive scan over ntk+1 entries ends with the total
        k_count<<<(unsigned)((ntk + 1 + 255) / 256), 256, 0, s>>>(a, cnt, bad);
        IBM_HIP(hipGetLastError());
        IBM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, off, (int)(ntk + 1), s));
        IBM_HIP(ibm::dev_malloc_async(&tmp, tmp_bytes, s));
        IBM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, off, (int)(ntk + 1), s));
        int hbad = 0;
        IBM_HIP(hipMemcpyAsync(&total, off + ntk, sizeof(total), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        IBM_HIP(hipFreeAsync(tmp, s));
        tmp = nullptr;
        if (hbad) {
            set_error("ibm_tag_geometry: triangle coordinates must be finite with magnitude 0 or in [2^-200, 2^200]");
            rc = IBM_ERR_ARG;
        }
    }
    unsigned blocks = (unsigned)((total + 255) / 256);
    if (blocks > 65536u * 4u) blocks = 65536u * 4u;
    if (rc == IBM_OK && total > 0) {
        k_lines<<<blocks, 256, 0, s>>>(a, off, total, c->tagmask, nullptr, nullptr);
        IBM_HIP(hipGetLastError());
    }
    // offsets of the compact list
    unsigned long long nlist = 0;
    if (rc == IBM_OK) {
        const uint8_t* mb = reinterpret_cast<const uint8_t*>(c->tagmask);
        hipcub::TransformInputIterator<uint32_t, PopcountByte, const uint8_t*> it(mb, PopcountByte());
        size_t bytes = 0;
        IBM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, it, c->tag_off, (int)N, s));
        IBM_HIP(ibm::dev_malloc_async(&tmp, bytes, s));
        IBM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, it, c->tag_off, (int)N, s));
        IBM_HIP(ibm::dev_malloc_async((void**)&dtotal, sizeof(unsigned long long), s));
        k_list_total<<<1, 1, 0, s>>>(c->tag_off, mb, N, dtotal);
        IBM_HIP(hipGetLastError());
        IBM_HIP(hipMemcpyAsync(&nlist, dtotal, sizeof(nlist), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        IBM_HIP(hipFreeAsync(tmp, s));
        IBM_HIP(hipFreeAsync(dtotal, s));
        // the per-cell offsets are 32-bit and a scan of N popcounts is exact below 2^32
        if (nlist >= 0xFFFFFFFFull) {
            set_error("ibm_tag_geometry: more than 2^32-1 blocked (cell, direction) pairs");
            rc = IBM_ERR_ARG;
        }
    }
    if (rc == IBM_OK && (long long)nlist > c->tag_cap) {
        if (c->tag_list) IBM_HIP(hipFree(c->tag_list));
        c->tag_list = nullptr;
        c->tag_cap = 0;
        const long long cap = (long long)nlist + (long long)nlist / 8 + 64;
        if (ibm::dev_malloc(&c->tag_list, sizeof(double) * (size_t)cap) != hipSuccess) {
            (void)hipGetLastError();
            set_error("ibm_tag_geometry: out of device memory for the theta list");
            rc = IBM_ERR_OOM;
        } else {
            c->tag_cap = cap;
        }
    }
    if (rc == IBM_OK && nlist > 0) {
        const unsigned long long two = 0x4000000000000000ull;   // bits of 2.0 (open)
        k_fill_u64<<<2048, 256, 0, s>>>((unsigned long long*)c->tag_list, (long long)nlist, two);
        k_lines<<<blocks, 256, 0, s>>>(a, off, total, c->tagmask, c->tag_off, (unsigned long long*)c->tag_list);
        IBM_HIP(hipGetLastError());
    }
    if (cnt) IBM_HIP(hipFreeAsync(cnt, s));
    if (off) IBM_HIP(hipFreeAsync(off, s));
    if (bad) IBM_HIP(hipFreeAsync(bad, s));
    if (rc == IBM_OK) {
        c->tag_ncut = (long long)nlist;
        c->tagged = true;
    }
    return rc;
}

int tag_expand(ibm_ctx* c, double* theta, hipStream_t s) {
    ThetaSrc t{nullptr, reinterpret_cast<const uint8_t*>(c->tagmask), c->tag_off, c->tag_list};
    k_expand<<<4096, 256, 0, s>>>(c->N, t, theta);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int tag_matches(ibm_ctx* c, const uint8_t* blocked, bool* same, hipStream_t s) {
    int* flag = (int*)c->counter + 9;   // spare slot of the ticket array
    k_fill_i32<<<1, 1, 0, s>>>(flag, 1, 0);
    k_differs<<<4096, 256, 0, s>>>(c->N, blocked, reinterpret_cast<const uint8_t*>(c->tagmask), flag);
    int h = 0;
    IBM_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    *same = h == 0;
    return IBM_OK;
}

void tag_release(ibm_ctx* c) {
    if (c->tagmask) (void)hipFree(c->tagmask);
    if (c->tag_off) (void)hipFree(c->tag_off);
    if (c->tag_list) (void)hipFree(c->tag_list);
    c->tagmask = nullptr;
    c->tag_off = nullptr;
    c->tag_list = nullptr;
    c->tag_cap = 0;
    c->tag_ncut = 0;
    c->tagged = false;
}

}  // namespace ibm
