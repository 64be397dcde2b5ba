/*
 * Oracle: fluid/ghost tagging of a triangle soup on a uniform Cartesian grid.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load this file.
 *
 * What it computes (Sec. 2.3.1, dummy-cell construction, and the ray test of
 * the same section): for every pair of face-adjacent cell centres, the closed
 * axis-parallel segment joining them is "blocked" when it meets some closed
 * triangle of the soup.  The neighbour behind such a crossing is a ghost cell
 * for that cell only.  No inside/outside decision is made anywhere.
 *
 * Reading: the paper's Moller-Trumbore test with a tuned determinant error is
 * replaced by exact signs.  Each sign is evaluated in exact integer arithmetic
 * (a plain schoolbook bignum, below), so edges and vertices count as part of
 * the triangle and a ray through a shared edge cannot slip between the two
 * triangles.  Triangles whose projection along the ray axis has zero area are
 * parallel to the ray and never block it.
 *
 * theta, the distance from the cell's own centre to its nearest crossing on
 * that segment divided by dx, is evaluated with one fixed double-precision
 * formula: the crossing coordinate is the barycentric combination of the
 * vertex coordinates with the plain double 2-D sub-triangle areas as weights,
 * then clamped to [0, 1].  Compile with -ffp-contract=off.
 *
 * Domain faces (including periodic wrap faces) are never tagged.
 *
 * bary_eps (>= 0, at most 0.5): the paper's tuned tolerance of the ray / triangle
 * test (Sec. 2.3.1: adjusting it keeps rays from slipping through gaps).  With
 * bary_eps > 0 a grid line also meets the triangle when it misses it by at most
 * bary_eps in barycentric terms: each plain double sub-triangle area w_m (the theta
 * weights above), taken with the exact orientation sign of the projected triangle,
 * is at least -bary_eps |w_a + w_b + w_c|.  The exact test alone decides at 0, so
 * the blocked set only grows with bary_eps.  The segment that is crossed is still
 * decided exactly.
 *
 * Cell index c = i + nx*(j + ny*k).  Direction bits 0..5 = -x,+x,-y,+y,-z,+z.
 * theta layout: theta[6*c + dir], 2.0 where the direction is open.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------- bignum --- */
/* Signed integer of up to NL 32-bit limbs, little-endian magnitude. */
#define NL 240

typedef struct {
    int sign; /* -1, 0, +1 */
    int n;    /* limbs in use */
    uint32_t d[NL];
} big;

static void big_zero(big *a) { a->sign = 0; a->n = 0; }

static void big_trim(big *a)
{
    while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
    if (a->n == 0) a->sign = 0;
}

/* |a| compared with |b| */
static int mag_cmp(const big *a, const big *b)
{
    if (a->n != b->n) return a->n < b->n ? -1 : 1;
    for (int i = a->n - 1; i >= 0; --i)
        if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
    return 0;
}

/* r = |a| + |b| (magnitudes only) */
static void mag_add(big *r, const big *a, const big *b)
{
    int n = a->n > b->n ? a->n : b->n;
    uint64_t carry = 0;
    for (int i = 0; i < n; ++i) {
        uint64_t s = carry;
        if (i < a->n) s += a->d[i];
        if (i < b->n) s += b->d[i];
        r->d[i] = (uint32_t)s;
        carry = s >> 32;
    }
    r->n = n;
    if (carry) { r->d[n] = (uint32_t)carry; r->n = n + 1; }
}

/* r = |a| - |b|, requires |a| >= |b| */
static void mag_sub(big *r, const big *a, const big *b)
{
    int64_t borrow = 0;
    for (int i = 0; i < a->n; ++i) {
        int64_t s = (int64_t)a->d[i] - borrow - (i < b->n ? (int64_t)b->d[i] : 0);
        if (s < 0) { s += ((int64_t)1 << 32); borrow = 1; } else borrow = 0;
        r->d[i] = (uint32_t)s;
    }
    r->n = a->n;
}

/* r = a + b (signed); r may alias neither */
static void big_add(big *r, const big *a, const big *b)
{
    if (a->sign == 0) { *r = *b; return; }
    if (b->sign == 0) { *r = *a; return; }
    if (a->sign == b->sign) {
        mag_add(r, a, b);
        r->sign = a->sign;
    } else {
        int c = mag_cmp(a, b);
        if (c == 0) { big_zero(r); return; }
        if (c > 0) { mag_sub(r, a, b); r->sign = a->sign; }
        else { mag_sub(r, b, a); r->sign = b->sign; }
    }
    big_trim(r);
}

static void big_neg(big *a) { a->sign = -a->sign; }

static void big_sub(big *r, const big *a, const big *b)
{
    big nb = *b;
    big_neg(&nb);
    big_add(r, a, &nb);
}

static void big_mul(big *r, const big *a, const big *b)
{
    if (a->sign == 0 || b->sign == 0) { big_zero(r); return; }
    int n = a->n + b->n;
    if (n > NL) abort(); /* cannot happen for finite doubles with NL = 240 */
    memset(r->d, 0, sizeof(uint32_t) * (size_t)n);
    for (int i = 0; i < a->n; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < b->n; ++j) {
            uint64_t t = (uint64_t)a->d[i] * b->d[j] + r->d[i + j] + carry;
            r->d[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        int k = i + b->n;
        while (carry) {
            uint64_t t = (uint64_t)r->d[k] + carry;
            r->d[k] = (uint32_t)t;
            carry = t >> 32;
            ++k;
        }
    }
    r->n = n;
    r->sign = a->sign * b->sign;
    big_trim(r);
}

/* Exponent of the last significant bit of a finite nonzero double x:
 * x = m * 2^e with m an odd integer. */
static int low_exp(double x)
{
    int ex;
    double f = frexp(fabs(x), &ex);      /* x = f * 2^ex, f in [0.5,1) */
    uint64_t m = (uint64_t)ldexp(f, 53); /* exact: 53-bit integer */
    int e = ex - 53;
    while ((m & 1u) == 0) { m >>= 1; ++e; }
    return e;
}

/* a = x / 2^E exactly, where E <= low_exp(x) */
static void big_from_double(big *a, double x, int E)
{
    big_zero(a);
    if (x == 0.0) return;
    int ex;
    double f = frexp(fabs(x), &ex);
    uint64_t m = (uint64_t)ldexp(f, 53);
    int sh = ex - 53 - E; /* may be negative only by the trailing zero bits of m */
    while (sh < 0) { m >>= 1; ++sh; }
    int limb = sh / 32, bit = sh % 32;
    if (limb + 3 > NL) abort();
    memset(a->d, 0, sizeof(uint32_t) * (size_t)(limb + 3));
    unsigned __int128 v = (unsigned __int128)m << bit;
    a->d[limb] = (uint32_t)v;
    a->d[limb + 1] = (uint32_t)(v >> 32);
    a->d[limb + 2] = (uint32_t)(v >> 64);
    a->n = limb + 3;
    a->sign = x < 0 ? -1 : 1;
    big_trim(a);
}

static int common_exp(const double *v, int n)
{
    int E = 0, any = 0;
    for (int i = 0; i < n; ++i) {
        if (v[i] == 0.0) continue;
        int e = low_exp(v[i]);
        if (!any || e < E) E = e;
        any = 1;
    }
    return E;
}

/* Exact sign of (a_u-p_u)(b_v-p_v) - (a_v-p_v)(b_u-p_u): twice the signed
 * area of the 2-D triangle (p, a, b). */
static int orient2d_sign(double pu, double pv, double au, double av, double bu, double bv)
{
    double v[6] = {pu, pv, au, av, bu, bv};
    int E = common_exp(v, 6);
    big P[6];
    for (int i = 0; i < 6; ++i) big_from_double(&P[i], v[i], E);
    big d1, d2, d3, d4, t1, t2, r;
    big_sub(&d1, &P[2], &P[0]);
    big_sub(&d2, &P[5], &P[1]);
    big_sub(&d3, &P[3], &P[1]);
    big_sub(&d4, &P[4], &P[0]);
    big_mul(&t1, &d1, &d2);
    big_mul(&t2, &d3, &d4);
    big_sub(&r, &t1, &t2);
    return r.sign;
}

/* Exact sign of sum_m w_m (m_k - t), where w_a = area(p,b,c), w_b = area(p,c,a),
 * w_c = area(p,a,b) in the (u,v) projection: this equals W * (x* - t), with W
 * the projected area of the triangle and x* the crossing coordinate. */
static int crossing_sign(double pu, double pv, double t, const double *A, const double *B,
                         const double *C, int ku, int kv, int kk)
{
    double v[12] = {pu, pv, t, A[ku], A[kv], A[kk], B[ku], B[kv], B[kk], C[ku], C[kv], C[kk]};
    int E = common_exp(v, 12);
    big X[12];
    for (int i = 0; i < 12; ++i) big_from_double(&X[i], v[i], E);
    /* relative coordinates */
    big au, av, ak, bu, bv, bk, cu, cv, ck;
    big_sub(&au, &X[3], &X[0]);  big_sub(&av, &X[4], &X[1]);  big_sub(&ak, &X[5], &X[2]);
    big_sub(&bu, &X[6], &X[0]);  big_sub(&bv, &X[7], &X[1]);  big_sub(&bk, &X[8], &X[2]);
    big_sub(&cu, &X[9], &X[0]);  big_sub(&cv, &X[10], &X[1]); big_sub(&ck, &X[11], &X[2]);
    big t1, t2, wa, wb, wc, s1, s2, s3, acc, acc2;
    /* w_a = bu*cv - bv*cu */
    big_mul(&t1, &bu, &cv); big_mul(&t2, &bv, &cu); big_sub(&wa, &t1, &t2);
    /* w_b = cu*av - cv*au */
    big_mul(&t1, &cu, &av); big_mul(&t2, &cv, &au); big_sub(&wb, &t1, &t2);
    /* w_c = au*bv - av*bu */
    big_mul(&t1, &au, &bv); big_mul(&t2, &av, &bu); big_sub(&wc, &t1, &t2);
    big_mul(&s1, &wa, &ak);
    big_mul(&s2, &wb, &bk);
    big_mul(&s3, &wc, &ck);
    big_add(&acc, &s1, &s2);
    big_add(&acc2, &acc, &s3);
    return acc2.sign;
}

/* --------------------------------------------------------- tagging --- */

static double centre(const double *origin, double dx, int ax, int64_t i)
{
    return origin[ax] + ((double)i + 0.5) * dx;
}

/* a line index, clamped in double before the integer cast */
static int64_t clampi(double v, int64_t lo, int64_t hi)
{
    if (v < (double)lo) v = (double)lo;
    if (v > (double)hi) v = (double)hi;
    return (int64_t)v;
}

static void put_theta(double *theta, int64_t c, int dir, double th)
{
    if (th < theta[6 * c + dir]) theta[6 * c + dir] = th;
}

/* Returns 0 on success, -1 on a non-finite coordinate. */
int oracle_tag(const double *tri, int64_t ntri, const int32_t *n, double dx, const double *origin,
               double bary_eps, uint8_t *blocked, double *theta)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    const int64_t ncell = nx * ny * nz;
    memset(blocked, 0, (size_t)ncell);
    for (int64_t c = 0; c < 6 * ncell; ++c) theta[c] = 2.0;
    for (int64_t t = 0; t < 9 * ntri; ++t)
        if (!isfinite(tri[t])) return -1;

    for (int64_t t = 0; t < ntri; ++t) {
        const double *A = tri + 9 * t, *B = A + 3, *C = A + 6;
        for (int k = 0; k < 3; ++k) {
            const int u = (k + 1) % 3, v = (k + 2) % 3;
            const int64_t nn[3] = {nx, ny, nz};
            double umin = fmin(A[u], fmin(B[u], C[u])), umax = fmax(A[u], fmax(B[u], C[u]));
            double vmin = fmin(A[v], fmin(B[v], C[v])), vmax = fmax(A[v], fmax(B[v], C[v]));
            double kmin = fmin(A[k], fmin(B[k], C[k])), kmax = fmax(A[k], fmax(B[k], C[k]));
            /* the triangle grown by bary_eps in barycentric terms stays inside its bounding
               box widened by 2 bary_eps times the extent on each side (its corners are
               a + bary_eps (2a - b - c) and the like) */
            const double gu = 2.0 * bary_eps * (umax - umin), gv = 2.0 * bary_eps * (vmax - vmin);
            const double gk = 2.0 * bary_eps * (kmax - kmin);
            umin -= gu; umax += gu; vmin -= gv; vmax += gv; kmin -= gk; kmax += gk;
            /* exact orientation of the projected triangle (zero: parallel to the lines) */
            const int sT = orient2d_sign(A[u], A[v], B[u], B[v], C[u], C[v]);
            /* candidate grid lines: generous bounding box, the exact test decides */
            int64_t j0 = clampi(floor((umin - origin[u]) / dx - 0.5) - 1.0, 0, nn[u]);
            int64_t j1 = clampi(ceil((umax - origin[u]) / dx - 0.5) + 1.0, -1, nn[u] - 1);
            int64_t l0 = clampi(floor((vmin - origin[v]) / dx - 0.5) - 1.0, 0, nn[v]);
            int64_t l1 = clampi(ceil((vmax - origin[v]) / dx - 0.5) + 1.0, -1, nn[v] - 1);
            int64_t i0 = clampi(floor((kmin - origin[k]) / dx - 0.5) - 1.0, 0, nn[k]);
            /* segments (i, i+1) inside the domain */
            int64_t i1 = clampi(ceil((kmax - origin[k]) / dx - 0.5) + 1.0, -1, nn[k] - 2);
            for (int64_t j = j0; j <= j1; ++j) {
                for (int64_t l = l0; l <= l1; ++l) {
                    const double pu = centre(origin, dx, u, j), pv = centre(origin, dx, v, l);
                    /* point in closed projected triangle, exactly */
                    int sa = orient2d_sign(pu, pv, B[u], B[v], C[u], C[v]);
                    int sb = orient2d_sign(pu, pv, C[u], C[v], A[u], A[v]);
                    int sc = orient2d_sign(pu, pv, A[u], A[v], B[u], B[v]);
                    int sW;
                    if (sa >= 0 && sb >= 0 && sc >= 0 && (sa + sb + sc) > 0) sW = 1;
                    else if (sa <= 0 && sb <= 0 && sc <= 0 && (sa + sb + sc) < 0) sW = -1;
                    else sW = 0;
                    /* double crossing coordinate, fixed operation order */
                    double dau = A[u] - pu, dav = A[v] - pv;
                    double dbu = B[u] - pu, dbv = B[v] - pv;
                    double dcu = C[u] - pu, dcv = C[v] - pv;
                    double wa = dbu * dcv - dbv * dcu;
                    double wb = dcu * dav - dcv * dau;
                    double wc = dau * dbv - dav * dbu;
                    double num = (wa * A[k] + wb * B[k]) + wc * C[k];
                    double den = (wa + wb) + wc;
                    if (sW == 0) {
                        /* missed exactly: hit within the tolerance only */
                        if (!(bary_eps > 0.0) || sT == 0) continue;
                        const double st = (double)sT, lim = -bary_eps * fabs(den);
                        if (!(wa * st >= lim && wb * st >= lim && wc * st >= lim)) continue;
                        sW = sT;
                    }
                    double xs = num / den;
                    for (int64_t i = i0; i <= i1; ++i) {
                        const double xa = centre(origin, dx, k, i), xb = centre(origin, dx, k, i + 1);
                        int s_lo = crossing_sign(pu, pv, xa, A, B, C, u, v, k) * sW; /* sign(x*-xa) */
                        int s_hi = crossing_sign(pu, pv, xb, A, B, C, u, v, k) * sW; /* sign(x*-xb) */
                        if (s_lo < 0 || s_hi > 0) continue;
                        double tl = (xs - xa) / dx, th = (xb - xs) / dx;
                        if (tl < 0.0) tl = 0.0;
                        if (tl > 1.0) tl = 1.0;
                        if (th < 0.0) th = 0.0;
                        if (th > 1.0) th = 1.0;
                        int64_t idx[3];
                        idx[k] = i; idx[u] = j; idx[v] = l;
                        int64_t ca = idx[0] + nx * (idx[1] + ny * idx[2]);
                        idx[k] = i + 1;
                        int64_t cb = idx[0] + nx * (idx[1] + ny * idx[2]);
                        blocked[ca] |= (uint8_t)(1u << (2 * k + 1));
                        blocked[cb] |= (uint8_t)(1u << (2 * k));
                        put_theta(theta, ca, 2 * k + 1, tl);
                        put_theta(theta, cb, 2 * k, th);
                    }
                }
            }
        }
    }
    return 0;
}

/* Exposed for the predicate pins. */
int oracle_orient2d_sign(double pu, double pv, double au, double av, double bu, double bv)
{
    return orient2d_sign(pu, pv, au, av, bu, bv);
}

int oracle_crossing_sign(double pu, double pv, double t, const double *A, const double *B,
                         const double *C, int k)
{
    return crossing_sign(pu, pv, t, A, B, C, (k + 1) % 3, (k + 2) % 3, k);
}
