// Crank-Nicolson momentum predictor (eq. (crank-nicolson)) and its BiCGStab solve
// (Sec. 2.1), templated on the cell-field type T (double for the plain path, float for
// the mixed path); dot products and all solver scalars are double.
//
// With H the explicit momentum right-hand side and L its part linear in the velocity
// (flux-form central advection by the frozen face velocity U^n, diffusion with
// nu + nu_t,f), the increment delta = u* - u^n of one step solves, per component,
//     A delta = (I - dt/2 L) delta = dt H^n,
// a nonsymmetric system (advection).  The three components are solved together: one
// launch per pass serves all of them, so the coefficients (U on six faces, nu_t of the
// cell and its neighbours, the blocked mask) are read once for three systems, while
// each component keeps its own BiCGStab scalars and stops on its own.
//
// BiCGStab iteration it in five passes; the scalars come from per-block partial sums
// that the next pass adds up in block order (every block computes the same totals):
//   D_it  (elementwise): stop test on ||r||; rho = <r0, r>; beta = (rho/rho_prev)
//         (alpha/omega); p = r + beta (p - omega v)   (p = r at it = 0)
//   AP_it (stencil):     v = A p;  <r0, v>
//   S_it  (elementwise): alpha = rho / <r0, v>;  s = r - alpha v, stored over r
//   AS_it (stencil):     t = A s;  <t, s>, <t, t>, <s, s>
//   X_it  (elementwise): omega = <t,s>/<t,t> (0 when ||s|| is already small: the
//         half-step exit); x += alpha p + omega s; r = s - omega t;  <r0, r>, <r, r>
// The vector updates are kept out of the stencil passes so each stencil gathers one
// array (forming p or s on the fly at seven points gathered three or two arrays per
// component, and measured slower).  Algorithmic traffic per cell and iteration, three
// components of T = double: D reads r, p, v, writes p (96 B); AP reads p, r0, U on
// three faces, nu_t and the mask and writes v (105 B); S reads r, v, writes r (72 B);
// AS reads s and the coefficients and writes t (81 B); X reads x, p, s, t, r0 and
// writes x, r (168 B).  522 B in all.

#include "common.h"

namespace ibm {
namespace {

// partial-sum slots (each MAX_BLOCKS doubles)
constexpr int CS_R0R = 0;   // <r0, r>      x3  (written by the init pass and X)
constexpr int CS_RR = 3;    // <r, r>       x3  (init, X)
constexpr int CS_BB = 6;    // <b, b>       x3  (init)
constexpr int CS_R0V = 9;   // <r0, v>      x3  (P)
constexpr int CS_TS = 12;   // <t, s>       x3  (S)
constexpr int CS_TT = 15;   // <t, t>       x3  (S)
constexpr int CS_SS = 18;   // <s, s>       x3  (S)
constexpr int CS_SLOTS = 21;

// (A q)_c for component m, A = I - dt/2 L (identity at dead-end cells), from the value
// qc at the cell and nb[d] across each face (the neighbour, or anything where the face
// is blocked or a non-periodic domain face: those take the ghosts); src(m, n) gives q
// at cell n for the opposite cell of an eq. (q_axis) ghost.
template <class T, class Src>
__device__ inline T apply_nb(const Geo& g, const Sten& st, const Src& src, int m, long long c, uint8_t msk,
                             const bool (&bnd)[6], const T (&Uf)[6], const T (&visc)[6], T qc, const T (&nb)[6],
                             T hdt, T idx, T idx2) {
    T L = (T)0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        T qn;
        if ((msk >> d) & 1) {
            // eq. (q_axis) ghost with a zero wall velocity
            const uint32_t id = cut_id(st, c, msk, d);
            double v = st.a_c[id] * (double)qc;
            const int32_t o = st.opp[id];
            if (o >= 0) v += st.a_o[id] * (double)src(m, o);
            qn = (T)v;
        } else if (bnd[d]) {
            const int kind = g.bc[d];
            qn = (kind == IBM_BC_INFLOW || (kind == IBM_BC_SLIP && m == (d >> 1))) ? -qc : qc;
        } else {
            qn = nb[d];
        }
        const T s = (d & 1) ? (T)1 : (T)-1;
        L = L - s * Uf[d] * ((T)0.5 * (qc + qn)) * idx + visc[d] * (qn - qc) * idx2;
    }
    return qc - hdt * L;
}

// Z-marching sweep over (64x4 tile, z-slab) items, the order of the pressure passes:
// each thread walks one column of its slab and carries the values of the vector at
// z-1, z and z+1 (three components), the eddy viscosity of the three planes and the
// face velocity under the cell, so a z-neighbour is read once; x and y neighbours
// come from the cache lines the wavefront and the neighbouring tiles read.  For
// every cell and active component it calls emit(c, m, q_c, (A q)_c).
template <class T, class Src, class Emit>
__device__ inline void cn_march(const Geo& g, const Sten& st, const C3<double>& U, const T* nut, T nu, T hdt,
                                const int (&act)[3], const Src& src, Emit&& emit) {
    const T idx = (T)(1.0 / g.dx), idx2 = (T)(1.0 / (g.dx * g.dx));
    const int nzc = slab_count(g.nz);
    const long long tiles = (long long)g.ntx * g.nty;
    const long long items = tiles * nzc;
    const int nblk = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nblk);
    const long long w0 = items * ch / nblk, w1 = items * (ch + 1) / nblk;
    const long long plane = (long long)g.nx * g.ny;
    const T uin[3] = {(T)g.uin[0], (T)g.uin[1], (T)g.uin[2]};
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
        bool bnd[6];
        bnd[0] = i == 0 && g.bc[0] != IBM_BC_PERIODIC;
        bnd[1] = i == g.nx - 1 && g.bc[1] != IBM_BC_PERIODIC;
        bnd[2] = j == 0 && g.bc[2] != IBM_BC_PERIODIC;
        bnd[3] = j == g.ny - 1 && g.bc[3] != IBM_BC_PERIODIC;
        const int zb = z0 == 0 ? g.nz - 1 : z0 - 1;
        T qb[3], qc[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            qb[m] = act[m] ? src(m, col + plane * zb) : (T)0;
            qc[m] = act[m] ? src(m, col + plane * z0) : (T)0;
        }
        T nb_b = nut ? nut[col + plane * zb] : (T)0;
        T nb_c = nut ? nut[col + plane * z0] : (T)0;
        T uz_b = (T)U.p[2][col + plane * zb];
        for (int k = z0; k < z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = col + plane * k;
            const long long ct = col + plane * zt;
            bnd[4] = k == 0 && g.bc[4] != IBM_BC_PERIODIC;
            bnd[5] = k == g.nz - 1 && g.bc[5] != IBM_BC_PERIODIC;
            T qt[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) qt[m] = act[m] ? src(m, ct) : (T)0;
            const T nb_t = nut ? nut[ct] : (T)0;
            const uint8_t msk = st.mask[c];
            const bool dead = dead_cell(st, c, msk);
            T Uf[6];
            Uf[0] = bnd[0] ? (g.bc[0] == IBM_BC_INFLOW ? uin[0] : (T)0) : (T)U.p[0][c + ow];
            Uf[1] = (T)U.p[0][c];
            Uf[2] = bnd[2] ? (g.bc[2] == IBM_BC_INFLOW ? uin[1] : (T)0) : (T)U.p[1][c + os];
            Uf[3] = (T)U.p[1][c];
            Uf[4] = bnd[4] ? (g.bc[4] == IBM_BC_INFLOW ? uin[2] : (T)0) : uz_b;
            Uf[5] = (T)U.p[2][c];
            T nn[6];
            nn[0] = nut ? nut[c + ow] : (T)0;
            nn[1] = nut ? nut[c + oe] : (T)0;
            nn[2] = nut ? nut[c + os] : (T)0;
            nn[3] = nut ? nut[c + on] : (T)0;
            nn[4] = nb_b;
            nn[5] = nb_t;
            T visc[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const bool closed = bnd[d] || ((msk >> d) & 1);
                visc[d] = nu + (closed ? nb_c : (T)0.5 * (nb_c + nn[d]));
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                if (!act[m]) continue;
                T out;
                if (dead) {
                    out = qc[m];
                } else {
                    const T nbv[6] = {src(m, c + ow), src(m, c + oe), src(m, c + os), src(m, c + on), qb[m], qt[m]};
                    out = apply_nb(g, st, src, m, c, msk, bnd, Uf, visc, qc[m], nbv, hdt, idx, idx2);
                }
                emit(c, m, qc[m], out);
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                qb[m] = qc[m];
                qc[m] = qt[m];
            }
            nb_b = nb_c;
            nb_c = nb_t;
            uz_b = Uf[5];
        }
    }
}

template <class T>
struct SrcPlain {
    const T* q[3];
    __device__ T operator()(int m, long long n) const { return q[m][n]; }
};

// totals of K slots (three components each) over nparts blocks, in block order
template <int K>
__device__ inline void slot_totals(const double* part, const int (&slot)[K], int nparts, double* sh,
                                   double (&out)[K][3]) {
    double v[3 * K];
#pragma unroll
    for (int q = 0; q < 3 * K; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nparts; b += NT) {
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
            for (int m = 0; m < 3; ++m) v[3 * q + m] += part[(slot[q] + m) * MAX_BLOCKS + b];
    }
    block_reduce<3 * K>(v, sh);
#pragma unroll
    for (int q = 0; q < K; ++q)
#pragma unroll
        for (int m = 0; m < 3; ++m) out[q][m] = v[3 * q + m];
}

template <int K>
__device__ inline void write_partials(double* part, const int (&slot)[K], const double (&v)[3 * K]) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
            for (int m = 0; m < 3; ++m) part[(slot[q] + m) * MAX_BLOCKS + blockIdx.x] = v[3 * q + m];
    }
}

// The done flag as one value for the whole block: block 0 of the running pass may set
// it while other blocks start, so it is read once and shared, and every wave of a
// block takes the same path through the barriers that follow.
__device__ inline bool block_done(const CnState* cs) {
    __shared__ int d;
    if (threadIdx.x == 0) d = __atomic_load_n(&cs->done, __ATOMIC_RELAXED);
    __syncthreads();
    const bool r = d != 0;
    __syncthreads();
    return r;
}

// y = A q for the three components (ibm_momentum_apply)
template <class T>
__global__ void __launch_bounds__(NT) k_cn_apply(Geo g, Sten st, C3<double> U, const T* nut, T nu, T hdt, C3<T> q,
                                                 V3<T> y) {
    SrcPlain<T> src{{q.p[0], q.p[1], q.p[2]}};
    const int act[3] = {1, 1, 1};
    cn_march(g, st, U, nut, nu, hdt, act, src, [&](long long c, int m, T, T aq) { y.p[m][c] = aq; });
}

// r = b - A x, r0 = r; partials <r0,r> (= <r,r>), <r,r>, <b,b>.  b may alias x: b is
// read at the cell only, x at the cell and its neighbours, and neither is written.
template <class T>
__global__ void __launch_bounds__(NT) k_cn_init(Geo g, Sten st, C3<double> U, const T* nut, T nu, T hdt, C3<T> b,
                                                C3<T> x, V3<T> r, V3<T> r0, double* part) {
    __shared__ double sh[4 * 9];
    SrcPlain<T> src{{x.p[0], x.p[1], x.p[2]}};
    double v[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = 0.0;
    const int act[3] = {1, 1, 1};
    cn_march(g, st, U, nut, nu, hdt, act, src, [&](long long c, int m, T, T ax) {
        const T bc = b.p[m][c];
        const T rc = bc - ax;
        r.p[m][c] = rc;
        r0.p[m][c] = rc;
        v[m] += (double)rc * (double)rc;
        v[6 + m] += (double)bc * (double)bc;
    });
#pragma unroll
    for (int m = 0; m < 3; ++m) v[3 + m] = v[m];
    block_reduce<9>(v, sh);
    const int sl[3] = {CS_R0R, CS_RR, CS_BB};
    write_partials<3>(part, sl, v);
}

#define CN_CELLS(c, N) \
    for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < (N); c += (long long)gridDim.x * NT)

// Pass D of iteration it (see the file comment).  At it == 0 it also turns the init
// partials into the per-component tolerances and zeroes x of a component with b = 0.
template <class T>
__global__ void __launch_bounds__(NT) k_cn_dir(Geo g, V3<T> x, C3<T> r, V3<T> p, C3<T> v, double* part, int nparts,
                                               int it, int max_iter, double tol, CnState* cs) {
    if (block_done(cs)) return;
    __shared__ double sh[4 * 9];
    const int par = it & 1, pp = (it + 1) & 1;
    double tot[3][3];
    const int sl[3] = {CS_R0R, CS_RR, CS_BB};
    slot_totals<3>(part, sl, nparts, sh, tot);
    int act[3];
    T beta[3], omega[3];
    int status = CN_RUNNING;
    int fin_iters[3] = {-1, -1, -1};
    double tol2[3], rho[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        act[m] = 0;
        beta[m] = (T)0;
        omega[m] = (T)0;
        rho[m] = tot[0][m];
        const double rr = tot[1][m];
        if (it == 0) {
            const double bb = tot[2][m];
            tol2[m] = tol * tol * bb;
            if (!(rr == rr) || !(bb == bb)) status = CN_NAN;
            else if (bb == 0.0 || rr <= tol2[m]) fin_iters[m] = 0;
            else act[m] = 1;
        } else {
            tol2[m] = cs->tol2[m];
            if (!cs->active[pp][m]) continue;
            if (!(rr == rr)) status = CN_NAN;
            else if (cs->sconv[pp][m] || rr <= tol2[m]) fin_iters[m] = it;
            else if (it >= max_iter) {
                fin_iters[m] = it;
                if (status == CN_RUNNING) status = CN_MAXITER;
            } else if (rho[m] == 0.0) status = CN_BREAKDOWN;
            else {
                act[m] = 1;
                beta[m] = (T)((rho[m] / cs->rho[pp][m]) * (cs->alpha[pp][m] / cs->omega[pp][m]));
                omega[m] = (T)cs->omega[pp][m];
            }
        }
    }
    const bool any = act[0] || act[1] || act[2];
    const bool stop = status == CN_NAN || status == CN_BREAKDOWN || !any;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            if (it == 0) {
                cs->tol2[m] = tol2[m];
                cs->bb[m] = tot[2][m];
            }
            cs->rho[par][m] = rho[m];
            cs->active[par][m] = act[m];
            cs->sconv[par][m] = 0;
            if (fin_iters[m] >= 0) cs->iters[m] = fin_iters[m];
        }
        if (status == CN_MAXITER && !any) cs->status = CN_MAXITER;
        if (status == CN_NAN || status == CN_BREAKDOWN) cs->status = status;
        else if (!any && cs->status == CN_RUNNING) cs->status = CN_CONVERGED;
        if (stop) cs->done = 1;
    }
    const long long N = (long long)g.nx * g.ny * g.nz;
    if (it == 0 && (tot[2][0] == 0.0 || tot[2][1] == 0.0 || tot[2][2] == 0.0)) {
        CN_CELLS(c, N)
#pragma unroll
        for (int m = 0; m < 3; ++m)
            if (tot[2][m] == 0.0) x.p[m][c] = (T)0;
    }
    if (stop) return;
    CN_CELLS(c, N)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        if (!act[m]) continue;
        p.p[m][c] = it == 0 ? r.p[m][c] : r.p[m][c] + beta[m] * (p.p[m][c] - omega[m] * v.p[m][c]);
    }
}

// Pass AP of iteration it: v = A p, <r0, v>.
template <class T>
__global__ void __launch_bounds__(NT) k_cn_ap(Geo g, Sten st, C3<double> U, const T* nut, T nu, T hdt, C3<T> p,
                                              V3<T> v, C3<T> r0, double* part, int it, CnState* cs) {
    if (block_done(cs)) return;
    __shared__ double sh3[4 * 3];
    const int par = it & 1;
    int act[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) act[m] = cs->active[par][m];
    SrcPlain<T> src{{p.p[0], p.p[1], p.p[2]}};
    double acc[3] = {0.0, 0.0, 0.0};
    cn_march(g, st, U, nut, nu, hdt, act, src, [&](long long c, int m, T, T vc) {
        v.p[m][c] = vc;
        acc[m] += (double)r0.p[m][c] * (double)vc;
    });
    block_reduce<3>(acc, sh3);
    const int so[1] = {CS_R0V};
    write_partials<1>(part, so, acc);
}

// Pass S of iteration it: alpha = rho / <r0, v>; s = r - alpha v over r.
template <class T>
__global__ void __launch_bounds__(NT) k_cn_s(Geo g, V3<T> r, C3<T> v, double* part, int nparts, int it,
                                             CnState* cs) {
    if (block_done(cs)) return;
    __shared__ double sh[4 * 9];
    const int par = it & 1;
    double tot[1][3];
    const int sl[1] = {CS_R0V};
    slot_totals<1>(part, sl, nparts, sh, tot);
    int act[3];
    T alpha[3];
    bool broke = false;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        act[m] = cs->active[par][m];
        alpha[m] = (T)0;
        if (!act[m]) continue;
        if (tot[0][m] == 0.0 || !(tot[0][m] == tot[0][m])) broke = true;
        else alpha[m] = (T)(cs->rho[par][m] / tot[0][m]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < 3; ++m) cs->alpha[par][m] = (double)alpha[m];
        if (broke) {
            cs->status = CN_BREAKDOWN;
            cs->done = 1;
        }
    }
    if (broke) return;
    const long long N = (long long)g.nx * g.ny * g.nz;
    CN_CELLS(c, N)
#pragma unroll
    for (int m = 0; m < 3; ++m)
        if (act[m]) r.p[m][c] = r.p[m][c] - alpha[m] * v.p[m][c];
}

// Pass AS of iteration it: t = A s, <t, s>, <t, t>, <s, s>.
template <class T>
__global__ void __launch_bounds__(NT) k_cn_as(Geo g, Sten st, C3<double> U, const T* nut, T nu, T hdt, C3<T> sv,
                                              V3<T> tv, double* part, int it, CnState* cs) {
    if (block_done(cs)) return;
    __shared__ double sh[4 * 9];
    const int par = it & 1;
    int act[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) act[m] = cs->active[par][m];
    SrcPlain<T> src{{sv.p[0], sv.p[1], sv.p[2]}};
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
    cn_march(g, st, U, nut, nu, hdt, act, src, [&](long long c, int m, T sc, T tc) {
        tv.p[m][c] = tc;
        acc[m] += (double)tc * (double)sc;
        acc[3 + m] += (double)tc * (double)tc;
        acc[6 + m] += (double)sc * (double)sc;
    });
    block_reduce<9>(acc, sh);
    const int so[3] = {CS_TS, CS_TT, CS_SS};
    write_partials<3>(part, so, acc);
}

// Pass X of iteration it: omega; x += alpha p + omega s; r = s - omega t (s is in r).
template <class T>
__global__ void __launch_bounds__(NT) k_cn_x(Geo g, V3<T> x, V3<T> r, C3<T> r0, C3<T> p, C3<T> tv, double* part,
                                             int nparts, int it, CnState* cs) {
    if (block_done(cs)) return;
    __shared__ double sh[4 * 9];
    const int par = it & 1;
    double tot[3][3];
    const int sl[3] = {CS_TS, CS_TT, CS_SS};
    slot_totals<3>(part, sl, nparts, sh, tot);
    int act[3], sconv[3];
    T alpha[3], omega[3];
    bool broke = false;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        act[m] = cs->active[par][m];
        sconv[m] = 0;
        alpha[m] = (T)cs->alpha[par][m];
        omega[m] = (T)0;
        if (!act[m]) continue;
        if (tot[2][m] <= cs->tol2[m]) {
            sconv[m] = 1;
        } else {
            const double w = tot[0][m] / tot[1][m];
            if (w == 0.0 || !(w == w)) broke = true;
            else omega[m] = (T)w;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            cs->omega[par][m] = (double)omega[m];
            cs->sconv[par][m] = sconv[m];
        }
        if (broke) {
            cs->status = CN_BREAKDOWN;
            cs->done = 1;
        }
    }
    if (broke) return;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const long long N = (long long)g.nx * g.ny * g.nz;
    CN_CELLS(c, N) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            if (!act[m]) continue;
            const T sc = r.p[m][c];
            T rn = sc;
            if (sconv[m]) {
                x.p[m][c] = x.p[m][c] + alpha[m] * p.p[m][c];
            } else {
                x.p[m][c] = x.p[m][c] + alpha[m] * p.p[m][c] + omega[m] * sc;
                rn = sc - omega[m] * tv.p[m][c];
                r.p[m][c] = rn;
            }
            acc[m] += (double)r0.p[m][c] * (double)rn;
            acc[3 + m] += (double)rn * (double)rn;
        }
    }
    block_reduce<6>(acc, sh);
    const int so[2] = {CS_R0R, CS_RR};
    write_partials<2>(part, so, acc);
}

// u* = u + delta away from dead-end cells (those already hold their wall velocity)
template <class T>
__global__ void __launch_bounds__(NT) k_cn_finish(Geo g, Sten st, C3<T> u, C3<T> dx, V3<T> us) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        const long long c = cidx(g, i, j, k);
        if (dead_cell(st, c, st.mask[c])) continue;
#pragma unroll
        for (int m = 0; m < 3; ++m) us.p[m][c] = u.p[m][c] + dx.p[m][c];
    }
}

__global__ void k_cn_reset(CnState* cs) {
    if (threadIdx.x == 0) {
        cs->status = CN_RUNNING;
        cs->done = 0;
        for (int m = 0; m < 3; ++m) {
            cs->iters[m] = 0;
            cs->active[0][m] = cs->active[1][m] = 0;
            cs->sconv[0][m] = cs->sconv[1][m] = 0;
        }
    }
}

// workspace vector w (0 x, 1 r, 2 r0, 3 p, 4 v, 5 t), component m
template <class T>
inline T* ws_vec(ibm_ctx* c, int w, int m) {
    return (T*)c->cn_ws + ((long long)w * 3 + m) * c->N;
}

template <class T>
int cn_solve_t(ibm_ctx* c, const T* const* b, T* const* x, double* const* U, const T* nut, double nu, double dt,
               double tol, int max_iter, int iters[3], hipStream_t s) {
    const Geo& g = c->geo;
    const Sten st = sten_of(c);
    const int nb = march_blocks(g);   // the marching passes set the count; all passes share it
    const C3<double> UU{{U[0], U[1], U[2]}};
    const T tnu = (T)nu, hdt = (T)(0.5 * dt);
    auto cv = [&](int w) { return C3<T>{{ws_vec<T>(c, w, 0), ws_vec<T>(c, w, 1), ws_vec<T>(c, w, 2)}}; };
    auto vv = [&](int w) { return V3<T>{{ws_vec<T>(c, w, 0), ws_vec<T>(c, w, 1), ws_vec<T>(c, w, 2)}}; };
    const V3<T> xx{{x[0], x[1], x[2]}};
    const C3<T> xc{{x[0], x[1], x[2]}};
    const C3<T> bb{{b[0], b[1], b[2]}};
    k_cn_reset<<<1, 64, 0, s>>>(c->cn_state);
    k_cn_init<T><<<nb, NT, 0, s>>>(g, st, UU, nut, tnu, hdt, bb, xc, vv(1), vv(2), c->cn_part);
    IBM_HIP(hipGetLastError());
    // passes in order D_0 AP_0 S_0 AS_0 X_0 D_1 ...; every batch ends with a pass D,
    // whose stop test the host then reads
    constexpr int NP = 5;
    long long pass = 0;
    auto launch = [&](long long q) {
        const int it = (int)(q / NP), kind = (int)(q % NP);
        if (kind == 0)
            launch_timed(c, TK_CN_D, k_cn_dir<T>, nb, s, g, xx, cv(1), vv(3), cv(4), c->cn_part, nb, it, max_iter, tol,
                         c->cn_state);
        else if (kind == 1)
            launch_timed(c, TK_CN_AP, k_cn_ap<T>, nb, s, g, st, UU, nut, tnu, hdt, cv(3), vv(4), cv(2), c->cn_part, it,
                         c->cn_state);
        else if (kind == 2)
            launch_timed(c, TK_CN_S, k_cn_s<T>, nb, s, g, vv(1), cv(4), c->cn_part, nb, it, c->cn_state);
        else if (kind == 3)
            launch_timed(c, TK_CN_AS, k_cn_as<T>, nb, s, g, st, UU, nut, tnu, hdt, cv(1), vv(5), c->cn_part, it,
                         c->cn_state);
        else
            launch_timed(c, TK_CN_X, k_cn_x<T>, nb, s, g, xx, vv(1), cv(2), cv(3), cv(5), c->cn_part, nb, it,
                         c->cn_state);
    };
    int batch = c->cn_last_iters > 0 ? c->cn_last_iters + 1 : 4;
    while (true) {
        // iterations pass/NP .. pass/NP + batch - 1, then the next pass D
        const long long end = (pass / NP + batch) * NP;
        const long long last = end < (long long)NP * max_iter ? end : (long long)NP * max_iter;
        for (; pass <= last; ++pass) launch(pass);
        IBM_HIP(hipGetLastError());
        IBM_HIP(hipMemcpyAsync(c->h_cn_state, c->cn_state, sizeof(CnState), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (c->h_cn_state->done) break;
        if (pass > (long long)NP * max_iter) {
            set_error("momentum solve: state not final after the iteration cap");
            return IBM_ERR_HIP;
        }
        batch = 4;
    }
    timing_collect(c);
    const CnState& h = *c->h_cn_state;
    int most = 0;
    for (int m = 0; m < 3; ++m) {
        iters[m] = h.iters[m];
        if (h.iters[m] > most) most = h.iters[m];
    }
    c->cn_last_iters = most;
    if (h.status == CN_CONVERGED) return IBM_OK;
    if (h.status == CN_NAN) {
        set_error("momentum solve: non-finite residual");
        return IBM_ERR_NAN;
    }
    set_error(h.status == CN_BREAKDOWN ? "momentum solve: BiCGStab breakdown"
                                       : "momentum solve: iteration cap reached");
    return IBM_NOT_CONVERGED;
}

}  // namespace

int cn_prepare(ibm_ctx* c) {
    if (c->cn_ws) return IBM_OK;
    const size_t ts = c->precision == IBM_FP64 ? sizeof(double) : sizeof(float);
    const size_t bytes = ts * 18 * (size_t)c->N;
    // all or nothing: a partly allocated workspace would pass the readiness check
    if (ibm::dev_malloc(&c->cn_ws, bytes) != hipSuccess ||
        ibm::dev_malloc((void**)&c->cn_part, sizeof(double) * CS_SLOTS * MAX_BLOCKS) != hipSuccess ||
        ibm::dev_malloc((void**)&c->cn_state, sizeof(CnState)) != hipSuccess ||
        ibm::host_malloc(&c->h_cn_state, sizeof(CnState)) != hipSuccess) {
        (void)hipGetLastError();
        cn_release(c);
        set_error("Crank-Nicolson workspace: out of memory");
        return IBM_ERR_OOM;
    }
    c->cn_last_iters = 0;
    return IBM_OK;
}

int cn_apply(ibm_ctx* c, const void* const* q, double* const* U, const void* nut, double nu, double dt,
             void* const* out, hipStream_t s) {
    const Geo& g = c->geo;
    const C3<double> UU{{U[0], U[1], U[2]}};
    if (c->precision == IBM_FP64) {
        k_cn_apply<double><<<march_blocks(g), NT, 0, s>>>(
            g, sten_of(c), UU, (const double*)nut, nu, 0.5 * dt,
            C3<double>{{(const double*)q[0], (const double*)q[1], (const double*)q[2]}},
            V3<double>{{(double*)out[0], (double*)out[1], (double*)out[2]}});
    } else {
        k_cn_apply<float><<<march_blocks(g), NT, 0, s>>>(
            g, sten_of(c), UU, (const float*)nut, (float)nu, (float)(0.5 * dt),
            C3<float>{{(const float*)q[0], (const float*)q[1], (const float*)q[2]}},
            V3<float>{{(float*)out[0], (float*)out[1], (float*)out[2]}});
    }
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int cn_solve(ibm_ctx* c, const void* const* b, void* const* x, double* const* U, const void* nut, double nu,
             double dt, double tol, int max_iter, int iters[3], hipStream_t s) {
    if (!c->cn_ws) {
        set_error("Crank-Nicolson: call ibm_prepare_crank_nicolson first (it allocates the solver workspace)");
        return IBM_ERR_ARG;
    }
    if (c->precision == IBM_FP64) {
        const double* bp[3] = {(const double*)b[0], (const double*)b[1], (const double*)b[2]};
        double* xp[3] = {(double*)x[0], (double*)x[1], (double*)x[2]};
        return cn_solve_t<double>(c, bp, xp, U, (const double*)nut, nu, dt, tol, max_iter, iters, s);
    }
    const float* bp[3] = {(const float*)b[0], (const float*)b[1], (const float*)b[2]};
    float* xp[3] = {(float*)x[0], (float*)x[1], (float*)x[2]};
    return cn_solve_t<float>(c, bp, xp, U, (const float*)nut, nu, dt, tol < 1e-6 ? 1e-6 : tol, max_iter, iters, s);
}

// Crank-Nicolson predictor after k_predict has written dt H^n (dv - u at dead-end
// cells) into the workspace's x and the dead-end velocities into u*: solve for the
// increment in place, then u* = u^n + delta.
int cn_predict(ibm_ctx* c, void** u, double** U, const ibm_step_params* prm, int iters[3], hipStream_t s) {
    const double tol = prm->mom_tol > 0.0 ? prm->mom_tol : 1e-10;
    const int max_iter = prm->mom_max_iter > 0 ? prm->mom_max_iter : 200;
    void* xs[3];
    const size_t ts = c->precision == IBM_FP64 ? sizeof(double) : sizeof(float);
    for (int m = 0; m < 3; ++m) xs[m] = (char*)c->cn_ws + ts * (size_t)m * (size_t)c->N;
    int rc = cn_solve(c, xs, xs, U, c->nut, prm->nu, prm->dt, tol, max_iter, iters, s);
    if (rc) return rc;
    const Geo& g = c->geo;
    if (c->precision == IBM_FP64) {
        k_cn_finish<double><<<grid_blocks(g), NT, 0, s>>>(
            g, sten_of(c), C3<double>{{(const double*)u[0], (const double*)u[1], (const double*)u[2]}},
            C3<double>{{(const double*)xs[0], (const double*)xs[1], (const double*)xs[2]}},
            V3<double>{{(double*)c->ustar[0], (double*)c->ustar[1], (double*)c->ustar[2]}});
    } else {
        k_cn_finish<float><<<grid_blocks(g), NT, 0, s>>>(
            g, sten_of(c), C3<float>{{(const float*)u[0], (const float*)u[1], (const float*)u[2]}},
            C3<float>{{(const float*)xs[0], (const float*)xs[1], (const float*)xs[2]}},
            V3<float>{{(float*)c->ustar[0], (float*)c->ustar[1], (float*)c->ustar[2]}});
    }
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

void cn_release(ibm_ctx* c) {
    if (c->cn_ws) (void)hipFree(c->cn_ws);
    if (c->cn_part) (void)hipFree(c->cn_part);
    if (c->cn_state) (void)hipFree(c->cn_state);
    if (c->h_cn_state) (void)hipHostFree(c->h_cn_state);
    c->cn_ws = nullptr;
    c->cn_part = nullptr;
    c->cn_state = nullptr;
    c->h_cn_state = nullptr;
}

}  // namespace ibm
