// Per-step kernels of the fractional step (Sec. 2.1), templated on the cell-field
// type T (double for the plain path, float for the mixed path); face velocities U,
// pressure and the Poisson right-hand side are always double.
//
// Every kernel walks 64x4 tiles of one z-plane, one cell per thread, with the
// XCD-aware tile order of common.h.  Face neighbours are read straight from global
// memory: within a wavefront the x-neighbours are the same cache lines, the y- and
// z-neighbours were just touched by the tiles before on the same XCD, so each value
// comes from HBM about once.  Cells with a blocked face take the one branch that
// looks up the cut list (the paper's single 'if' into the dummy-cell data, Sec. 2.3.1).

#include <initializer_list>
#include <mutex>

#include "common.h"

namespace ibm {

namespace {

// eq. (q_axis) ghost of component m behind blocked face d of cell c
template <class T>
__device__ inline double ghost(const Sten& st, const T* q, long long c, uint8_t msk, int d, int m,
                               const double* wall, double qc) {
    uint32_t id = cut_id(st, c, msk, d);
    double w = wall ? wall[3 * (long long)id + m] : 0.0;
    double v = st.a_ib[id] * w + st.a_c[id] * qc;
    int32_t o = st.opp[id];
    if (o >= 0) v += st.a_o[id] * (double)q[o];
    return v;
}

// velocity ghost behind a domain face: inflow Dirichlet u_in, slip (odd normal,
// even tangential), outflow zero gradient
__device__ inline double bc_ghost(const Geo& g, int d, int m, double qc) {
    int kind = g.bc[d];
    if (kind == IBM_BC_INFLOW) return 2.0 * g.uin[m] - qc;
    if (kind == IBM_BC_SLIP && m == (d >> 1)) return -qc;
    return qc;
}

template <class T, class A>
__device__ inline void nbvals(const Geo& g, const Sten& st, const T* q, int m, int i, int j, int k, long long c,
                              uint8_t msk, const double* wall, A qc, A (&nb)[6]) {
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        bool bnd;
        long long n = nb_index(g, i, j, k, d, bnd);
        if ((msk >> d) & 1) nb[d] = (A)ghost(st, q, c, msk, d, m, wall, (double)qc);
        else if (bnd) nb[d] = (A)bc_ghost(g, d, m, (double)qc);
        else nb[d] = (A)q[n];
    }
}

// Value of component m two cells away across face d of cell (i, j, k), that face being
// open (interior or periodic): the neighbour's own value across its face d, i.e. its
// eq. (q_axis) ghost where that face is blocked, its domain-face ghost at a domain
// face, else the next cell (the far cell of a QUICK stencil).
template <class T>
__device__ inline double far_value(const Geo& g, const Sten& st, const T* q, int m, int i, int j, int k, int d,
                                   const double* wall) {
    const int ax = d >> 1;
    const int n_ax = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
    int co = (ax == 0 ? i : (ax == 1 ? j : k)) + ((d & 1) ? 1 : -1);
    co = co < 0 ? co + n_ax : (co >= n_ax ? co - n_ax : co);
    const int ii = ax == 0 ? co : i, jj = ax == 1 ? co : j, kk = ax == 2 ? co : k;
    const long long n = cidx(g, ii, jj, kk);
    const uint8_t mn = st.mask[n];
    const double qn = (double)q[n];
    if ((mn >> d) & 1) return ghost(st, q, n, mn, d, m, wall, qn);
    bool bnd;
    const long long nn = nb_index(g, ii, jj, kk, d, bnd);
    if (bnd) return bc_ghost(g, d, m, qn);
    return (double)q[nn];
}

// ------------------------------------------------------------------ per-cell forms
//
// The step kernels run in two parts.  A cell is "special" when it has a blocked face or
// lies on a non-periodic domain face (dead-end cells are closed on all six faces): only
// there do ghosts and boundary values enter.  The fast sweeps below compute every other
// cell with the plain 7-point stencil, branch-free, several cells per lane; the per-cell
// forms here then process the context's list of special cells (one thread each) with the
// full ghost and boundary logic, which is the paper's single branch into the dummy-cell
// data (Sec. 2.3.1).  The two parts write disjoint cells.  On grids the fast sweeps do
// not cover (nx not a multiple of their vector width, or the hybrid QUICK face value),
// the per-cell forms run over every cell.

// Coherent structure model (Sec. 2.3): G_ij by central differences, S, W, Q, E,
// F_CS = Q/E, C = C1 |F_CS|^(3/2), nu_t = C dx^2 sqrt(S_ij S_ij).
template <class T>
struct CsmOp {
    Sten st;
    C3<T> u;
    const double* wall;
    T* nut;
    double c1;
    __device__ void operator()(const Geo& g, int i, int j, int k) const {
        const long long c = cidx(g, i, j, k);
        const uint8_t msk = st.mask[c];
        T G[3][3];
        const T inv2dx = (T)(1.0 / (2.0 * g.dx));
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T nb[6];
            T qc = u.p[a][c];
            nbvals<T, T>(g, st, u.p[a], a, i, j, k, c, msk, wall, qc, nb);
#pragma unroll
            for (int b = 0; b < 3; ++b) G[a][b] = (nb[2 * b + 1] - nb[2 * b]) * inv2dx;
        }
        nut[c] = csm_value<T>(G, c1, g.dx);
    }
    template <class TT>
    __device__ static TT csm_value(const TT (&G)[3][3], double c1, double dx) {
        TT SS = 0, WW = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                TT s = (TT)0.5 * (G[a][b] + G[b][a]);
                TT w = (TT)0.5 * (G[a][b] - G[b][a]);
                SS += s * s;
                WW += w * w;
            }
        TT Q = (TT)0.5 * (WW - SS);
        TT E = (TT)0.5 * (WW + SS);
        TT F = E > (TT)0 ? Q / E : (TT)0;
        TT aF = F < (TT)0 ? -F : F;
        TT C = (TT)c1 * aF * sqrt(aF);
        return C * (TT)(dx * dx) * sqrt(SS);
    }
};

// Momentum predictor (Sec. 2.1, explicit Adams-Bashforth form):
// H = -(1/dx) sum_f s U_f (q_c + q_nb)/2 + (1/dx^2) sum_f (nu + nu_t,f)(q_nb - q_c) + g,
// u* = u + dt ((1 + r/2) H - (r/2) H_prev), forward Euler on the first step.  q_nb is the
// eq. (q_axis) ghost behind blocked faces, which realises the direct forcing of
// eq. (forcing_term).  Dead-end cells are frozen at their mean wall velocity.
// The face value is the hybrid of Sec. 3: the central (q_c + q_nb)/2 blended with
// weight `quick` with the QUICK value (Leonard 1979) (6 q_up + 3 q_down - q_farup)/8,
// upstream by the sign of the outward face velocity; the far cell beyond a blocked or
// domain face is the first ghost's line continued, 2 q_nb - q_c.
// With cn set (Crank-Nicolson, eq. (crank-nicolson)) the kernel writes instead the
// right-hand side dt H of the increment system into rhs (dv - u at dead-end cells) and
// u* only at dead-end cells (dv); H goes to hio as in the explicit form.
template <class T>
struct PredictOp {
    Sten st;
    C3<T> u;
    C3<double> U;
    const T* nut;
    V3<T> hio, us, rhs;
    const double* wall;
    double dt, w_now, w_prev, nu, body[3], quick;
    int first, cn;
    __device__ void operator()(const Geo& g, int i, int j, int k) const {
        const T idx = (T)(1.0 / g.dx);
        const T idx2 = (T)(1.0 / (g.dx * g.dx));
        const long long c = cidx(g, i, j, k);
        const uint8_t msk = st.mask[c];
        const T nut_c = nut[c];
        T visc[6];
        T Uf[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            bool bnd;
            const long long n = nb_index(g, i, j, k, d, bnd);
            const bool closed = bnd || ((msk >> d) & 1);
            visc[d] = (T)nu + (closed ? nut_c : (T)0.5 * (nut_c + nut[n]));
            const int ax = d >> 1;
            if (d & 1) {
                Uf[d] = (T)U.p[ax][c];
            } else if (bnd) {
                Uf[d] = g.bc[d] == IBM_BC_INFLOW ? (T)g.uin[ax] : (T)0;
            } else {
                Uf[d] = (T)U.p[ax][n];
            }
        }
        const int nbits = __builtin_popcount((unsigned)msk);
        const bool dead = st.has_dead && nbits >= 5 && ((st.flags[c] >> 14) & 1);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T qc = u.p[m][c];
            T nb[6];
            nbvals<T, T>(g, st, u.p[m], m, i, j, k, c, msk, wall, qc, nb);
            T h = (T)body[m];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const T s = (d & 1) ? (T)1 : (T)-1;
                T qf = (T)0.5 * (qc + nb[d]);
                if (quick != 0.0) {
                    T qq;
                    if (s * Uf[d] > (T)0) {
                        qq = ((T)6 * qc + (T)3 * nb[d] - nb[d ^ 1]) / (T)8;
                    } else {
                        bool bnd;
                        (void)nb_index(g, i, j, k, d, bnd);
                        const T n2 = (bnd || ((msk >> d) & 1)) ? (T)2 * nb[d] - qc
                                                               : (T)far_value(g, st, u.p[m], m, i, j, k, d, wall);
                        qq = ((T)6 * nb[d] + (T)3 * qc - n2) / (T)8;
                    }
                    qf = (T)(1.0 - quick) * qf + (T)quick * qq;
                }
                h = h - s * Uf[d] * qf * idx + visc[d] * (nb[d] - qc) * idx2;
            }
            T v;
            if (first || cn) v = qc + (T)dt * h;
            else v = qc + (T)dt * ((T)w_now * h - (T)w_prev * hio.p[m][c]);
            T b = (T)dt * h;
            if (dead) {
                const uint32_t id0 = st.cut_off[c];
                double acc = 0.0;
                for (int q = 0; q < nbits; ++q) acc += wall ? wall[3 * (long long)(id0 + q) + m] : 0.0;
                v = (T)(acc / (double)nbits);
                b = v - qc;
                h = (T)0;
            }
            if (cn) {
                rhs.p[m][c] = b;
                if (dead) us.p[m][c] = v;
            } else {
                us.p[m][c] = v;
            }
            hio.p[m][c] = h;
        }
    }
};

// normal wall velocity on the +k face of cell c (blocked): mean of the two cuts
// that see the face, one from each side
template <class T>
__device__ inline double wall_face(const Sten& st, long long c, uint8_t msk, long long nb, int k,
                                   const double* wall) {
    if (!wall) return 0.0;
    uint32_t a = cut_id(st, c, msk, 2 * k + 1);
    uint8_t mn = st.mask[nb];
    uint32_t b = cut_id(st, nb, mn, 2 * k);
    return 0.5 * (wall[3 * (long long)a + k] + wall[3 * (long long)b + k]);
}

// Face velocity U* and b = div(U*)/dt (eq. poisson).  U* is the mean of the two
// predicted cell velocities on open faces, the wall normal velocity on blocked faces
// and the boundary value on domain faces.  Each cell also evaluates its -faces, so no
// second pass is needed.
template <class T>
struct RhsOp {
    Sten st;
    C3<T> us;
    V3<double> U;
    double* b;
    const double* wall;
    double dt;
    __device__ void operator()(const Geo& g, int i, int j, int k) const {
        const double idx = 1.0 / g.dx;
        const long long c = cidx(g, i, j, k);
        const uint8_t msk = st.mask[c];
        double div = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double qc = (double)us.p[a][c];
            const int dp = 2 * a + 1, dm = 2 * a;
            bool bp, bm;
            const long long np = nb_index(g, i, j, k, dp, bp);
            const long long nm = nb_index(g, i, j, k, dm, bm);
            double Up, Um;
            if ((msk >> dp) & 1) Up = wall_face<T>(st, c, msk, np, a, wall);
            else if (bp) Up = g.bc[dp] == IBM_BC_INFLOW ? g.uin[a] : (g.bc[dp] == IBM_BC_OUTFLOW ? qc : 0.0);
            else Up = 0.5 * (qc + (double)us.p[a][np]);
            if ((msk >> dm) & 1) Um = wall_face<T>(st, nm, st.mask[nm], c, a, wall);
            else if (bm) Um = g.bc[dm] == IBM_BC_INFLOW ? g.uin[a] : 0.0;
            else Um = 0.5 * ((double)us.p[a][nm] + qc);
            U.p[a][c] = Up;
            div += (Up - Um) * idx;
        }
        b[c] = div / dt;
    }
};

// Correction (eq. correction): U = U* - dt (p_nb - p_c)/dx on open faces, U* + 2 dt p_c/dx
// on outlet faces (p = 0 on the face), unchanged on blocked/inflow/slip faces;
// u = u* - dt (p_E - p_W)/(2 dx) with the Neumann ghost p_c behind blocked, inflow and
// slip faces and the Dirichlet ghost -p_c behind outlet faces.
template <class T>
struct ProjectOp {
    Sten st;
    C3<T> us;
    V3<double> U;
    const double* p;
    V3<T> u;
    double dt;
    __device__ void operator()(const Geo& g, int i, int j, int k) const {
        const double idx = 1.0 / g.dx;
        const long long c = cidx(g, i, j, k);
        const uint8_t msk = st.mask[c];
        const double pc = p[c];
        const bool dead = st.has_dead && __builtin_popcount((unsigned)msk) >= 5 && ((st.flags[c] >> 14) & 1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int dp = 2 * a + 1, dm = 2 * a;
            bool bp, bm;
            const long long np = nb_index(g, i, j, k, dp, bp);
            const long long nm = nb_index(g, i, j, k, dm, bm);
            const bool openp = !bp && !((msk >> dp) & 1);
            const bool openm = !bm && !((msk >> dm) & 1);
            const bool outp = bp && g.bc[dp] == IBM_BC_OUTFLOW;
            const bool outm = bm && g.bc[dm] == IBM_BC_OUTFLOW;
            const double pE = openp ? p[np] : (outp ? -pc : pc);
            const double pW = openm ? p[nm] : (outm ? -pc : pc);
            double Uc = U.p[a][c];
            if (openp) Uc = Uc - dt * (pE - pc) * idx;
            else if (outp) Uc = Uc + 2.0 * dt * pc * idx;
            U.p[a][c] = Uc;
            const double usc = (double)us.p[a][c];
            const double v = dead ? usc : usc - dt * (pE - pW) / (2.0 * g.dx);
            u.p[a][c] = (T)v;
        }
    }
};

// every cell (tile walk with the XCD chunk map)
template <class Op>
__global__ void __launch_bounds__(NT) k_all(Geo g, Op op) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        op(g, i, j, k);
    }
}

// the listed (special) cells, one thread each
template <class Op>
__global__ void __launch_bounds__(NT) k_fix(Geo g, const int32_t* __restrict__ cells, long long n, Op op) {
    for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < n; e += (long long)gridDim.x * NT) {
        const long long c = cells[e];
        const int i = (int)(c % g.nx);
        const int j = (int)((c / g.nx) % g.ny);
        const int k = (int)(c / ((long long)g.nx * g.ny));
        op(g, i, j, k);
    }
}

// ------------------------------------------------------------------ fast sweeps
//
// Work item = (tile of 64 lanes x V cells in x by TY rows, z slab), slab-major with the
// XCD chunk map.  Each lane owns V consecutive cells of one row and walks the slab's
// planes, carrying the planes below and above in registers; x neighbours inside the V
// cells are register shifts, the two outer ones single loads, y neighbours vector loads
// from the L2.  A cell is written only when it is not special.

template <class T, int V>
__device__ inline void vload(const T* __restrict__ p, long long c, T (&o)[V]) {
    constexpr int B = (int)sizeof(T) * V;
    static_assert(B == 8 || B == 16 || B == 32, "vector width");
    if constexpr (B == 8) {
        const uint2 w = *reinterpret_cast<const uint2*>(p + c);
        __builtin_memcpy(o, &w, 8);
    } else if constexpr (B == 16) {
        const uint4 w = *reinterpret_cast<const uint4*>(p + c);
        __builtin_memcpy(o, &w, 16);
    } else {
        const uint4 w0 = *reinterpret_cast<const uint4*>(p + c);
        const uint4 w1 = *reinterpret_cast<const uint4*>(p + c + V / 2);
        __builtin_memcpy(o, &w0, 16);
        __builtin_memcpy(reinterpret_cast<char*>(o) + 16, &w1, 16);
    }
}

// store the cells whose bit is set in keep (all V: one vector store)
template <class T, int V>
__device__ inline void vstore(T* __restrict__ p, long long c, const T (&o)[V], unsigned keep) {
    constexpr unsigned ALL = (1u << V) - 1u;
    constexpr int B = (int)sizeof(T) * V;
    if (keep == ALL) {
        if constexpr (B == 8) {
            uint2 w;
            __builtin_memcpy(&w, o, 8);
            *reinterpret_cast<uint2*>(p + c) = w;
        } else if constexpr (B == 16) {
            uint4 w;
            __builtin_memcpy(&w, o, 16);
            *reinterpret_cast<uint4*>(p + c) = w;
        } else {
            uint4 w0, w1;
            __builtin_memcpy(&w0, o, 16);
            __builtin_memcpy(&w1, reinterpret_cast<const char*>(o) + 16, 16);
            *reinterpret_cast<uint4*>(p + c) = w0;
            *reinterpret_cast<uint4*>(p + c + V / 2) = w1;
        }
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
            if ((keep >> v) & 1u) p[c + v] = o[v];
    }
}

// Column of a fast-sweep work item: V cells (i0 .. i0 + V - 1) of row j, planes z0 .. z1 - 1.
struct VCol {
    int i0, j, z0, z1;
    long long col, ow, oe, os, on;   // row start; cells i0 - 1 and i0 + V; rows j -+ 1 (wrapping)
    bool bw, be, bsn;                // first / last cell on a -x / +x domain face; row on a y domain face
    bool valid;
};

template <int V>
__device__ inline VCol vcol(const Geo& g, long long w, int ntxv, long long tiles, int nzc) {
    VCol z;
    const int zc = (int)(w / tiles);
    const long long t = w % tiles;
    z.i0 = (int)(t % ntxv) * (64 * V) + V * (int)(threadIdx.x % 64);
    z.j = (int)(t / ntxv) * TY + (int)(threadIdx.x / 64);
    z.z0 = (int)((long long)g.nz * zc / nzc);
    z.z1 = (int)((long long)g.nz * (zc + 1) / nzc);
    z.valid = z.i0 < g.nx && z.j < g.ny;
    const int iw = z.i0 == 0 ? g.nx - 1 : z.i0 - 1;
    const int ie = z.i0 + V >= g.nx ? 0 : z.i0 + V;
    const int js = z.j == 0 ? g.ny - 1 : z.j - 1, jn = z.j == g.ny - 1 ? 0 : z.j + 1;
    z.col = (long long)z.i0 + (long long)g.nx * z.j;
    z.ow = (long long)iw - z.i0;
    z.oe = (long long)ie - z.i0;
    z.os = (long long)g.nx * (js - z.j);
    z.on = (long long)g.nx * (jn - z.j);
    z.bw = z.i0 == 0 && g.bc[0] != IBM_BC_PERIODIC;
    z.be = z.i0 + V >= g.nx && g.bc[1] != IBM_BC_PERIODIC;
    z.bsn = (z.j == 0 && g.bc[2] != IBM_BC_PERIODIC) || (z.j == g.ny - 1 && g.bc[3] != IBM_BC_PERIODIC);
    return z;
}

// the lane's cells that are not special in plane k (bit v = cell i0 + v)
template <int V>
__device__ inline unsigned plain_cells(const Geo& g, const VCol& z, const uint8_t* __restrict__ mask, long long c,
                                       int k) {
    if (z.bsn || (k == 0 && g.bc[4] != IBM_BC_PERIODIC) || (k == g.nz - 1 && g.bc[5] != IBM_BC_PERIODIC)) return 0u;
    uint8_t m[V];
    if constexpr (V == 4) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(mask + c);
        __builtin_memcpy(m, &w, 4);
    } else {
        const uint16_t w = *reinterpret_cast<const uint16_t*>(mask + c);
        __builtin_memcpy(m, &w, 2);
    }
    unsigned keep = 0u;
#pragma unroll
    for (int v = 0; v < V; ++v) keep |= (m[v] == 0 ? 1u : 0u) << v;
    if (z.bw) keep &= ~1u;
    if (z.be) keep &= ~(1u << (V - 1));
    return keep;
}

template <int V>
__device__ inline void vcol_range(const Geo& g, int& ntxv, long long& tiles, int& nzc, long long& w0, long long& w1) {
    ntxv = (g.nx + 64 * V - 1) / (64 * V);
    tiles = (long long)ntxv * g.nty;
    nzc = slab_count(g.nz);
    const long long items = tiles * nzc;
    const int nb = gridDim.x;
    const int ch = xcd_chunk(blockIdx.x, nb);
    w0 = items * ch / nb;
    w1 = items * (ch + 1) / nb;
}

template <int V>
inline int vcol_blocks(const Geo& g) {
    const long long items = (long long)((g.nx + 64 * V - 1) / (64 * V)) * g.nty * slab_count(g.nz);
    return (int)(items < MAX_BLOCKS ? items : MAX_BLOCKS);
}

template <class T, int V>
__global__ void __launch_bounds__(NT) k_csm_fast(Geo g, const uint8_t* __restrict__ mask, C3<T> u,
                                                 T* __restrict__ nut, double c1) {
    int ntxv, nzc;
    long long tiles, w0, w1;
    vcol_range<V>(g, ntxv, tiles, nzc, w0, w1);
    const long long plane = (long long)g.nx * g.ny;
    const T inv2dx = (T)(1.0 / (2.0 * g.dx));
    for (long long w = w0; w < w1; ++w) {
        const VCol zc = vcol<V>(g, w, ntxv, tiles, nzc);
        if (!zc.valid) continue;
        const int zb = zc.z0 == 0 ? g.nz - 1 : zc.z0 - 1;
        T qb[3][V], qm[3][V];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            vload<T, V>(u.p[a], zc.col + plane * zb, qb[a]);
            vload<T, V>(u.p[a], zc.col + plane * zc.z0, qm[a]);
        }
        for (int k = zc.z0; k < zc.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = zc.col + plane * k;
            T qt[3][V];
#pragma unroll
            for (int a = 0; a < 3; ++a) vload<T, V>(u.p[a], zc.col + plane * zt, qt[a]);
            const unsigned keep = plain_cells<V>(g, zc, mask, c, k);
            if (keep) {
                T G[V][3][3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const T* q = u.p[a];
                    T ys[V], yn[V];
                    vload<T, V>(q, c + zc.os, ys);
                    vload<T, V>(q, c + zc.on, yn);
                    const T xw = q[c + zc.ow], xe = q[c + zc.oe];
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const T left = v ? qm[a][v - 1] : xw;
                        const T right = v < V - 1 ? qm[a][v + 1] : xe;
                        G[v][a][0] = (right - left) * inv2dx;
                        G[v][a][1] = (yn[v] - ys[v]) * inv2dx;
                        G[v][a][2] = (qt[a][v] - qb[a][v]) * inv2dx;
                    }
                }
                T o[V];
#pragma unroll
                for (int v = 0; v < V; ++v) o[v] = CsmOp<T>::template csm_value<T>(G[v], c1, g.dx);
                vstore<T, V>(nut, c, o, keep);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    qb[a][v] = qm[a][v];
                    qm[a][v] = qt[a][v];
                }
        }
    }
}

// central face value only (the hybrid QUICK value takes the per-cell form everywhere)
template <class T, int V>
__global__ void __launch_bounds__(NT) k_predict_fast(Geo g, const uint8_t* __restrict__ mask, PredictOp<T> op) {
    int ntxv, nzc;
    long long tiles, w0, w1;
    vcol_range<V>(g, ntxv, tiles, nzc, w0, w1);
    const long long plane = (long long)g.nx * g.ny;
    const T idx = (T)(1.0 / g.dx);
    const T idx2 = (T)(1.0 / (g.dx * g.dx));
    for (long long w = w0; w < w1; ++w) {
        const VCol zc = vcol<V>(g, w, ntxv, tiles, nzc);
        if (!zc.valid) continue;
        const int zb = zc.z0 == 0 ? g.nz - 1 : zc.z0 - 1;
        T qb[3][V], qm[3][V], nb_[V], nm_[V];
        double uzb[V];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            vload<T, V>(op.u.p[m], zc.col + plane * zb, qb[m]);
            vload<T, V>(op.u.p[m], zc.col + plane * zc.z0, qm[m]);
        }
        vload<T, V>(op.nut, zc.col + plane * zb, nb_);
        vload<T, V>(op.nut, zc.col + plane * zc.z0, nm_);
        vload<double, V>(op.U.p[2], zc.col + plane * zb, uzb);
        for (int k = zc.z0; k < zc.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = zc.col + plane * k;
            T qt[3][V], nt_[V];
#pragma unroll
            for (int m = 0; m < 3; ++m) vload<T, V>(op.u.p[m], zc.col + plane * zt, qt[m]);
            vload<T, V>(op.nut, zc.col + plane * zt, nt_);
            double uzc[V];
            vload<double, V>(op.U.p[2], c, uzc);
            const unsigned keep = plain_cells<V>(g, zc, mask, c, k);
            if (keep) {
                // face eddy viscosity and face velocities of the V cells, faces 0..5
                T nys[V], nyn[V];
                vload<T, V>(op.nut, c + zc.os, nys);
                vload<T, V>(op.nut, c + zc.on, nyn);
                const T nxw = op.nut[c + zc.ow], nxe = op.nut[c + zc.oe];
                double ux[V], uy[V], uys[V];
                vload<double, V>(op.U.p[0], c, ux);
                vload<double, V>(op.U.p[1], c, uy);
                vload<double, V>(op.U.p[1], c + zc.os, uys);
                const double uxw = op.U.p[0][c + zc.ow];
                T visc[V][6], Uf[V][6];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T nc = nm_[v];
                    const T nn[6] = {v ? nm_[v - 1] : nxw, v < V - 1 ? nm_[v + 1] : nxe, nys[v], nyn[v], nb_[v], nt_[v]};
#pragma unroll
                    for (int d = 0; d < 6; ++d) visc[v][d] = (T)op.nu + (T)0.5 * (nc + nn[d]);
                    Uf[v][0] = (T)(v ? ux[v - 1] : uxw);
                    Uf[v][1] = (T)ux[v];
                    Uf[v][2] = (T)uys[v];
                    Uf[v][3] = (T)uy[v];
                    Uf[v][4] = (T)uzb[v];
                    Uf[v][5] = (T)uzc[v];
                }
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const T* q = op.u.p[m];
                    T ys[V], yn[V], hp[V];
                    vload<T, V>(q, c + zc.os, ys);
                    vload<T, V>(q, c + zc.on, yn);
                    const T xw = q[c + zc.ow], xe = q[c + zc.oe];
                    if (!(op.first || op.cn)) vload<T, V>(op.hio.p[m], c, hp);
                    T ov[V], oh[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const T qc = qm[m][v];
                        const T nb[6] = {v ? qm[m][v - 1] : xw, v < V - 1 ? qm[m][v + 1] : xe, ys[v], yn[v],
                                         qb[m][v], qt[m][v]};
                        T h = (T)op.body[m];
#pragma unroll
                        for (int d = 0; d < 6; ++d) {
                            const T s = (d & 1) ? (T)1 : (T)-1;
                            const T qf = (T)0.5 * (qc + nb[d]);
                            h = h - s * Uf[v][d] * qf * idx + visc[v][d] * (nb[d] - qc) * idx2;
                        }
                        if (op.cn) ov[v] = (T)op.dt * h;
                        else if (op.first) ov[v] = qc + (T)op.dt * h;
                        else ov[v] = qc + (T)op.dt * ((T)op.w_now * h - (T)op.w_prev * hp[v]);
                        oh[v] = h;
                    }
                    vstore<T, V>(op.cn ? op.rhs.p[m] : op.us.p[m], c, ov, keep);
                    vstore<T, V>(op.hio.p[m], c, oh, keep);
                }
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    qb[m][v] = qm[m][v];
                    qm[m][v] = qt[m][v];
                }
                nb_[v] = nm_[v];
                nm_[v] = nt_[v];
                uzb[v] = uzc[v];
            }
        }
    }
}

template <class T, int V>
__global__ void __launch_bounds__(NT) k_rhs_fast(Geo g, const uint8_t* __restrict__ mask, RhsOp<T> op) {
    int ntxv, nzc;
    long long tiles, w0, w1;
    vcol_range<V>(g, ntxv, tiles, nzc, w0, w1);
    const long long plane = (long long)g.nx * g.ny;
    const double idx = 1.0 / g.dx;
    for (long long w = w0; w < w1; ++w) {
        const VCol zc = vcol<V>(g, w, ntxv, tiles, nzc);
        if (!zc.valid) continue;
        const int zb = zc.z0 == 0 ? g.nz - 1 : zc.z0 - 1;
        T wb[V], wm[V];
        vload<T, V>(op.us.p[2], zc.col + plane * zb, wb);
        vload<T, V>(op.us.p[2], zc.col + plane * zc.z0, wm);
        for (int k = zc.z0; k < zc.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = zc.col + plane * k;
            T wt[V];
            vload<T, V>(op.us.p[2], zc.col + plane * zt, wt);
            const unsigned keep = plain_cells<V>(g, zc, mask, c, k);
            if (keep) {
                double div[V], Ux[V], Uy[V], Uz[V];
                T qx[V], qy[V], qys[V], qyn[V];
                vload<T, V>(op.us.p[0], c, qx);
                const double xw = (double)op.us.p[0][c + zc.ow], xe = (double)op.us.p[0][c + zc.oe];
                vload<T, V>(op.us.p[1], c, qy);
                vload<T, V>(op.us.p[1], c + zc.os, qys);
                vload<T, V>(op.us.p[1], c + zc.on, qyn);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    double qc = (double)qx[v];
                    double Up = 0.5 * (qc + (v < V - 1 ? (double)qx[v + 1] : xe));
                    double Um = 0.5 * ((v ? (double)qx[v - 1] : xw) + qc);
                    Ux[v] = Up;
                    div[v] = 0.0;
                    div[v] += (Up - Um) * idx;
                    qc = (double)qy[v];
                    Up = 0.5 * (qc + (double)qyn[v]);
                    Um = 0.5 * ((double)qys[v] + qc);
                    Uy[v] = Up;
                    div[v] += (Up - Um) * idx;
                    qc = (double)wm[v];
                    Up = 0.5 * (qc + (double)wt[v]);
                    Um = 0.5 * ((double)wb[v] + qc);
                    Uz[v] = Up;
                    div[v] += (Up - Um) * idx;
                    div[v] = div[v] / op.dt;
                }
                vstore<double, V>(op.U.p[0], c, Ux, keep);
                vstore<double, V>(op.U.p[1], c, Uy, keep);
                vstore<double, V>(op.U.p[2], c, Uz, keep);
                vstore<double, V>(op.b, c, div, keep);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                wb[v] = wm[v];
                wm[v] = wt[v];
            }
        }
    }
}

template <class T, int V>
__global__ void __launch_bounds__(NT) k_project_fast(Geo g, const uint8_t* __restrict__ mask, ProjectOp<T> op) {
    int ntxv, nzc;
    long long tiles, w0, w1;
    vcol_range<V>(g, ntxv, tiles, nzc, w0, w1);
    const long long plane = (long long)g.nx * g.ny;
    const double idx = 1.0 / g.dx;
    for (long long w = w0; w < w1; ++w) {
        const VCol zc = vcol<V>(g, w, ntxv, tiles, nzc);
        if (!zc.valid) continue;
        const int zb = zc.z0 == 0 ? g.nz - 1 : zc.z0 - 1;
        double pb[V], pm[V];
        vload<double, V>(op.p, zc.col + plane * zb, pb);
        vload<double, V>(op.p, zc.col + plane * zc.z0, pm);
        for (int k = zc.z0; k < zc.z1; ++k) {
            const int zt = k == g.nz - 1 ? 0 : k + 1;
            const long long c = zc.col + plane * k;
            double pt[V];
            vload<double, V>(op.p, zc.col + plane * zt, pt);
            const unsigned keep = plain_cells<V>(g, zc, mask, c, k);
            if (keep) {
                double ps[V], pn[V];
                vload<double, V>(op.p, c + zc.os, ps);
                vload<double, V>(op.p, c + zc.on, pn);
                const double pw = op.p[c + zc.ow], pe = op.p[c + zc.oe];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    double Ua[V];
                    T ua[V];
                    vload<double, V>(op.U.p[a], c, Ua);
                    vload<T, V>(op.us.p[a], c, ua);
                    double Uo[V];
                    T uo[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const double pc = pm[v];
                        const double pE = a == 0 ? (v < V - 1 ? pm[v + 1] : pe) : (a == 1 ? pn[v] : pt[v]);
                        const double pW = a == 0 ? (v ? pm[v - 1] : pw) : (a == 1 ? ps[v] : pb[v]);
                        double Uc = Ua[v];
                        Uc = Uc - op.dt * (pE - pc) * idx;
                        Uo[v] = Uc;
                        const double usc = (double)ua[v];
                        uo[v] = (T)(usc - op.dt * (pE - pW) / (2.0 * g.dx));
                    }
                    vstore<double, V>(op.U.p[a], c, Uo, keep);
                    vstore<T, V>(op.u.p[a], c, uo, keep);
                }
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                pb[v] = pm[v];
                pm[v] = pt[v];
            }
        }
    }
}

// ||div U||_2^2 and max |div U| (FP64 divergence check); per-block sums and maxima,
// combined by the last block in block order
__global__ void __launch_bounds__(NT) k_div(Geo g, C3<double> U, double* partials) {
    __shared__ double sh[NT];
    __shared__ double shm[NT];
    long long t0, t1;
    tile_range(g, t0, t1);
    __shared__ double shu[NT];
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        double div = 0.0;
        for (int a = 0; a < 3; ++a) {
            bool bm;
            long long nm = nb_index(g, i, j, k, 2 * a, bm);
            double Um = bm ? (g.bc[2 * a] == IBM_BC_INFLOW ? g.uin[a] : 0.0) : U.p[a][nm];
            double Uc = U.p[a][c];
            div += (Uc - Um) / g.dx;
            v2 = fmax(v2, fmax(fabs(Uc), fabs(Um)));
        }
        v0 += div * div;
        v1 = fmax(v1, fabs(div));
    }
    sh[threadIdx.x] = v0;
    shm[threadIdx.x] = v1;
    shu[threadIdx.x] = v2;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[threadIdx.x] += sh[threadIdx.x + s];
            shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + s]);
            shu[threadIdx.x] = fmax(shu[threadIdx.x], shu[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = sh[0];
        partials[MAX_BLOCKS + blockIdx.x] = shm[0];
        partials[2 * MAX_BLOCKS + blockIdx.x] = shu[0];
    }
}

// one block: sum of the squared divergence, max |div|, max |U| over the block partials
__global__ void __launch_bounds__(NT) k_div_final(const double* partials, int nparts, double* out) {
    __shared__ double sh[NT];
    __shared__ double shm[NT];
    __shared__ double shu[NT];
    double acc = 0.0, mx = 0.0, mu = 0.0;
    for (int b = threadIdx.x; b < nparts; b += NT) {
        acc += partials[b];
        mx = fmax(mx, partials[MAX_BLOCKS + b]);
        mu = fmax(mu, partials[2 * MAX_BLOCKS + b]);
    }
    sh[threadIdx.x] = acc;
    shm[threadIdx.x] = mx;
    shu[threadIdx.x] = mu;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[threadIdx.x] += sh[threadIdx.x + s];
            shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + s]);
            shu[threadIdx.x] = fmax(shu[threadIdx.x], shu[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0];
        out[1] = shm[0];
        out[2] = shu[0];
    }
}

// Initial state: u = u0; U = u0 on open/periodic/outflow faces, mean wall normal
// velocity on blocked faces, boundary value on inflow/slip faces; p = 0; H = 0.
template <class T>
__global__ void __launch_bounds__(NT) k_init(Geo g, Sten st, V3<T> u, V3<double> U, double* p, V3<T> h,
                                             double u0x, double u0y, double u0z, const double* wall) {
    long long t0, t1;
    tile_range(g, t0, t1);
    const double u0[3] = {u0x, u0y, u0z};
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        uint8_t msk = st.mask[c];
        for (int a = 0; a < 3; ++a) {
            u.p[a][c] = (T)u0[a];
            h.p[a][c] = (T)0;
            int dp = 2 * a + 1;
            bool bp;
            long long np = nb_index(g, i, j, k, dp, bp);
            double v = u0[a];
            if (bp && g.bc[dp] == IBM_BC_INFLOW) v = g.uin[a];
            else if (bp && g.bc[dp] == IBM_BC_SLIP) v = 0.0;
            if ((msk >> dp) & 1) v = wall_face<T>(st, c, msk, np, a, wall);
            U.p[a][c] = v;
        }
        p[c] = 0.0;
    }
}

__global__ void k_cut_points(Geo g, long long ncut, const int32_t* cell, const uint8_t* dir, const double* theta,
                             double* X) {
    for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < ncut;
         id += (long long)gridDim.x * blockDim.x) {
        long long c = cell[id];
        int i = (int)(c % g.nx);
        int j = (int)((c / g.nx) % g.ny);
        int k = (int)(c / ((long long)g.nx * g.ny));
        double x = g.ox + ((double)i + 0.5) * g.dx;
        double y = g.oy + ((double)j + 0.5) * g.dx;
        double z = g.oz + ((double)k + 0.5) * g.dx;
        int d = dir[id];
        double s = (d & 1) ? 1.0 : -1.0;
        double off = s * theta[id] * g.dx;
        int ax = d >> 1;
        if (ax == 0) x += off; else if (ax == 1) y += off; else z += off;
        X[3 * id] = x;
        X[3 * id + 1] = y;
        X[3 * id + 2] = z;
    }
}

// Force on the surface: F_p += dx^2 s p_c e_k, F_v -= dx^2 (nu + nu_t,c)(q_GC - q_c)/dx,
// summed over the cut list in a fixed order.
template <class T>
__global__ void __launch_bounds__(NT) k_forces(long long ncut, const int32_t* cell, const uint8_t* dir,
                                               const double* a_ib, const double* a_c, const double* a_o,
                                               const int32_t* opp, C3<T> u, const double* p, const T* nut,
                                               double nu, double dx, const double* wall, double* partials,
                                               int pstride) {
    __shared__ double sh[6 * NT];
    double v[6] = {0, 0, 0, 0, 0, 0};
    const double A = dx * dx;
    long long per = (ncut + gridDim.x - 1) / gridDim.x;
    long long b0 = per * blockIdx.x, b1 = b0 + per < ncut ? b0 + per : ncut;
    for (long long id = b0 + threadIdx.x; id < b1; id += NT) {
        long long c = cell[id];
        int d = dir[id];
        int ax = d >> 1;
        double s = (d & 1) ? 1.0 : -1.0;
        v[ax] += s * p[c] * A;
        double vis = nu + (nut ? (double)nut[c] : 0.0);
        int32_t o = opp[id];
        for (int m = 0; m < 3; ++m) {
            double qc = (double)u.p[m][c];
            double w = wall ? wall[3 * id + m] : 0.0;
            double gh = a_ib[id] * w + a_c[id] * qc;
            if (o >= 0) gh += a_o[id] * (double)u.p[m][o];
            v[3 + m] -= vis * (gh - qc) / dx * A;
        }
    }
    block_reduce<6>(v, sh);
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) partials[a * pstride + blockIdx.x] = v[a];
}

// sum a (0..5) of the block partials (stride pstride between sums) in block order
__global__ void __launch_bounds__(NT) k_sum6(const double* partials, int nparts, int pstride, double* out) {
    __shared__ double sh[6 * NT];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nparts; b += NT)
        for (int a = 0; a < 6; ++a) v[a] += partials[a * pstride + b];
    block_reduce<6>(v, sh);
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) out[a] = v[a];
}

// Mean removal on every enclosed component: one block per component, fixed order.
__global__ void __launch_bounds__(NT) k_remove_means(const int32_t* cells, const long long* start, double* a) {
    __shared__ double sh[NT];
    long long s0 = start[blockIdx.x], s1 = start[blockIdx.x + 1];
    double v[1] = {0.0};
    for (long long q = s0 + threadIdx.x; q < s1; q += NT) v[0] += a[cells[q]];
    block_reduce<1>(v, sh);
    double mean = v[0] / (double)(s1 - s0);
    for (long long q = s0 + threadIdx.x; q < s1; q += NT) a[cells[q]] -= mean;
}

template <class T>
__global__ void k_copy(const T* a, T* b, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <class T>
__global__ void k_zero(T* a, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = (T)0;
}

// vector width of the fast sweeps: 16 bytes of cell-field type per lane
template <class T>
constexpr int vwidth() {
    return sizeof(T) == 4 ? 4 : 2;
}

inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// the fast sweeps need nx divisible by their width, aligned cell fields (T) and 16-byte
// aligned double fields, and the special-cell list of the stencil build
template <class T>
bool fast_ok(const ibm_ctx* c, std::initializer_list<const void*> tf, std::initializer_list<const void*> df) {
    constexpr int V = vwidth<T>();
    if (c->geo.nx % V != 0 || !c->spec_ready) return false;
    for (const void* p : tf)
        if (!aligned(p, sizeof(T) * V)) return false;
    for (const void* p : df)
        if (!aligned(p, 16)) return false;
    return aligned(c->mask, 4);
}

template <class Op>
void fix_special(const ibm_ctx* c, const Op& op, hipStream_t s) {
    if (c->nspec == 0) return;
    const long long nbk = (c->nspec + NT - 1) / NT;
    k_fix<Op><<<(int)(nbk < 16384 ? nbk : 16384), NT, 0, s>>>(c->geo, c->spec_cells, c->nspec, op);
}

template <class T>
int predict_t(ibm_ctx* c, void** u, double** U, void** h, const double* wall, const ibm_step_params* prm,
              hipStream_t s) {
    constexpr int V = vwidth<T>();
    const Geo& g = c->geo;
    Sten st = sten_of(c);
    C3<T> uu{{(const T*)u[0], (const T*)u[1], (const T*)u[2]}};
    T* nut = (T*)c->nut;
    const bool fast = fast_ok<T>(c, {u[0], u[1], u[2], h[0], h[1], h[2], nut, c->ustar[0], c->ustar[1], c->ustar[2]},
                                 {U[0], U[1], U[2]});
    if (prm->csm_on) {
        const CsmOp<T> op{st, uu, wall, nut, prm->c1};
        if (fast) {
            k_csm_fast<T, V><<<vcol_blocks<V>(g), NT, 0, s>>>(g, c->mask, uu, nut, prm->c1);
            fix_special(c, op, s);
        } else {
            k_all<CsmOp<T>><<<grid_blocks(g), NT, 0, s>>>(g, op);
        }
    } else {
        k_zero<T><<<2048, 256, 0, s>>>(nut, c->N);
    }
    c->nut_valid = true;
    C3<double> UU{{U[0], U[1], U[2]}};
    V3<T> hh{{(T*)h[0], (T*)h[1], (T*)h[2]}};
    V3<T> us{{(T*)c->ustar[0], (T*)c->ustar[1], (T*)c->ustar[2]}};
    // variable-step Adams-Bashforth weights, r = dt / dt_prev
    const double r = prm->dt_prev > 0.0 ? prm->dt / prm->dt_prev : 1.0;
    const bool cn = prm->scheme == IBM_SCHEME_CN;
    V3<T> rhs{{nullptr, nullptr, nullptr}};
    if (cn) {
        // the increment's right-hand side goes where the solve keeps x (its initial guess)
        T* x = (T*)c->cn_ws;
        for (int a = 0; a < 3; ++a) rhs.p[a] = x + (long long)a * c->N;
    }
    const PredictOp<T> op{st, uu, UU, (const T*)nut, hh, us, rhs, wall, prm->dt, 1.0 + 0.5 * r, 0.5 * r, prm->nu,
                          {prm->body_force[0], prm->body_force[1], prm->body_force[2]}, prm->quick,
                          prm->step == 0 ? 1 : 0, cn ? 1 : 0};
    const bool fast_p = fast && prm->quick == 0.0 && (!cn || aligned(rhs.p[0], sizeof(T) * V));
    // both parts of the predictor are timed together (slot TK_PREDICT)
    timing_begin(c, TK_PREDICT, s);
    if (fast_p) {
        k_predict_fast<T, V><<<vcol_blocks<V>(g), NT, 0, s>>>(g, c->mask, op);
        fix_special(c, op, s);
    } else {
        k_all<PredictOp<T>><<<grid_blocks(g), NT, 0, s>>>(g, op);
    }
    timing_end(c, TK_PREDICT, s);
    IBM_HIP(hipGetLastError());   // its events are collected after the solve's next synchronisation
    return IBM_OK;
}

template <class T>
int rhs_t(ibm_ctx* c, double** U, const double* wall, double dt, hipStream_t s) {
    constexpr int V = vwidth<T>();
    const Geo& g = c->geo;
    C3<T> us{{(const T*)c->ustar[0], (const T*)c->ustar[1], (const T*)c->ustar[2]}};
    V3<double> UU{{U[0], U[1], U[2]}};
    const RhsOp<T> op{sten_of(c), us, UU, c->b, wall, dt};
    if (fast_ok<T>(c, {c->ustar[0], c->ustar[1], c->ustar[2]}, {U[0], U[1], U[2], c->b})) {
        k_rhs_fast<T, V><<<vcol_blocks<V>(g), NT, 0, s>>>(g, c->mask, op);
        fix_special(c, op, s);
    } else {
        k_all<RhsOp<T>><<<grid_blocks(g), NT, 0, s>>>(g, op);
    }
    IBM_HIP(hipGetLastError());
    return remove_means(c, c->b, s);
}

template <class T>
int project_t(ibm_ctx* c, void** u, double** U, const double* p, double dt, hipStream_t s) {
    constexpr int V = vwidth<T>();
    const Geo& g = c->geo;
    C3<T> us{{(const T*)c->ustar[0], (const T*)c->ustar[1], (const T*)c->ustar[2]}};
    V3<double> UU{{U[0], U[1], U[2]}};
    V3<T> uu{{(T*)u[0], (T*)u[1], (T*)u[2]}};
    const ProjectOp<T> op{sten_of(c), us, UU, p, uu, dt};
    if (fast_ok<T>(c, {c->ustar[0], c->ustar[1], c->ustar[2], u[0], u[1], u[2]}, {U[0], U[1], U[2], p})) {
        k_project_fast<T, V><<<vcol_blocks<V>(g), NT, 0, s>>>(g, c->mask, op);
        fix_special(c, op, s);
    } else {
        k_all<ProjectOp<T>><<<grid_blocks(g), NT, 0, s>>>(g, op);
    }
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

template <class T>
int init_t(ibm_ctx* c, void** u, double** U, double* p, void** h, const double* u0, const double* wall,
           hipStream_t s) {
    const Geo& g = c->geo;
    V3<T> uu{{(T*)u[0], (T*)u[1], (T*)u[2]}};
    V3<T> hh{{(T*)h[0], (T*)h[1], (T*)h[2]}};
    V3<double> UU{{U[0], U[1], U[2]}};
    k_init<T><<<grid_blocks(g), NT, 0, s>>>(g, sten_of(c), uu, UU, p, hh, u0[0], u0[1], u0[2], wall);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

// blocks of the force reduction: one cut per thread, at most FORCE_BLOCKS blocks
constexpr int FORCE_BLOCKS = 1024;
inline int force_blocks(long long ncut) {
    const long long nbk = (ncut + NT - 1) / NT;
    return (int)(nbk < FORCE_BLOCKS ? nbk : FORCE_BLOCKS);
}

// Block partials of the allocation-free force entry point (ibm_forces_noalloc): six
// sums x FORCE_BLOCKS blocks, 48 KiB per GPU for the life of the process.  Host code
// never uses this name as an address: force_scratch_init stores each device's own
// address of the array (hipGetSymbolAddress) and the launches take that pointer.
static __device__ __align__(256) double scratch[6 * FORCE_BLOCKS];
constexpr int SCRATCH_DEVICES = 64;
static double* g_scratch_ptr[SCRATCH_DEVICES];
static std::mutex g_scratch_mu;

template <class T>
int forces_t(ibm_ctx* c, void* const* u, const double* p, const void* nut, double nu, const double* wall,
             double* out, hipStream_t s) {
    C3<T> uu{{(const T*)u[0], (const T*)u[1], (const T*)u[2]}};
    const T* nt = nut ? (const T*)nut : (c->nut_valid ? (const T*)c->nut : nullptr);
    if (c->ncut == 0) {
        for (int a = 0; a < 6; ++a) out[a] = 0.0;
        return IBM_OK;
    }
    const int nb = force_blocks(c->ncut);
    k_forces<T><<<nb, NT, 0, s>>>(c->ncut, c->cut_cell, c->cut_dir, c->a_ib, c->a_c, c->a_o, c->cut_opp, uu, p, nt,
                                  nu, c->geo.dx, wall, c->partials, MAX_BLOCKS);
    k_sum6<<<1, NT, 0, s>>>(c->partials, nb, MAX_BLOCKS, c->red);
    IBM_HIP(hipGetLastError());
    IBM_HIP(hipMemcpyAsync(c->h_red, c->red, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    for (int a = 0; a < 6; ++a) out[a] = c->h_red[a];
    return IBM_OK;
}

}  // namespace

int remove_means(ibm_ctx* c, double* a, hipStream_t s) {
    if (c->ncomp <= 0) return IBM_OK;
    k_remove_means<<<c->ncomp, NT, 0, s>>>(c->enc_cells, c->comp_start, a);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int cut_points_run(ibm_ctx* c, double* xyz, hipStream_t s) {
    if (c->ncut == 0) return IBM_OK;
    long long nbk = (c->ncut + 255) / 256;
    int nb = (int)(nbk < 4096 ? nbk : 4096);
    k_cut_points<<<nb, 256, 0, s>>>(c->geo, c->ncut, c->cut_cell, c->cut_dir, c->cut_theta, xyz);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int init_state_run(ibm_ctx* c, void** u, double** U, double* p, void** h, const double* u0, const double* wall,
                   hipStream_t s) {
    return c->precision == IBM_FP64 ? init_t<double>(c, u, U, p, h, u0, wall, s)
                                    : init_t<float>(c, u, U, p, h, u0, wall, s);
}

int step_predict(ibm_ctx* c, void** u, double** U, void** h, const double* wall, const ibm_step_params* prm,
                 hipStream_t s) {
    return c->precision == IBM_FP64 ? predict_t<double>(c, u, U, h, wall, prm, s)
                                    : predict_t<float>(c, u, U, h, wall, prm, s);
}

int step_rhs(ibm_ctx* c, double** U, const double* wall, double dt, hipStream_t s) {
    return c->precision == IBM_FP64 ? rhs_t<double>(c, U, wall, dt, s) : rhs_t<float>(c, U, wall, dt, s);
}

int step_project(ibm_ctx* c, void** u, double** U, const double* p, double dt, hipStream_t s) {
    return c->precision == IBM_FP64 ? project_t<double>(c, u, U, p, dt, s) : project_t<float>(c, u, U, p, dt, s);
}

int divergence_norms(ibm_ctx* c, double** U, double* l2, double* linf, double* umax, hipStream_t s) {
    C3<double> UU{{U[0], U[1], U[2]}};
    const int nb = grid_blocks(c->geo);
    k_div<<<nb, NT, 0, s>>>(c->geo, UU, c->partials);
    k_div_final<<<1, NT, 0, s>>>(c->partials, nb, c->red);
    IBM_HIP(hipGetLastError());
    IBM_HIP(hipMemcpyAsync(c->h_red, c->red, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    *l2 = sqrt(c->h_red[0]);
    *linf = c->h_red[1];
    *umax = c->h_red[2];
    return IBM_OK;
}

int forces_run(ibm_ctx* c, void* const* u, const double* p, const void* nut, double nu, const double* wall,
               double* out, hipStream_t s) {
    return c->precision == IBM_FP64 ? forces_t<double>(c, u, p, nut, nu, wall, out, s)
                                    : forces_t<float>(c, u, p, nut, nu, wall, out, s);
}

// Resolves the current device's address of the force scratch array, once per device
// (called by ibm_create with the context's device current).
int force_scratch_init(int device) {
    if (device < 0 || device >= SCRATCH_DEVICES) {
        set_error("force scratch: device index beyond the supported range");
        return IBM_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return IBM_OK;
    void* ptr = nullptr;
    IBM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = static_cast<double*>(ptr);
    return IBM_OK;
}

// ibm_forces with the block partials in the per-device scratch array and the six sums
// left on the device (out_dev); no allocation, no host synchronisation.  Same launch
// shape and summation order as forces_t, so the sums are bit-identical.
template <class T>
static int forces_noalloc_t(ibm_ctx* c, void* const* u, const double* p, const void* nut, double nu,
                            const double* wall, double* out_dev, hipStream_t s) {
    double* part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        part = g_scratch_ptr[c->device];
    }
    if (!part) {
        set_error("ibm_forces_noalloc: force scratch not resolved for this device");
        return IBM_ERR_ARG;
    }
    C3<T> uu{{(const T*)u[0], (const T*)u[1], (const T*)u[2]}};
    const T* nt = nut ? (const T*)nut : (c->nut_valid ? (const T*)c->nut : nullptr);
    const int nb = force_blocks(c->ncut);
    if (nb > FORCE_BLOCKS) {
        set_error("ibm_forces_noalloc: more block partials than the scratch array holds");
        return IBM_ERR_ARG;
    }
    if (nb > 0)
        k_forces<T><<<nb, NT, 0, s>>>(c->ncut, c->cut_cell, c->cut_dir, c->a_ib, c->a_c, c->a_o, c->cut_opp, uu, p,
                                      nt, nu, c->geo.dx, wall, part, FORCE_BLOCKS);
    k_sum6<<<1, NT, 0, s>>>(part, nb, FORCE_BLOCKS, out_dev);   // nb = 0 writes zeros
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int forces_noalloc_run(ibm_ctx* c, void* const* u, const double* p, const void* nut, double nu,
                       const double* wall, double* out_dev, hipStream_t s) {
    return c->precision == IBM_FP64 ? forces_noalloc_t<double>(c, u, p, nut, nu, wall, out_dev, s)
                                    : forces_noalloc_t<float>(c, u, p, nut, nu, wall, out_dev, s);
}

int copy_cells(ibm_ctx* c, const void* src, void* dst, bool is_double, hipStream_t s) {
    if (is_double) k_copy<double><<<2048, 256, 0, s>>>((const double*)src, (double*)dst, c->N);
    else k_copy<float><<<2048, 256, 0, s>>>((const float*)src, (float*)dst, c->N);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace ibm
