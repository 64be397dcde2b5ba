// Internal declarations shared by the gfx950 kernels and the C ABI host code.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>

#include "ibm.h"

namespace ibm {

constexpr int TX = 64;          // tile width in x (one wavefront)
constexpr int TY = 4;           // tile height in y
constexpr int NT = TX * TY;     // threads per block for cell kernels
constexpr int MAX_BLOCKS = 8192;  // cap for grid-stride kernels with reductions
constexpr int NXCD = 8;         // gfx950: 8 XCDs, each with its own L2

// Per-launch geometry of the grid and the boundary kinds, passed by value.
struct Geo {
    int nx, ny, nz;
    int ntx, nty;               // tiles per axis
    long long ntiles;
    double dx;
    double ox, oy, oz;
    int bc[6];
    double uin[3];
    int nblocks;                // launched blocks (grid-stride over tiles)
};

struct Solver {                 // device-resident scalars of the Krylov loops
    double fnorm2;              // ||f||^2 of the current solve
    double tol2;                // tol^2 * fnorm2
    double rz, rz_new, rr, dq, alpha, beta;
    double bnorm2;              // <b,b> of the current solve
    double r64norm2;            // <r,r> of the FP64 residual at the last init sweep
    int converged;
    int iters;
    int nan_seen;
    int stop_it;                // iteration at which the solve stopped (STOP_NONE while running)
};

// The kernels of a Krylov loop decide to stop inside a launch (every block sums the same
// partials and so takes the same decision), and the launch that decides still has work
// to finish in all its blocks (the last x update).  A block must therefore never skip
// because of a flag written by its own launch: block 0 records the iteration of the
// stopping launch in stop_it, and a kernel of iteration `it` skips only when the solve
// stopped at an earlier iteration (stop_it < gate, gate = it for kernels that run up to
// and including the stop test of iteration it, it + 1 for the ones after it).  A value
// written by the current launch is never below its gate.
constexpr int STOP_NONE = 0x7fffffff;
__device__ inline bool stopped_before(const Solver* sv, int gate) {
    return sv->stop_it < gate;
}

// Device-resident state of the batched BiCGStab of the Crank-Nicolson predictor (one
// system per velocity component).  Scalars of iteration it live in entry [it & 1]:
// a pass reads the previous iteration's entry while its block 0 writes the current one.
struct CnState {
    double tol2[3];             // tol^2 <b,b> per component
    double bb[3];               // <b,b>
    double rho[2][3];           // <r0, r_it>
    double alpha[2][3];
    double omega[2][3];
    int active[2][3];           // component still iterating in iteration it
    int sconv[2][3];            // converged at the half step of iteration it (||s|| small)
    int iters[3];               // iterations made, set when a component stops
    int status;                 // CN_* below
    int done;                   // every component stopped: later passes return at once
};
enum { CN_RUNNING = 0, CN_CONVERGED = 1, CN_MAXITER = 2, CN_BREAKDOWN = 3, CN_NAN = 4 };
constexpr int TK_SLOTS_MAX = 10;  // timed kernel slots (the TK_* launch slots)

}  // namespace ibm

struct ibm_ctx {
    int device;
    int precision;
    ibm::Geo geo;
    long long N;
    // tagging output kept for the stencil build
    // tagging kept for the stencil build: blocked bits (padded 4-byte words, one byte
    // per cell) and the compact theta list, one entry per blocked (cell, dir) in cell
    // then direction order, tag_off[c] = index of cell c's first entry
    uint32_t* tagmask;
    uint32_t* tag_off;
    double* tag_list;
    long long tag_cap;      // entries tag_list holds
    long long tag_ncut;     // entries in use
    bool tagged;
    // stencil
    uint8_t* mask;          // effective blocked bits
    uint8_t* pcode;         // pressure operator code: bits 0-5 open faces, bits 6-7 outlet faces
    uint16_t* flags;
    int32_t* label;
    uint32_t* cut_off;      // exclusive prefix of popcount(mask)
    long long ncut;
    long long ncut_cap;
    int32_t* cut_cell;
    uint8_t* cut_dir;
    double* cut_theta;
    double* a_ib;
    double* a_c;
    double* a_o;
    int32_t* cut_opp;
    int ncomp;              // enclosed components
    long long nenc;         // cells in enclosed components
    int32_t* enc_cells;     // sorted by (component, cell)
    long long* comp_start;  // ncomp + 1
    long long enc_cap;
    int comp_cap;
    int has_dead;
    bool stencil_ready;
    // cells with a blocked face or on a non-periodic domain face, in cell order: the step
    // kernels give them the full ghost and boundary treatment after a plain sweep
    int32_t* spec_cells;
    long long nspec;
    long long spec_cap;
    bool spec_ready;
    // per-step workspace
    void* ustar[3];
    void* nut;
    double* b;
    double* bwork;
    double* r;
    double* d;
    double* q;
    double* zbuf;           // M^-1 r of the conjugate-gradient loop
    double* x64;            // FP64 scratch (refinement / fallback)
    float* r32;             // mixed: inner FCG vectors
    float* z32;
    float* d32;
    float* q32;
    float* e32;
    float* zprev32;
    double* partials;       // 16 * MAX_BLOCKS (16 reduction slots)
    unsigned int* counter;  // last-block tickets
    ibm::Solver* solver;    // device scalars
    ibm::Solver* h_solver;  // pinned host mirror
    double* h_red;          // pinned host scalars
    double* red;            // device reduction outputs (8 doubles)
    void* cnn;              // preconditioner network (IBM_SOLVER_FCG_CNN), not owned
    int last_iters;         // iterations of the previous FP64 solve (batch sizing)
    int last_iters_inner;   // iterations of the previous FP32 correction solve
    bool nut_valid;
    // optional per-kernel event timing of the Krylov sweeps (ibm_timing_enable)
    int timing_on;
    int ev_cap;             // event pairs per timed kernel
    int ev_used[ibm::TK_SLOTS_MAX];
    hipEvent_t* ev[ibm::TK_SLOTS_MAX];  // 2 * ev_cap events per timed kernel
    double t_ms[ibm::TK_SLOTS_MAX];     // accumulated kernel time
    long long t_launches[ibm::TK_SLOTS_MAX];
    long long t_real_iters; // iterations that did work (the rest exit at once)
    // Crank-Nicolson predictor workspace, allocated by its first use: six vectors
    // (x, r, r0, p, v, t) of three components of the cell type
    void* cn_ws;
    double* cn_part;        // 21 * MAX_BLOCKS partial sums
    ibm::CnState* cn_state;
    ibm::CnState* h_cn_state;  // pinned host mirror
    int cn_last_iters;      // iterations of the previous momentum solve (batch sizing)
    // triangle bins of the near-field force's thin-plate filter (grow-only, first use)
    long long* bin_count;   // 2 * (bins + 1): counts / fill cursor, then offsets
    int* bin_ids;
    uint8_t* bin_occ;       // 24 crossing flags per triangle
    char* bin_tmp;          // scan workspace
    long long bin_cap, bin_ids_cap, bin_occ_cap, bin_tmp_cap;
    // optional progress hook, called at the solver's host convergence polls
    ibm_progress_fn progress;
    void* progress_user;
    long long progress_iters; // iterations made by the current solve before this segment
};

namespace ibm {

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define IBM_HIP(call)                                                  \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return ibm::hip_fail(_e, #call);         \
    } while (0)

inline int grid_blocks(const Geo& g) {
    long long t = g.ntiles;
    return (int)(t < MAX_BLOCKS ? t : MAX_BLOCKS);
}

// ---------------------------------------------------------------- stencil view

// Device pointers of the velocity stencil (cut list and coefficients of eq. (q_axis)).
struct Sten {
    const uint8_t* mask;
    const uint32_t* cut_off;
    const double* a_ib;
    const double* a_c;
    const double* a_o;
    const int32_t* opp;
    const uint16_t* flags;
    int has_dead;
};

template <class T>
struct V3 {
    T* p[3];
};
template <class T>
struct C3 {
    const T* p[3];
};

inline Sten sten_of(const ibm_ctx* c) {
    return Sten{c->mask, c->cut_off, c->a_ib, c->a_c, c->a_o, c->cut_opp, c->flags, c->has_dead};
}

// index of the cut of cell c in direction d (bit d of msk set)
__device__ inline uint32_t cut_id(const Sten& st, long long c, uint8_t msk, int d) {
    return st.cut_off[c] + (uint32_t)__builtin_popcount((unsigned)msk & ((1u << d) - 1u));
}

// dead-end cell (closed in all six directions by the filter of eq. (deadend_filter))
__device__ inline bool dead_cell(const Sten& st, long long c, uint8_t msk) {
    return st.has_dead && __builtin_popcount((unsigned)msk) >= 5 && ((st.flags[c] >> 14) & 1);
}

// ---------------------------------------------------------------- device helpers

// Logical chunk of block b so that the blocks resident on one XCD (b % 8) walk one
// contiguous range of tiles: neighbouring planes stay in that XCD's L2.
__device__ inline int xcd_chunk(int b, int nb) {
    int per = nb / NXCD;
    int full = per * NXCD;
    if (b >= full) return b;
    return (b % NXCD) * per + b / NXCD;
}

// z-slabs of the marching sweeps (pressure passes, Crank-Nicolson passes): about 32
// planes per slab, a multiple of the XCD count
__host__ __device__ inline int slab_count(int nz) {
    int want = (nz + 31) / 32;
    want = ((want + 7) / 8) * 8;
    if (want > nz) want = nz;
    return want < 1 ? 1 : want;
}

// Tile range [t0, t1) of this block.
__device__ inline void tile_range(const Geo& g, long long& t0, long long& t1) {
    int nb = gridDim.x;
    int ch = xcd_chunk(blockIdx.x, nb);
    t0 = g.ntiles * ch / nb;
    t1 = g.ntiles * (ch + 1) / nb;
}

__device__ inline bool tile_cell(const Geo& g, long long t, int& i, int& j, int& k) {
    int tx = (int)(t % g.ntx);
    long long r = t / g.ntx;
    int ty = (int)(r % g.nty);
    k = (int)(r / g.nty);
    i = tx * TX + (threadIdx.x % TX);
    j = ty * TY + (threadIdx.x / TX);
    return i < g.nx && j < g.ny;
}

__device__ inline long long cidx(const Geo& g, int i, int j, int k) {
    return (long long)i + (long long)g.nx * ((long long)j + (long long)g.ny * k);
}

// Neighbour index across direction d (wrapping), and whether the face is a
// non-periodic domain face.
__device__ inline long long nb_index(const Geo& g, int i, int j, int k, int d, bool& boundary) {
    int ax = d >> 1;
    int s = (d & 1) ? 1 : -1;
    int n = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
    int co = ax == 0 ? i : (ax == 1 ? j : k);
    int cn = co + s;
    boundary = false;
    if (cn < 0 || cn >= n) {
        if (g.bc[d] != IBM_BC_PERIODIC) boundary = true;
        cn = (cn + n) % n;
    }
    int ii = i, jj = j, kk = k;
    if (ax == 0) ii = cn; else if (ax == 1) jj = cn; else kk = cn;
    return cidx(g, ii, jj, kk);
}

// Deterministic block reduction of NV doubles over NT threads: butterfly within each
// wavefront, then the wavefront totals in wavefront order; every thread gets the result.
template <int NV>
__device__ inline void block_reduce(double (&v)[NV], double* sh /* at least 4 * NV */) {
    constexpr int NW = NT / 64;
    const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        double x = v[a];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sh[a * NW + wid] = x;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += sh[a * NW + w];
        v[a] = t;
    }
    __syncthreads();
}

}  // namespace ibm

// Host-side launchers implemented in the .hip files.
namespace ibm {
// theta of the stencil build: a dense cells x 6 array, or the compact list of the
// context's tagging (2.0 where a direction is open)
struct ThetaSrc {
    const double* dense;
    const uint8_t* mask;
    const uint32_t* off;
    const double* list;
};
__device__ inline double theta_of(const ThetaSrc& t, long long c, int d) {
    if (t.dense) return t.dense[6 * c + d];
    const unsigned m = t.mask[c];
    if (!((m >> d) & 1u)) return 2.0;
    return t.list[t.off[c] + (uint32_t)__builtin_popcount(m & ((1u << d) - 1u))];
}

int tag_run(ibm_ctx* c, const double* tri, long long ntri, double bary_eps, hipStream_t s);
int tag_expand(ibm_ctx* c, double* theta, hipStream_t s);
int tag_matches(ibm_ctx* c, const uint8_t* blocked, bool* same, hipStream_t s);
void tag_release(ibm_ctx* c);
int stencil_run(ibm_ctx* c, const uint8_t* blocked, const ThetaSrc& theta, int deadend, hipStream_t s);
int cut_points_run(ibm_ctx* c, double* xyz, hipStream_t s);
int remove_means(ibm_ctx* c, double* a, hipStream_t s);
int laplacian_run(ibm_ctx* c, const double* x, double* y, hipStream_t s);
int march_blocks(const Geo& g);
int init_state_run(ibm_ctx* c, void** u, double** U, double* p, void** h, const double* u0,
                   const double* wall, hipStream_t s);
// initial guess of a step's solve: p <- 2 p - p_prev where that leaves the smaller
// residual of L x = b, and p_prev <- p (old)
int step_initial_guess(ibm_ctx* c, const double* b, double* p, double* p_prev, hipStream_t s);
int step_predict(ibm_ctx* c, void** u, double** U, void** h, const double* wall, const ibm_step_params* prm,
                 hipStream_t s);
int step_rhs(ibm_ctx* c, double** U, const double* wall, double dt, hipStream_t s);
int step_project(ibm_ctx* c, void** u, double** U, const double* p, double dt, hipStream_t s);
int divergence_norms(ibm_ctx* c, double** U, double* l2, double* linf, double* umax, hipStream_t s);
int poisson_run(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st,
                hipStream_t s);
int true_residual(ibm_ctx* c, const double* b, const double* x, double* rel, hipStream_t s);
int pcg64(ibm_ctx* c, const double* b, double* x, double tol, int max_iter, int check_every, int* iters,
          hipStream_t s);
int cnn_fcg_solve(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st, hipStream_t s);
// z = D^-1 r + s net([r/s, g]) inside a solve (cnn.hip), or with omega > 0 that map
// between two damped Jacobi steps; see cnn_precondition_solver there
int cnn_precondition_solver(void* net, ibm_ctx* c, const float* r, const float* rp, float* z, double* partials,
                            int nparts, int rr_slot, int zr_slot, int zrp_slot, int r1_slot, double omega, Solver* sv,
                            int it, int check, hipStream_t s);
// the smoothing passes of that two-level form (poisson.hip)
int smooth_pre(ibm_ctx* c, const float* r, float* r1, double omega, double* partials, int nparts, int r1_slot,
               int rr_slot, Solver* sv, int it, int check, hipStream_t s);
int smooth_post(ibm_ctx* c, const float* z2, const float* r, const float* rp, float* z, double omega,
                double* partials, int nparts, int zr_slot, int zrp_slot, const Solver* sv, int gate, hipStream_t s);
bool cnn_covers(const void* net, long long cells);
int cnn_prepare_geometry(void* net, ibm_ctx* c, hipStream_t s);
// timing helpers (poisson.hip)
// timed kernel slots: the two CG passes (or the preconditioner and the passes of the
// learned solve), the dominant convolution of the learned preconditioner, spare
// (other), the five BiCGStab passes of the Crank-Nicolson predictor, the momentum
// right-hand side / predictor kernel
enum { TK_SPMV = 0, TK_UPDATE = 1, TK_DIR = 2, TK_OTHER = 3, TK_CN_D = 4, TK_CN_AP = 5, TK_CN_S = 6, TK_CN_AS = 7,
       TK_CN_X = 8, TK_PREDICT = 9 };
// Launches kern<<<grid, NT, 0, s>>>(args...).  When timing slot k is on, the launch
// carries HIP's dispatch-level start/stop events (hipExtLaunchKernelGGL), so the time
// collected is the kernel's own, without the gaps between dispatches.
template <class F, class... Args>
inline void launch_timed(ibm_ctx* c, int k, F kern, int grid, hipStream_t s, Args... args) {
    if (c->timing_on && c->ev_used[k] < c->ev_cap) {
        const int e = c->ev_used[k]++;
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, s, c->ev[k][2 * e], c->ev[k][2 * e + 1], 0u, args...);
    } else {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, s, args...);
    }
}
void timing_begin(ibm_ctx* c, int k, hipStream_t s);
void timing_end(ibm_ctx* c, int k, hipStream_t s);
void timing_collect(ibm_ctx* c);
// Crank-Nicolson predictor (momentum.hip)
int cn_predict(ibm_ctx* c, void** u, double** U, const ibm_step_params* prm, int iters[3], hipStream_t s);
int cn_apply(ibm_ctx* c, const void* const* q, double* const* U, const void* nut, double nu, double dt,
             void* const* out, hipStream_t s);
int cn_solve(ibm_ctx* c, const void* const* b, void* const* x, double* const* U, const void* nut, double nu,
             double dt, double tol, int max_iter, int iters[3], hipStream_t s);
int cn_prepare(ibm_ctx* c);
void cn_release(ibm_ctx* c);
int shepard_run(ibm_ctx* c, const double* tri, long long ntri, const double* p, int filter, double* side,
                double* force, hipStream_t s);
void shepard_release(ibm_ctx* c);
// Every device and pinned-host allocation of the library goes through these (the
// count is reported by ibm_alloc_count, so a caller can check that a call allocated
// nothing).
void count_alloc();
template <class P>
inline hipError_t dev_malloc(P** p, size_t bytes) {
    const hipError_t e = hipMalloc((void**)p, bytes);
    if (e == hipSuccess) count_alloc();
    return e;
}
template <class P>
inline hipError_t dev_malloc_async(P** p, size_t bytes, hipStream_t s) {
    const hipError_t e = hipMallocAsync((void**)p, bytes, s);
    if (e == hipSuccess) count_alloc();
    return e;
}
template <class P>
inline hipError_t host_malloc(P** p, size_t bytes) {
    const hipError_t e = hipHostMalloc((void**)p, bytes, hipHostMallocDefault);
    if (e == hipSuccess) count_alloc();
    return e;
}

// Every C entry point is a function-try-block closed by IBM_CATCH_ALL, so no C++
// exception (a failed host allocation inside a container, ...) crosses the C ABI:
// std::bad_alloc becomes IBM_ERR_OOM, anything else IBM_ERR_ARG, with a message.
int abi_exception(bool oom, const char* what);
#define IBM_CATCH_ALL                                                                 \
    catch (const std::bad_alloc& e) { return ibm::abi_exception(true, e.what()); }     \
    catch (const std::exception& e) { return ibm::abi_exception(false, e.what()); }    \
    catch (...) { return ibm::abi_exception(false, "unknown exception"); }

int force_scratch_init(int device);
int forces_noalloc_run(ibm_ctx* c, void* const* u, const double* p, const void* nut, double nu,
                       const double* wall, double* out_dev, hipStream_t s);
int forces_run(ibm_ctx* c, void* const* u, const double* p, const void* nut, double nu, const double* wall,
               double* out, hipStream_t s);
}  // namespace ibm
