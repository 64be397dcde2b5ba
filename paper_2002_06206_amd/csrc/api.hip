// C ABI of the immersed-boundary step: argument checks, workspace ownership and
// launch sequencing.  All arithmetic of the step runs in the kernels of the other
// translation units; nothing here touches field data on the host.

#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "common.h"

namespace ibm {

static thread_local std::string g_err;
static std::atomic<long long> g_allocs{0};

void set_error(const std::string& msg) { g_err = msg; }

void count_alloc() { g_allocs.fetch_add(1, std::memory_order_relaxed); }

int abi_exception(bool oom, const char* what) {
    try {
        g_err = std::string(oom ? "host allocation failed: " : "internal error: ") + (what ? what : "");
    } catch (...) {
        g_err.clear();
    }
    return oom ? IBM_ERR_OOM : IBM_ERR_ARG;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? IBM_ERR_OOM : IBM_ERR_HIP;
}

int copy_cells(ibm_ctx* c, const void* src, void* dst, bool is_double, hipStream_t s);

}  // namespace ibm

using namespace ibm;

namespace {

int bad(const char* msg) {
    set_error(msg);
    return IBM_ERR_ARG;
}

template <class P>
int dalloc(P** p, size_t bytes) {
    hipError_t e = ibm::dev_malloc((void**)p, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        set_error(std::string("device allocation of ") + std::to_string(bytes) + " bytes failed");
        return IBM_ERR_OOM;
    }
    return IBM_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

int check_device(ibm_ctx* c) {
    int dev = -1;
    IBM_HIP(hipGetDevice(&dev));
    if (dev != c->device) return bad("context used on a different HIP device than the one it was created on");
    return IBM_OK;
}

int need_stencil(ibm_ctx* c) {
    if (!c) return bad("null context");
    if (!c->stencil_ready) return bad("ibm_build_stencils has not been called on this context");
    return check_device(c);
}

}  // namespace

extern "C" {

const char* ibm_last_error(void) { return g_err.c_str(); }

int ibm_alloc_count(int64_t* count_out) try {
    if (!count_out) return bad("ibm_alloc_count: null argument");
    *count_out = g_allocs.load(std::memory_order_relaxed);
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_create(const ibm_grid* grid, const ibm_bc* bc, int32_t precision, ibm_ctx** out) try {
    if (!grid || !bc || !out) return bad("ibm_create: null argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a)
        if (grid->n[a] < 3) return bad("ibm_create: every axis needs at least 3 cells");
    if (!(grid->dx > 0.0) || !std::isfinite(grid->dx)) return bad("ibm_create: dx must be positive and finite");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(grid->origin[a])) return bad("ibm_create: origin must be finite");
    long long N = (long long)grid->n[0] * grid->n[1] * grid->n[2];
    if (N >= (1ll << 31)) return bad("ibm_create: at most 2^31-1 cells");
    for (int d = 0; d < 6; ++d) {
        int k = bc->face[d];
        if (k < IBM_BC_PERIODIC || k > IBM_BC_SLIP) return bad("ibm_create: unknown boundary kind");
        if (k == IBM_BC_OUTFLOW && (d & 1) == 0) return bad("ibm_create: OUTFLOW is only supported on + faces");
    }
    for (int a = 0; a < 3; ++a)
        if ((bc->face[2 * a] == IBM_BC_PERIODIC) != (bc->face[2 * a + 1] == IBM_BC_PERIODIC))
            return bad("ibm_create: PERIODIC must be set on both faces of an axis");
    if (precision != IBM_FP64 && precision != IBM_MIXED) return bad("ibm_create: unknown precision");

    ibm_ctx* c = new (std::nothrow) ibm_ctx();
    if (!c) return bad("ibm_create: host allocation failed");
    std::memset((void*)c, 0, sizeof(*c));
    IBM_HIP(hipGetDevice(&c->device));
    c->precision = precision;
    c->N = N;
    Geo& g = c->geo;
    g.nx = grid->n[0];
    g.ny = grid->n[1];
    g.nz = grid->n[2];
    g.ntx = (g.nx + TX - 1) / TX;
    g.nty = (g.ny + TY - 1) / TY;
    g.ntiles = (long long)g.ntx * g.nty * g.nz;
    g.dx = grid->dx;
    g.ox = grid->origin[0];
    g.oy = grid->origin[1];
    g.oz = grid->origin[2];
    for (int d = 0; d < 6; ++d) g.bc[d] = bc->face[d];
    for (int a = 0; a < 3; ++a) g.uin[a] = bc->u_in[a];
    g.nblocks = grid_blocks(g);

    const size_t ts = precision == IBM_FP64 ? sizeof(double) : sizeof(float);
    const size_t padN = (size_t)((N + 3) / 4) * 4 + 64;
    int rc = IBM_OK;
    if (!rc) rc = dalloc(&c->mask, padN);
    if (!rc) rc = dalloc(&c->pcode, padN);
    if (!rc) rc = dalloc(&c->flags, sizeof(uint16_t) * N);
    if (!rc) rc = dalloc(&c->label, sizeof(int32_t) * N);
    if (!rc) rc = dalloc(&c->cut_off, sizeof(uint32_t) * N);
    for (int a = 0; a < 3 && !rc; ++a) rc = dalloc((char**)&c->ustar[a], ts * N);
    if (!rc) rc = dalloc((char**)&c->nut, ts * N);
    if (!rc) rc = dalloc(&c->b, sizeof(double) * N);
    if (!rc) rc = dalloc(&c->bwork, sizeof(double) * N);
    if (!rc) rc = dalloc(&c->r, sizeof(double) * N);
    if (!rc) rc = dalloc(&c->d, sizeof(double) * N);
    if (!rc) rc = dalloc(&c->q, sizeof(double) * N);
    if (!rc) rc = dalloc(&c->zbuf, sizeof(double) * N);
    // FP32 vectors of the mixed-precision correction solve
    if (!rc) rc = dalloc(&c->r32, sizeof(float) * N);
    if (!rc) rc = dalloc(&c->z32, sizeof(float) * N);
    if (!rc) rc = dalloc(&c->d32, sizeof(float) * N);
    if (!rc) rc = dalloc(&c->q32, sizeof(float) * N);
    if (!rc) rc = dalloc(&c->e32, sizeof(float) * N);
    if (!rc) rc = dalloc(&c->zprev32, sizeof(float) * N);   // FCG: previous residual
    if (!rc) rc = dalloc(&c->partials, sizeof(double) * 16 * MAX_BLOCKS);
    if (!rc) rc = dalloc(&c->counter, sizeof(unsigned int) * 16);
    if (!rc) rc = dalloc(&c->solver, sizeof(Solver));
    if (!rc) rc = dalloc(&c->red, sizeof(double) * 8);
    if (!rc) {
        hipError_t e1 = ibm::host_malloc(&c->h_solver, sizeof(Solver));
        hipError_t e2 = ibm::host_malloc(&c->h_red, sizeof(double) * 8);
        if (e1 != hipSuccess || e2 != hipSuccess) rc = hip_fail(e1 != hipSuccess ? e1 : e2, "hipHostMalloc");
    }
    if (!rc) rc = force_scratch_init(c->device);
    if (!rc) {
        hipError_t e = hipMemset(c->counter, 0, sizeof(unsigned int) * 16);
        if (e == hipSuccess) e = hipMemset(c->solver, 0, sizeof(Solver));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = hip_fail(e, "ibm_create initialisation");
    }
    if (rc) {
        ibm_destroy(c);
        return rc;
    }
    *out = c;
    return IBM_OK;
} IBM_CATCH_ALL

static void free_events(ibm_ctx* c) {
    for (int k = 0; k < TK_SLOTS_MAX; ++k) {
        if (!c->ev[k]) continue;
        for (int e = 0; e < 2 * c->ev_cap; ++e) (void)hipEventDestroy(c->ev[k][e]);
        delete[] c->ev[k];
        c->ev[k] = nullptr;
    }
    c->ev_cap = 0;
}

int ibm_destroy(ibm_ctx* c) try {
    if (!c) return IBM_OK;
    (void)hipDeviceSynchronize();
    free_events(c);
    cn_release(c);
    shepard_release(c);
    tag_release(c);
    void* ps[] = {c->mask, c->pcode, c->flags, c->label, c->cut_off, c->cut_cell, c->cut_dir,
                  c->cut_theta, c->a_ib, c->a_c, c->a_o, c->cut_opp, c->enc_cells, c->comp_start,
                  c->ustar[0], c->ustar[1], c->ustar[2], c->nut, c->b, c->bwork, c->r, c->d, c->q, c->zbuf, c->x64,
                  c->r32, c->z32, c->d32, c->q32, c->e32, c->zprev32, c->partials, c->counter, c->solver, c->red,
                  c->spec_cells};
    for (void* p : ps) dfree(p);
    if (c->h_solver) (void)hipHostFree(c->h_solver);
    if (c->h_red) (void)hipHostFree(c->h_red);
    delete c;
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_tag_geometry(ibm_ctx* c, const double* tri, int64_t ntri, double bary_eps, uint8_t* blocked, double* theta,
                     void* stream) try {
    if (!c) return bad("null context");
    if (int rc = check_device(c)) return rc;
    if (ntri < 0 || (ntri > 0 && !tri) || !blocked) return bad("ibm_tag_geometry: bad triangle or output pointer");
    if (ntri > (1ll << 40)) return bad("ibm_tag_geometry: too many triangles");
    if (!(bary_eps >= 0.0 && bary_eps <= 0.5)) return bad("ibm_tag_geometry: bary_eps must lie in [0, 0.5]");
    hipStream_t s = (hipStream_t)stream;
    const long long N = c->N;
    if (!c->tagmask) {
        if (int rc = dalloc(&c->tagmask, (size_t)((N + 3) / 4) * 4 + 64)) return rc;
    }
    if (!c->tag_off) {
        if (int rc = dalloc(&c->tag_off, sizeof(uint32_t) * N)) return rc;
    }
    int rc = tag_run(c, tri, ntri, bary_eps, s);
    if (rc < 0) return rc;
    IBM_HIP(hipMemcpyAsync(blocked, c->tagmask, N, hipMemcpyDeviceToDevice, s));
    if (theta) {
        if ((rc = tag_expand(c, theta, s))) return rc;
    }
    return rc;
} IBM_CATCH_ALL

int ibm_build_stencils(ibm_ctx* c, const uint8_t* blocked, const double* theta, int32_t deadend, uint16_t* flags,
                       int32_t* label, int64_t* n_cut_out, void* stream) try {
    if (!c) return bad("null context");
    if (int rc = check_device(c)) return rc;
    if (!blocked) return bad("ibm_build_stencils: null blocked");
    hipStream_t s = (hipStream_t)stream;
    ThetaSrc src{theta, nullptr, nullptr, nullptr};
    const bool own = theta == nullptr;
    if (own) {
        if (!c->tagged)
            return bad("ibm_build_stencils: theta is NULL and the context holds no tagging (none ran, or a "
                       "previous build consumed it)");
        bool same = false;
        if (int rc = tag_matches(c, blocked, &same, s)) return rc;
        if (!same) return bad("ibm_build_stencils: with theta NULL, blocked must be the context's tagging output");
        src = ThetaSrc{nullptr, reinterpret_cast<const uint8_t*>(c->tagmask), c->tag_off, c->tag_list};
    }
    c->stencil_ready = false;
    c->last_iters = 0;
    c->nut_valid = false;
    int rc = stencil_run(c, blocked, src, deadend ? 1 : 0, s);
    if (rc) return rc;
    if (flags) IBM_HIP(hipMemcpyAsync(flags, c->flags, sizeof(uint16_t) * c->N, hipMemcpyDeviceToDevice, s));
    if (label) IBM_HIP(hipMemcpyAsync(label, c->label, sizeof(int32_t) * c->N, hipMemcpyDeviceToDevice, s));
    if (n_cut_out) *n_cut_out = c->ncut;
    if (own) {
        // the cut list now holds what the step needs: release the tagging (the blocked
        // bits, 4 B of offsets per cell and the theta list)
        IBM_HIP(hipStreamSynchronize(s));
        tag_release(c);
    }
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cut_points(ibm_ctx* c, double* xyz, void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!xyz && c->ncut > 0) return bad("ibm_cut_points: null output");
    return cut_points_run(c, xyz, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_init_state(ibm_ctx* c, void* u[3], double* U[3], double* p, void* h[3], const double u0[3],
                   const double* wall, void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!u || !U || !p || !h || !u0) return bad("ibm_init_state: null argument");
    for (int a = 0; a < 3; ++a)
        if (!u[a] || !U[a] || !h[a]) return bad("ibm_init_state: null field pointer");
    return init_state_run(c, u, U, p, h, u0, wall, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_step(ibm_ctx* c, void* u[3], double* U[3], double* p, void* h[3], const double* wall,
             const ibm_step_params* prm, ibm_stats* st, void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!u || !U || !p || !h || !prm) return bad("ibm_step: null argument");
    for (int a = 0; a < 3; ++a)
        if (!u[a] || !U[a] || !h[a]) return bad("ibm_step: null field pointer");
    if (!(prm->dt > 0.0) || !(prm->nu >= 0.0) || prm->poisson.max_iter <= 0 || !(prm->poisson.tol > 0.0))
        return bad("ibm_step: need dt > 0, nu >= 0, tol > 0, max_iter > 0");
    if (prm->scheme != IBM_SCHEME_AB2 && prm->scheme != IBM_SCHEME_CN) return bad("ibm_step: unknown scheme");
    if (prm->p_prev == p) return bad("ibm_step: p_prev must be distinct from p");
    hipStream_t s = (hipStream_t)stream;
    const bool cn = prm->scheme == IBM_SCHEME_CN;
    if (cn && !c->cn_ws)
        return bad("ibm_step: the Crank-Nicolson scheme needs ibm_prepare_crank_nicolson first (it allocates the "
                   "solver workspace, so that ibm_step itself never allocates)");
    int rc = step_predict(c, u, U, h, wall, prm, s);
    if (rc) return rc;
    int mom_iters[3] = {0, 0, 0};
    if (cn) {
        rc = cn_predict(c, u, U, prm, mom_iters, s);
        if (rc) return rc;
    }
    rc = step_rhs(c, U, wall, prm->dt, s);
    if (rc) return rc;
    if (prm->p_prev) {
        rc = step_initial_guess(c, c->b, p, prm->p_prev, s);
        if (rc) return rc;
    }
    ibm_stats local;
    std::memset(&local, 0, sizeof(local));
    int prc = poisson_run(c, c->b, p, &prm->poisson, st ? &local : nullptr, s);
    if (prc < 0) return prc;
    rc = step_project(c, u, U, p, prm->dt, s);
    if (rc) return rc;
    if (st) {
        *st = local;
        for (int m = 0; m < 3; ++m) st->iters_momentum[m] = mom_iters[m];
        rc = divergence_norms(c, U, &st->div_l2, &st->div_linf, &st->umax, s);
        if (rc) return rc;
    }
    return prc;
} IBM_CATCH_ALL

int ibm_poisson_solve(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st,
                      void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!b || !x || !o) return bad("ibm_poisson_solve: null argument");
    if (o->max_iter <= 0 || !(o->tol > 0.0)) return bad("ibm_poisson_solve: need tol > 0 and max_iter > 0");
    hipStream_t s = (hipStream_t)stream;
    int rc = copy_cells(c, b, c->bwork, true, s);
    if (rc) return rc;
    rc = remove_means(c, c->bwork, s);
    if (rc) return rc;
    ibm_stats local;
    std::memset(&local, 0, sizeof(local));
    rc = poisson_run(c, c->bwork, x, o, &local, s);
    if (st && rc >= 0) *st = local;
    if (rc >= 0) IBM_HIP(hipStreamSynchronize(s));
    return rc;
} IBM_CATCH_ALL

int ibm_apply_laplacian(ibm_ctx* c, const double* x, double* y, void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!x || !y) return bad("ibm_apply_laplacian: null argument");
    return laplacian_run(c, x, y, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_prepare_crank_nicolson(ibm_ctx* c) try {
    if (!c) return bad("null context");
    if (int rc = check_device(c)) return rc;
    return cn_prepare(c);
} IBM_CATCH_ALL

int ibm_momentum_apply(ibm_ctx* c, const void* const q[3], double* const U[3], const void* nut, double nu,
                       double dt, void* const out[3], void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!q || !U || !out) return bad("ibm_momentum_apply: null argument");
    for (int a = 0; a < 3; ++a)
        if (!q[a] || !U[a] || !out[a]) return bad("ibm_momentum_apply: null field pointer");
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (out[a] == q[b]) return bad("ibm_momentum_apply: out must not alias q");
    if (!(dt >= 0.0) || !(nu >= 0.0)) return bad("ibm_momentum_apply: need dt >= 0 and nu >= 0");
    return cn_apply(c, q, U, nut, nu, dt, out, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_momentum_solve(ibm_ctx* c, const void* const b[3], void* const x[3], double* const U[3], const void* nut,
                       double nu, double dt, double tol, int32_t max_iter, int32_t iters_out[3], void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!b || !x || !U) return bad("ibm_momentum_solve: null argument");
    for (int a = 0; a < 3; ++a)
        if (!b[a] || !x[a] || !U[a]) return bad("ibm_momentum_solve: null field pointer");
    if (!(dt >= 0.0) || !(nu >= 0.0) || !(tol >= 0.0) || max_iter <= 0)
        return bad("ibm_momentum_solve: need dt >= 0, nu >= 0, tol >= 0, max_iter > 0");
    int it[3] = {0, 0, 0};
    const int rc = cn_solve(c, b, x, U, nut, nu, dt, tol, max_iter, it, (hipStream_t)stream);
    if (iters_out)
        for (int a = 0; a < 3; ++a) iters_out[a] = it[a];
    return rc;
} IBM_CATCH_ALL

int ibm_get_nut(ibm_ctx* c, void* out, void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!out) return bad("ibm_get_nut: null output");
    return copy_cells(c, c->nut, out, c->precision == IBM_FP64, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_get_rhs(ibm_ctx* c, double* out, void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!out) return bad("ibm_get_rhs: null output");
    return copy_cells(c, c->b, out, true, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_forces(ibm_ctx* c, void* const u[3], const double* p, const void* nut, double nu, const double* wall,
               double out[6], void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!u || !p || !out) return bad("ibm_forces: null argument");
    for (int a = 0; a < 3; ++a)
        if (!u[a]) return bad("ibm_forces: null velocity pointer");
    return forces_run(c, u, p, nut, nu, wall, out, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_forces_noalloc(ibm_ctx* c, void* const u[3], const double* p, const void* nut, double nu,
                       const double* wall, double* out_dev, void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (!u || !p || !out_dev) return bad("ibm_forces_noalloc: null argument");
    for (int a = 0; a < 3; ++a)
        if (!u[a]) return bad("ibm_forces_noalloc: null velocity pointer");
    return forces_noalloc_run(c, u, p, nut, nu, wall, out_dev, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_shepard_force(ibm_ctx* c, const double* tri, int64_t ntri, const double* p, int32_t thin_filter,
                      double* side, double force[3], void* stream) try {
    if (int rc = need_stencil(c)) return rc;
    if (ntri < 0 || (ntri > 0 && !tri) || !p || !force) return bad("ibm_shepard_force: bad arguments");
    return shepard_run(c, tri, ntri, p, thin_filter ? 1 : 0, side, force, (hipStream_t)stream);
} IBM_CATCH_ALL

int ibm_timing_enable(ibm_ctx* c, int32_t on) try {
    if (!c) return bad("null context");
    if (int rc = check_device(c)) return rc;
    if (on && c->ev_cap == 0) {
        const int cap = 8192;
        for (int k = 0; k < TK_SLOTS_MAX; ++k) {
            c->ev[k] = new (std::nothrow) hipEvent_t[2 * cap];
            if (!c->ev[k]) return bad("ibm_timing_enable: host allocation failed");
            for (int e = 0; e < 2 * cap; ++e) IBM_HIP(hipEventCreate(&c->ev[k][e]));
        }
        c->ev_cap = cap;
    }
    c->timing_on = on ? 1 : 0;
    for (int k = 0; k < TK_SLOTS_MAX; ++k) c->ev_used[k] = 0;
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_set_progress(ibm_ctx* c, ibm_progress_fn fn, void* user) try {
    if (!c) return bad("null context");
    c->progress = fn;
    c->progress_user = user;
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_timing_slot(ibm_ctx* c, int32_t slot, double out[2], int32_t reset) try {
    if (!c || !out) return bad("ibm_timing_slot: null argument");
    if (slot < 0 || slot >= TK_SLOTS_MAX) return bad("ibm_timing_slot: slot out of range");
    out[0] = c->t_ms[slot];
    out[1] = (double)c->t_launches[slot];
    if (reset) {
        c->t_ms[slot] = 0.0;
        c->t_launches[slot] = 0;
    }
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_timing_read(ibm_ctx* c, double out[10], int32_t reset) try {
    if (!c || !out) return bad("ibm_timing_read: null argument");
    for (int k = 0; k < 3; ++k) {
        out[k] = c->t_ms[k];
        out[3 + k] = (double)c->t_launches[k];
    }
    out[6] = (double)c->t_real_iters;
    out[7] = (double)c->N;
    out[8] = (double)c->ncut;
    out[9] = (double)c->precision;
    if (reset) {
        for (int k = 0; k < TK_SLOTS_MAX; ++k) {
            c->t_ms[k] = 0.0;
            c->t_launches[k] = 0;
        }
        c->t_real_iters = 0;
    }
    return IBM_OK;
} IBM_CATCH_ALL

}  // extern "C"
