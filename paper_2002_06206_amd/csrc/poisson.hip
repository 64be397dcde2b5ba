// Pressure Poisson solve (eq. poisson) on the immersed-boundary stencil.
//
// A = -L, L p = (1/dx^2)[sum over open faces (p_nb - p_c) - 2 p_c per outlet face],
// is symmetric positive semi-definite (the face blocking is symmetric), so the plain
// solver is Jacobi-preconditioned conjugate gradients in FP64, warm started.
// Each iteration is three fused sweeps (SpMV + <d,q>; x/r update + <r,r> + <r,z>;
// direction update); the scalars alpha and beta are formed on the device by the last
// block of each reduction, so the host only enqueues work.  Convergence is decided
// on the device after every update and turns the remaining enqueued sweeps into
// no-ops; the host polls between batches of iterations.

#include "common.h"

namespace ibm {
namespace {

// diagonal of A times dx^2: open faces + 2 per outlet face
__device__ inline double diag_count(const Geo& g, int i, int j, int k, uint8_t msk) {
    int cnt = 0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        int ax = d >> 1;
        int n = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
        int co = ax == 0 ? i : (ax == 1 ? j : k);
        bool bnd = (d & 1) ? (co == n - 1) : (co == 0);
        if (bnd && g.bc[d] != IBM_BC_PERIODIC) {
            if (g.bc[d] == IBM_BC_OUTFLOW) cnt += 2;
        } else if (!((msk >> d) & 1)) {
            cnt += 1;
        }
    }
    return (double)cnt;
}

// (L x)_c
__device__ inline double lap_at(const Geo& g, const uint8_t msk, const double* x, int i, int j, int k, long long c) {
    double xc = x[c];
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        bool bnd;
        long long n = nb_index(g, i, j, k, d, bnd);
        if (bnd) {
            if (g.bc[d] == IBM_BC_OUTFLOW) acc += -2.0 * xc;
        } else if (!((msk >> d) & 1)) {
            acc += x[n] - xc;
        }
    }
    return acc / (g.dx * g.dx);
}

__global__ void __launch_bounds__(NT) k_pcg_init(Geo g, const uint8_t* mask, const double* b, const double* x,
                                                 double* r, double* d, double* partials, unsigned int* counter,
                                                 Solver* sv, double tol) {
    __shared__ double sh[3 * NT];
    long long t0, t1;
    tile_range(g, t0, t1);
    double v[3] = {0.0, 0.0, 0.0};
    const double dx2 = g.dx * g.dx;
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        uint8_t msk = mask[c];
        double rc = -b[c] + lap_at(g, msk, x, i, j, k, c);
        double cnt = diag_count(g, i, j, k, msk);
        double z = cnt > 0.0 ? rc * dx2 / cnt : 0.0;
        r[c] = rc;
        d[c] = z;
        v[0] += b[c] * b[c];
        v[1] += rc * rc;
        v[2] += rc * z;
    }
    double tot[3];
    if (grid_reduce<3>(v, partials, counter, sh, tot) && threadIdx.x == 0) {
        sv->fnorm2 = tot[0];
        sv->tol2 = tol * tol * tot[0];
        sv->rr = tot[1];
        sv->rz = tot[2];
        sv->iters = 0;
        sv->nan_seen = 0;
        if (!(tot[1] == tot[1]) || !(tot[0] == tot[0])) {
            sv->nan_seen = 1;
            sv->converged = 3;
        } else if (tot[0] == 0.0) {
            sv->converged = 2;
        } else {
            sv->converged = tot[1] <= sv->tol2 ? 1 : 0;
        }
    }
}

__global__ void k_zero_if_trivial(Geo g, double* x, const Solver* sv) {
    if (sv->converged != 2) return;
    long long n = (long long)g.nx * g.ny * g.nz;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

__global__ void __launch_bounds__(NT) k_pcg_spmv(Geo g, const uint8_t* mask, const double* d, double* q,
                                                 double* partials, unsigned int* counter, Solver* sv) {
    if (sv->converged) return;
    __shared__ double sh[NT];
    long long t0, t1;
    tile_range(g, t0, t1);
    double v[1] = {0.0};
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        double qc = -lap_at(g, mask[c], d, i, j, k, c);
        q[c] = qc;
        v[0] += d[c] * qc;
    }
    double tot[1];
    if (grid_reduce<1>(v, partials, counter, sh, tot) && threadIdx.x == 0) {
        sv->dq = tot[0];
        sv->alpha = sv->rz / tot[0];
    }
}

__global__ void __launch_bounds__(NT) k_pcg_update(Geo g, const uint8_t* mask, double* x, const double* d,
                                                   const double* q, double* r, double* partials,
                                                   unsigned int* counter, Solver* sv) {
    if (sv->converged) return;
    __shared__ double sh[2 * NT];
    const double alpha = sv->alpha;
    long long t0, t1;
    tile_range(g, t0, t1);
    double v[2] = {0.0, 0.0};
    const double dx2 = g.dx * g.dx;
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        x[c] = x[c] + alpha * d[c];
        double rc = r[c] - alpha * q[c];
        r[c] = rc;
        double cnt = diag_count(g, i, j, k, mask[c]);
        double z = cnt > 0.0 ? rc * dx2 / cnt : 0.0;
        v[0] += rc * rc;
        v[1] += rc * z;
    }
    double tot[2];
    if (grid_reduce<2>(v, partials, counter, sh, tot) && threadIdx.x == 0) {
        sv->iters += 1;
        sv->rr = tot[0];
        if (!(tot[0] == tot[0])) {
            sv->nan_seen = 1;
            sv->converged = 3;
        } else if (tot[0] <= sv->tol2) {
            sv->converged = 1;
        } else {
            sv->beta = tot[1] / sv->rz;
            sv->rz = tot[1];
        }
    }
}

__global__ void __launch_bounds__(NT) k_pcg_dir(Geo g, const uint8_t* mask, const double* r, double* d,
                                                const Solver* sv) {
    if (sv->converged) return;
    const double beta = sv->beta;
    long long t0, t1;
    tile_range(g, t0, t1);
    const double dx2 = g.dx * g.dx;
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        double cnt = diag_count(g, i, j, k, mask[c]);
        double z = cnt > 0.0 ? r[c] * dx2 / cnt : 0.0;
        d[c] = z + beta * d[c];
    }
}

// ||b - L x||^2 and ||b||^2
__global__ void __launch_bounds__(NT) k_resid(Geo g, const uint8_t* mask, const double* b, const double* x,
                                              double* partials, unsigned int* counter, double* out) {
    __shared__ double sh[2 * NT];
    long long t0, t1;
    tile_range(g, t0, t1);
    double v[2] = {0.0, 0.0};
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        double res = b[c] - lap_at(g, mask[c], x, i, j, k, c);
        v[0] += res * res;
        v[1] += b[c] * b[c];
    }
    double tot[2];
    if (grid_reduce<2>(v, partials, counter, sh, tot) && threadIdx.x == 0) {
        out[0] = tot[0];
        out[1] = tot[1];
    }
}

}  // namespace

int true_residual(ibm_ctx* c, const double* b, const double* x, double* rel, hipStream_t s) {
    k_resid<<<grid_blocks(c->geo), NT, 0, s>>>(c->geo, c->mask, b, x, c->partials, c->counter, c->red);
    IBM_HIP(hipGetLastError());
    IBM_HIP(hipMemcpyAsync(c->h_red, c->red, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    *rel = c->h_red[1] > 0.0 ? sqrt(c->h_red[0] / c->h_red[1]) : 0.0;
    return IBM_OK;
}

// FP64 Jacobi PCG on L x = b (b already compatible); x in/out.  Sets *iters.
int pcg64(ibm_ctx* c, const double* b, double* x, double tol, int max_iter, int check_every, int* iters,
          hipStream_t s) {
    const Geo& g = c->geo;
    const int nb = grid_blocks(g);
    k_pcg_init<<<nb, NT, 0, s>>>(g, c->mask, b, x, c->r, c->d, c->partials, c->counter, c->solver, tol);
    k_zero_if_trivial<<<1024, 256, 0, s>>>(g, x, c->solver);
    IBM_HIP(hipGetLastError());
    if (check_every <= 0) check_every = 16;
    int batch = c->last_iters > 0 ? c->last_iters + 2 : check_every;
    int total = 0;
    while (true) {
        int n = batch;
        if (n > max_iter - total) n = max_iter - total;
        for (int it = 0; it < n; ++it) {
            k_pcg_spmv<<<nb, NT, 0, s>>>(g, c->mask, c->d, c->q, c->partials, c->counter, c->solver);
            k_pcg_update<<<nb, NT, 0, s>>>(g, c->mask, x, c->d, c->q, c->r, c->partials, c->counter, c->solver);
            k_pcg_dir<<<nb, NT, 0, s>>>(g, c->mask, c->r, c->d, c->solver);
        }
        IBM_HIP(hipGetLastError());
        total += n;
        IBM_HIP(hipMemcpyAsync(c->h_solver, c->solver, sizeof(Solver), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (c->h_solver->converged || total >= max_iter) break;
        batch = check_every;
    }
    *iters = c->h_solver->iters;
    c->last_iters = c->h_solver->iters;
    if (c->h_solver->converged == 3) {
        set_error("pressure solve: non-finite residual");
        return IBM_ERR_NAN;
    }
    return c->h_solver->converged ? IBM_OK : IBM_NOT_CONVERGED;
}

int poisson_run(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st, hipStream_t s) {
    int iters = 0;
    int rc = pcg64(c, b, x, o->tol, o->max_iter, o->check_every, &iters, s);
    if (rc < 0) return rc;
    int rc2 = remove_means(c, x, s);
    if (rc2) return rc2;
    if (st) {
        st->iters_inner = iters;
        st->iters_outer = 0;
        st->fallback_used = 0;
        st->status = rc;
        int rc3 = true_residual(c, b, x, &st->rel_residual, s);
        if (rc3) return rc3;
    }
    return rc;
}

}  // namespace ibm
