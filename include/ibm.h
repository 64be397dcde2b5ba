/*
 * ibm.h - C ABI of the MI355X (gfx950) topology-free immersed boundary time step.
 *
 * The method (Onishi & Tsubokura, arXiv:2002.06206): an incompressible LES step on
 * a uniform Cartesian grid, fractional step with a pressure Poisson solve
 * (Sec. 2.1, eqs. (crank-nicolson), (correction), (poisson)), driven directly by
 * an arbitrary, possibly non-watertight ("dirty") triangle soup (Sec. 2.3).  No
 * inside/outside decision is ever made: every grid-line segment between two cell
 * centres that meets a triangle makes the neighbour behind the crossing a ghost
 * cell for that cell only (Sec. 2.3.1), and the ghost value comes from the
 * axis-projected formula eq. (q_axis) (Sec. 2.3.2).
 *
 * Conventions shared by every entry point
 *  - Cells: c = i + nx*(j + ny*k), x fastest.  Cell centre = origin + (i + 0.5)*dx.
 *  - Directions: 0..5 = -x,+x,-y,+y,-z,+z; blocked masks use bit d for direction d.
 *  - Face velocities U[k] (k = x,y,z) hold the normal velocity on the +k face of
 *    every cell; the -k face of the first layer comes from the boundary kind.
 *  - All field pointers are caller-owned, contiguous DEVICE memory on the current
 *    HIP device.  Cell fields (u, H, nu_t) are double under IBM_FP64 and float
 *    under IBM_MIXED; U, p, b and wall velocities are always double.
 *  - `stream` is a hipStream_t (NULL = default stream).  Every call is enqueued on
 *    it and returns without waiting, except where a host output is requested
 *    (n_cut_out, stats, forces), which synchronises that stream.
 *  - Return codes: IBM_OK (0); IBM_NOT_CONVERGED (+1, tolerance not met within
 *    max_iter, results still written); negative codes are errors and leave the
 *    outputs unspecified: IBM_ERR_ARG (bad argument / shape / state),
 *    IBM_ERR_HIP (HIP runtime error), IBM_ERR_OOM (device allocation failed),
 *    IBM_ERR_NAN (non-finite residual).  ibm_last_error() gives a message
 *    (thread-local).  No C++ exception crosses this boundary.
 *  - Determinism: identical inputs on the same GPU give bit-identical outputs
 *    (all reductions use a fixed order; tagging uses order-independent atomics).
 *  - Calls on one context must not overlap (one stream at a time per context).
 */
#ifndef IBM_H
#define IBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { IBM_BC_PERIODIC = 0, IBM_BC_INFLOW = 1, IBM_BC_OUTFLOW = 2, IBM_BC_SLIP = 3 };
enum { IBM_FP64 = 0, IBM_MIXED = 1 };
enum {
    IBM_SOLVER_PCG_JACOBI = 0, /* FP64 Jacobi-preconditioned CG                          */
    IBM_SOLVER_FCG_CNN = 1,    /* FP64 refinement around FP32 flexible CG, CNN precond.   */
    IBM_SOLVER_FCG_JACOBI = 2, /* FP64 refinement around FP32 flexible CG, Jacobi precond.*/
    IBM_SOLVER_RBSOR = 3       /* FP64 red-black SOR (Sec. 2.1)                          */
};
/* momentum predictor of ibm_step: explicit Adams-Bashforth, or Crank-Nicolson with
 * BiCGStab (eq. (crank-nicolson), Sec. 2.1) */
enum { IBM_SCHEME_AB2 = 0, IBM_SCHEME_CN = 1 };
enum { IBM_OK = 0, IBM_NOT_CONVERGED = 1, IBM_ERR_ARG = -1, IBM_ERR_HIP = -2, IBM_ERR_OOM = -3,
       IBM_ERR_NAN = -4 };

/* Uniform Cartesian grid (the one-level case of the paper's cube grid, Sec. 2.2). */
typedef struct {
    int32_t n[3];      /* cells per axis, each >= 3                              */
    double dx;         /* cell size (> 0)                                         */
    double origin[3];  /* low corner of the domain                                */
} ibm_grid;

/* Outer boundary kinds, order -x,+x,-y,+y,-z,+z (the paper omits them, Sec. 2.1):
 * PERIODIC must be set on both faces of an axis; INFLOW = Dirichlet u_in with
 * zero-gradient pressure; OUTFLOW (only on a + face) = zero-gradient velocity with
 * p = 0 on the face; SLIP = zero normal velocity, zero-gradient tangential velocity
 * and pressure. */
typedef struct {
    int32_t face[6];
    double u_in[3];
} ibm_bc;

/* Pressure solver options.  tol is the relative residual ||b - L p||_2 / ||b||_2
 * (equivalently ||div U^{n+1}||_2 / (dt ||b||_2)). */
typedef struct {
    double tol;
    int32_t max_iter;        /* cap on (inner) iterations per solve                */
    int32_t kind;            /* IBM_SOLVER_*                                        */
    double inner_tol;        /* mixed kinds: reduction of the FP32 recursive        */
                             /* residual per segment before the FP64 residual      */
                             /* replaces it (default 0.1)                           */
    int32_t inner_max_iter;  /* mixed kinds: iteration cap per segment              */
    double stall_factor;     /* mixed kinds: fall back to FP64 PCG when a segment   */
                             /* reduces the FP64 residual by less than this factor  */
    int32_t check_every;     /* iterations enqueued between host convergence polls  */
    int32_t force_stall;     /* test hook: treat the first sweep as stalled; 1 = fall */
                             /* back to FP64 PCG, 2 = the retry of inner_restart 0   */
    double omega;            /* IBM_SOLVER_RBSOR: relaxation factor in (0, 2); <= 0: */
                             /* 2 / (1 + sin(pi / n_max)).  Cells are coloured by the */
                             /* parity of i + j + k; a sweep updates colour 0, then 1, */
                             /* x_c += omega (b_c - (L x)_c) / L_cc; the true residual */
                             /* is tested every check_every sweeps; max_iter counts  */
                             /* sweeps.  Periodic axes need an even cell count       */
                             /* (IBM_ERR_ARG otherwise).                              */
                             /* IBM_SOLVER_FCG_CNN: in (0, 1], the weight of the two  */
                             /* damped Jacobi steps around the network (the smoothed  */
                             /* form of ibm_cnn_precondition; needs nx % 4 == 0);    */
                             /* <= 0: the network's map alone.                        */
    int32_t inner_restart;   /* IBM_SOLVER_FCG_JACOBI: 0 = keep the search direction */
                             /* across residual replacements, and retry a stalled    */
                             /* segment from a fresh direction (up to 3 times per    */
                             /* solve) before the FP64 fallback; 1 = start every     */
                             /* segment from a fresh direction                       */
    int32_t pad;
} ibm_solver_opts;

/* One time step: momentum predictor, coherent structure model (Sec. 2.3) when csm_on,
 * body force, Poisson, projection.
 * scheme IBM_SCHEME_AB2: variable-step Adams-Bashforth,
 *   u* = u + dt [(1 + r/2) H^n - (r/2) H^{n-1}], r = dt/dt_prev (dt_prev <= 0 means
 *   dt_prev = dt, the constant-step 3/2, -1/2 weights); forward Euler when step == 0.
 * Advective face value: central, or with quick > 0 the hybrid of Sec. 3 blending the
 * QUICK value (Leonard 1979: (6 q_up + 3 q_down - q_farup)/8, upstream by the outward
 * face velocity); the far cell across a blocked or domain face is the first ghost's
 * line continued one cell (2 q_GC - q_c), elsewhere the neighbour's own neighbour.
 * scheme IBM_SCHEME_CN: Crank-Nicolson for advection (by the frozen face velocity U^n)
 *   and diffusion (nu + the eddy viscosity of u^n) together, eq. (crank-nicolson):
 *   with H the explicit right-hand side and L its part linear in u,
 *   (I - dt/2 L) (u* - u^n) = dt H^n for each component, solved by unpreconditioned
 *   BiCGStab from the explicit Euler increment until ||r|| <= mom_tol ||dt H^n||
 *   (on IBM_MIXED contexts, where the vectors are FP32, mom_tol is raised to at least
 *   1e-6).  Dead-end cells keep their mean wall velocity.  h_dev receives H^n.  Needs
 *   ibm_prepare_crank_nicolson on the context first (IBM_ERR_ARG otherwise). */
typedef struct {
    double dt;
    double dt_prev;         /* previous step's dt (<= 0: same as dt)                 */
    double nu;              /* molecular kinematic viscosity (1/Re in flow units)   */
    double c1;              /* CSM constant C1, 1/20 in the paper                   */
    int32_t csm_on;
    int32_t step;           /* 0 = first step (forward Euler), else AB2              */
    double body_force[3];
    ibm_solver_opts poisson;
    int32_t scheme;         /* IBM_SCHEME_AB2 or IBM_SCHEME_CN                       */
    int32_t mom_max_iter;   /* CN: BiCGStab iteration cap (<= 0: 200)                */
    double mom_tol;         /* CN: relative residual per component (<= 0: 1e-10)     */
    double quick;           /* weight w of the QUICK face value in the advective     */
                            /* flux, q_f = (1 - w) q_central + w q_QUICK (Sec. 3:    */
                            /* 0.1 in the paper's runs; 0 = central); explicit in    */
                            /* both schemes (the CN operator keeps central)          */
    double* p_prev;         /* NULL, or a device array of N doubles holding p^{n-1}: */
                            /* the pressure solve then starts from 2 p^n - p^{n-1}   */
                            /* when that leaves a smaller residual ||b - L x|| than  */
                            /* p^n (else from p^n), and p_prev receives p^n (set it  */
                            /* to p before the first step); distinct from p_dev      */
} ibm_step_params;

typedef struct {
    int32_t iters_inner;     /* CG / FCG iterations, FP64 fallback iterations included */
    int32_t iters_outer;     /* FP32 segments between FP64 residual replacements     */
                             /* (0 for plain PCG)                                    */
    int32_t fallback_used;   /* 1 when the FP64 PCG fallback ran                     */
    int32_t status;          /* return code of the solve                             */
    double rel_residual;     /* FP64 ||b - L p|| / ||b|| after the solve             */
    double div_l2;           /* ||div U^{n+1}||_2 over all cells (ibm_step only)     */
    double div_linf;         /* max |div U^{n+1}|                                    */
    double umax;             /* max |U| over all faces after the step (CFL control)  */
    int32_t iters_momentum[3]; /* CN: BiCGStab iterations per component (else 0)     */
    int32_t iters_fallback;  /* of iters_inner, the FP64 PCG fallback's iterations    */
} ibm_stats;

typedef struct ibm_ctx ibm_ctx;

/* Creates a context on the current HIP device and allocates the per-step
 * workspace once (no allocation happens later inside ibm_step or
 * ibm_poisson_solve).  precision = IBM_FP64 or IBM_MIXED. */
int ibm_create(const ibm_grid* grid, const ibm_bc* bc, int32_t precision, ibm_ctx** out);
int ibm_destroy(ibm_ctx* ctx);
const char* ibm_last_error(void);

/* Diagnostic: number of device and pinned-host allocations the library has made in this
 * process (every context, network and grid); *count_out receives it.  Comparing two
 * readings shows whether the calls between them allocated anything. */
int ibm_alloc_count(int64_t* count_out);

/* Tagging (Sec. 2.3.1): tri_dev = ntri x 3 vertices x xyz doubles (device).  For every
 * segment between face-adjacent cell centres inside the domain, decides exactly
 * whether the closed segment meets a closed triangle (edges and vertices inclusive;
 * triangles parallel to the segment never block), sets bit d of blocked_dev[c]
 * and bit d^1 of the neighbour, and stores theta = distance from the cell centre to
 * its nearest crossing / dx in [0,1] (2.0 where open).
 * theta uses one fixed double formula: the crossing coordinate is the barycentric
 * combination of the vertex coordinates weighted by the double 2-D sub-areas.
 * bary_eps (in [0, 0.5]; 0 = exact) is the tolerance of the paper's ray / triangle test
 * (Sec. 2.3.1: adjusting it keeps rays from slipping through gaps between triangles):
 * a grid line that misses a triangle exactly still meets it when each of the three
 * double sub-areas, signed by the exact orientation of the projected triangle, is at
 * least -bary_eps |sum of the sub-areas| (barycentric coordinates >= -bary_eps); the
 * crossed segment is still decided exactly.  The blocked set grows with bary_eps.
 * Domain and periodic-wrap faces are never tagged.  Coordinates must be finite
 * with magnitude 0 or within [2^-200, 2^200] (IBM_ERR_ARG otherwise).
 * blocked_dev: N bytes.  theta_dev: N*6 doubles (theta_dev[6*c + d]) for callers that
 * want the dense array, or NULL.  The context always keeps the tagging in compact form
 * for ibm_build_stencils: the blocked bits, a 32-bit offset per cell and one double per
 * blocked (cell, dir), about 5 B per cell plus 8 B per cut instead of the 48 B per
 * cell of a dense theta (which at 1024^3 would be 48 GiB).  Tagging runs the line
 * tests twice (bits, then the compact list); it allocates on the first call and when
 * the list outgrows its capacity. */
int ibm_tag_geometry(ibm_ctx* ctx, const double* tri_dev, int64_t ntri, double bary_eps, uint8_t* blocked_dev,
                     double* theta_dev, void* stream);

/* Stencil build (Sec. 2.3.1-2.3.2): from blocked bits and theta (theta_dev NULL = the
 * context's compact tagging from the last ibm_tag_geometry, whose blocked bits
 * blocked_dev must equal (IBM_ERR_ARG otherwise); the build then releases it, and
 * building again from it needs a new ibm_tag_geometry), applies the dead-end filter of
 * eq. (deadend_filter) when deadend != 0 (a cell closed in >= 5 directions is closed
 * in all six and frozen at the wall velocity; its open neighbours see a wall at its
 * centre, theta = 1), builds the cut list (one entry per blocked (cell, dir),
 * ordered by cell then dir) with the coefficients of eq. (q_axis), the classes of
 * eq. (dummy_cell_region), and the connected components of the pressure problem.
 * flags_dev (N uint16, or NULL): bits 0-5 effective blocked bits, bits 6-7 class
 * (0 fluid, 1 wall-including, 2 wall-adjacent), bits 8-13 theta < 0.5 per blocked
 * dir, bit 14 dead end, bit 15 enclosed (component without an outlet face).
 * label_dev (N int32, or NULL): smallest cell index of the cell's component over
 * open faces.  n_cut_out (host, or NULL): number of cuts. */
int ibm_build_stencils(ibm_ctx* ctx, const uint8_t* blocked_dev, const double* theta_dev,
                       int32_t deadend, uint16_t* flags_dev, int32_t* label_dev,
                       int64_t* n_cut_out, void* stream);

/* Crossing point X of every cut (n_cut x 3 doubles, device): the cell centre moved
 * by theta*dx along the cut direction.  Callers evaluate wall velocities u_IB(X). */
int ibm_cut_points(ibm_ctx* ctx, double* xyz_dev, void* stream);

/* Initial state: u = u0 in every cell, U = u0 on open and periodic faces, the mean
 * wall normal velocity of the two cuts on blocked faces, boundary values on domain
 * faces; p = 0; h = 0.  wall_dev: n_cut x 3 doubles or NULL (stationary walls). */
int ibm_init_state(ibm_ctx* ctx, void* u_dev[3], double* U_dev[3], double* p_dev, void* h_dev[3],
                   const double u0[3], const double* wall_dev, void* stream);

/* One fractional step (Sec. 2.1): coherent-structure eddy viscosity (Sec. 2.3), AB2
 * predictor in flux form with the axis-projected ghost values of eq. (q_axis)
 * across blocked faces, face velocity U* (Rhie-Chow style compact face velocity),
 * b = div U* / dt made compatible on enclosed components, pressure solve warm
 * started from p (or, with prm->p_prev, from the linear extrapolation 2 p - p_prev of
 * the two previous pressures when its residual is the smaller), projection of U and u,
 * FP64 divergence check.
 * u_dev, h_dev: in u^n, H^{n-1}; out u^{n+1}, H^n.  U_dev: in U^n, out U^{n+1}.
 * p_dev: in guess, out p^{n+1} (zero mean on enclosed components).
 * wall_dev: n_cut x 3 wall velocities u_IB at the crossing points, or NULL.
 * stats (host, or NULL): filled and the stream synchronised when non-NULL. */
int ibm_step(ibm_ctx* ctx, void* u_dev[3], double* U_dev[3], double* p_dev, void* h_dev[3],
             const double* wall_dev, const ibm_step_params* prm, ibm_stats* stats, void* stream);

/* Pressure Poisson solve (eq. (poisson)) on the context's stencil: L x = b where
 * L p = (1/dx^2)[sum over open faces (p_nb - p_c) - 2 p_c per outlet face];
 * blocked, inflow and slip faces are Neumann (ghost p = p_c, eq. (Mittal) with
 * zeta = 1, eta = 0).  b is made compatible (mean removed) on enclosed components
 * in a private copy; x (in: guess, out: solution) gets zero mean there.
 * Always synchronises the stream (the solver polls convergence). */
int ibm_poisson_solve(ibm_ctx* ctx, const double* b_dev, double* x_dev, const ibm_solver_opts* opts,
                      ibm_stats* stats, void* stream);

/* y = L x (the operator above), for tests. */
int ibm_apply_laplacian(ibm_ctx* ctx, const double* x_dev, double* y_dev, void* stream);

/* Allocates the Crank-Nicolson solver workspace of a context once (6 vectors of 3 cell
 * fields of the context's cell type, partial sums, a device state and its pinned host
 * mirror; freed by ibm_destroy), so that ibm_step and ibm_momentum_solve never allocate.
 * Idempotent.  IBM_ERR_OOM when any part cannot be allocated; nothing is then kept, so
 * the context stays without a workspace. */
int ibm_prepare_crank_nicolson(ibm_ctx* ctx);

/* Crank-Nicolson momentum operator (eq. (crank-nicolson)) for tests and callers with
 * their own time loop: out = (I - dt/2 L) q for the three components, L the part of the
 * momentum right-hand side linear in the velocity: flux-form central advection by the
 * face velocities U_dev (as ibm_step's U) and diffusion with nu + the face eddy
 * viscosity (mean of the two cells on open faces, the cell's own on closed ones);
 * ghosts behind blocked faces a_c q_c + a_o q_o (eq. (q_axis) with a zero wall
 * velocity), behind inflow faces and for the normal component at slip faces -q_c,
 * otherwise q_c.  Dead-end rows are the identity.  q_dev, out_dev: 3 cell fields of the
 * context's cell type (double for IBM_FP64, float for IBM_MIXED), out distinct from q;
 * nut_dev: a cell field of that type, or NULL for zero eddy viscosity. */
int ibm_momentum_apply(ibm_ctx* ctx, const void* const q_dev[3], double* const U_dev[3], const void* nut_dev,
                       double nu, double dt, void* const out_dev[3], void* stream);

/* Solves (I - dt/2 L) x = b (the operator of ibm_momentum_apply) for the three
 * components by unpreconditioned BiCGStab (Sec. 2.1): x_dev holds the initial guess on
 * entry and the solution on return; b_dev may equal x_dev.  Each component stops when
 * ||b - A x|| <= tol ||b|| at the start of an iteration or halfway through one; a zero b
 * gives x = 0.  iters_out (host, or NULL): iterations per component.  Needs
 * ibm_prepare_crank_nicolson first.  Returns
 * IBM_NOT_CONVERGED at max_iter or on a breakdown (rho = 0, <r0, v> = 0, omega = 0),
 * IBM_ERR_NAN on a non-finite residual.  Synchronises the stream. */
int ibm_momentum_solve(ibm_ctx* ctx, const void* const b_dev[3], void* const x_dev[3], double* const U_dev[3],
                       const void* nut_dev, double nu, double dt, double tol, int32_t max_iter,
                       int32_t iters_out[3], void* stream);

/* Copies of quantities from the last ibm_step: eddy viscosity (cell type) and the
 * compatible Poisson right-hand side b (double). */
int ibm_get_nut(ibm_ctx* ctx, void* out_dev, void* stream);
int ibm_get_rhs(ibm_ctx* ctx, double* out_dev, void* stream);

/* Force on the immersed surface as the momentum flux through every blocked face
 * (cut-face form of the near-field force): for each cut of cell c with direction
 * s*e_k, F_p += dx^2 s p_c e_k and F_v -= dx^2 (nu + nu_t,c)(q_GC - q_c)/dx, with
 * q_GC the eq. (q_axis) ghost of each velocity component.  nut_dev NULL = the
 * context's eddy viscosity from the last step (zero before any step).
 * out_host[6] = F_p xyz, F_v xyz.  Synchronises the stream.  Drag coefficients
 * follow eqs. (cd_sphere) / (cd_flat_plate) on the caller's side. */
int ibm_forces(ibm_ctx* ctx, void* const u_dev[3], const double* p_dev, const void* nut_dev, double nu,
               const double* wall_dev, double out_host[6], void* stream);

/* For callers that cannot allocate device memory or wait on the host (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the forces of
 * ibm_forces, same arguments, with the six sums F_p xyz, F_v xyz written to out_dev
 * (device, 6 doubles) asynchronously on the stream.  The call allocates nothing and does
 * not synchronise: its block partials live in a 48 KiB array that the library holds on
 * each GPU for the life of the process (6 sums x 1,024 blocks; the launch is capped at
 * 1,024 blocks, so every cut count fits).  The sums are bit-identical to ibm_forces'.
 * All calls on one GPU share that array: calls that overlap on one GPU (different
 * streams, or different contexts on concurrent streams) race; serialise them. */
int ibm_forces_noalloc(ibm_ctx* ctx, void* const u_dev[3], const double* p_dev, const void* nut_dev, double nu,
                       const double* wall_dev, double* out_dev, void* stream);

/* Near-field surface pressure and pressure force by Shepard interpolation (eq. (force)).
 * At every vertex X of a triangle (unit normal n from the right-handed vertex order)
 * the cell-centre pressure is averaged with weights 1/|X - x_k|^2 over the eight cell
 * centres x_k spanning the dual cell that contains X, separately for the points in
 * front (n . (x_k - X) > 0) and behind (< 0); points in the triangle's plane and
 * outside the grid are left out.  A triangle's front / back value is the mean over
 * its vertices that have one on that side; its force is A n (p_back - p_front), a side
 * without points contributing nothing.
 * thin_filter != 0 applies the filter Z of eq. (force_filter): a point gets weight zero
 * at a vertex when the segment from the vertex to it crosses a triangle of tri_dev at a
 * parameter t in (1e-6, 1] (Moller-Trumbore, edges inclusive; contacts at the vertex
 * itself do not count), so values from beyond the other face of a plate thinner than a
 * cell are cancelled.  The first filtered call allocates its triangle bins (4x4x4
 * cells, grow-only, freed by ibm_destroy); IBM_ERR_ARG when the bin lists would exceed
 * 2^31 entries.
 *   tri_dev   ntri x 3 vertices x 3 doubles (device; the layout ibm_tag_geometry takes)
 *   p_dev     cell pressure (device, FP64, the context's grid)
 *   side_dev  optional (device): ntri x 2 doubles, front and back pressure per
 *             triangle (NaN for a side without points, and for zero-area triangles)
 *   force_host[3]  the pressure force summed over the triangles (per-block partial
 *             sums in block order: deterministic).
 * Needs built stencils (for the grid).  Synchronises the stream.  Returns
 * IBM_ERR_ARG for ntri < 0 or null pointers. */
int ibm_shepard_force(ibm_ctx* ctx, const double* tri_dev, int64_t ntri, const double* p_dev, int32_t thin_filter,
                      double* side_dev, double force_host[3], void* stream);

/* ---- Learned preconditioner (an extension layered on the pressure solve of
 * eq. (poisson); the paper itself uses plain Krylov solves).
 *
 * Operator: a linear, symmetric positive semi-definite convolutional network of four
 * 3x3x3 convolutions with 16 channels and a geometry gate,
 *     G = hsig(Wg * g),  K x = W2 * ((W1 * x) . G),  net(x) = K^T K x,
 * with hsig(v) = min(max(v/4 + 1/2, 0), 1), g the open-face fraction of the cell
 * (open pressure faces / 6), "*" a
 * zero-padded 3x3x3 cross-correlation (taps at the grid faces are zero), K^T the
 * adjoint (flipped, transposed convolutions) and "." the per-channel product.  As the
 * preconditioner of IBM_SOLVER_FCG_CNN it maps a residual r to
 *     z = D^-1 r + s * net(r / s),   s = RMS of r over the cells,
 * D the diagonal of A = -L (symmetric positive definite; Jacobi for zero weights),
 * or, when the solver options' omega lies in (0, 1], that map between two damped
 * Jacobi steps (the smoothed form of ibm_cnn_precondition).  The network is trained
 * as the map alone.
 * Weights: IBM_CNN_NWEIGHTS floats: W1[t][0][co] (432 at offset 0), W2[t][ci][co]
 * (6912 at 432), Wg[t][0][co] (432 at 7344), row-major, tap
 * t = (dz+1)*9 + (dy+1)*3 + (dx+1) for offsets in {-1,0,1}.  The FP32 master copy
 * lives on the device.
 * Arithmetic: BF16 operands on the matrix cores with FP32 accumulation; activations
 * and backward signals are stored in BF16 (channels-last).
 * Field buffers are device memory, x fastest (cell c = i + nx*(j + ny*k)). */
#define IBM_CNN_NWEIGHTS 7776
typedef struct ibm_cnn ibm_cnn;

/* Creates a network on the current HIP device with all weights zero and workspace for
 * grids of up to max_cells cells: about 380 bytes per cell, or 72 with
 * IBM_CNN_INFERENCE_ONLY in flags (then only ibm_cnn_set/get_weights,
 * ibm_cnn_forward, ibm_cnn_precondition and the solver use it; training and backward
 * calls return IBM_ERR_ARG). */
#define IBM_CNN_INFERENCE_ONLY 1
int ibm_cnn_create(int64_t max_cells, int32_t flags, ibm_cnn** out);
int ibm_cnn_destroy(ibm_cnn* net);
/* Host FP32 weights in, n = IBM_CNN_NWEIGHTS; resets the Adam state.  Synchronous. */
int ibm_cnn_set_weights(ibm_cnn* net, const float* w_host, int64_t n);
int ibm_cnn_get_weights(ibm_cnn* net, float* w_host, int64_t n);
/* Network output y = net(x) (cells floats) for the input x_dev = cells x 2 BF16 bit
 * patterns (channel 0 = x, channel 1 = g) on an nx x ny x nz grid.  Keeps the
 * activations for ibm_cnn_backward. */
int ibm_cnn_forward(ibm_cnn* net, const uint16_t* x_dev, float* y_dev, int32_t nx, int32_t ny, int32_t nz,
                    void* stream);
/* Backward pass of the last forward for a scalar J with dJ/dy = dy (cells floats,
 * rounded to BF16): dJ/dw into dw_dev (IBM_CNN_NWEIGHTS floats, weight layout) and,
 * when dx_dev != NULL, dJ/dx and dJ/dg interleaved (cells x 2 floats). */
int ibm_cnn_backward(ibm_cnn* net, const float* dy_dev, float* dw_dev, float* dx_dev, void* stream);
/* Training loss of one pair (b, p) with L p = b on the context's stencil: with
 * f = -b and h = the preconditioned f,  loss = 1 - (f.h)^2 / ((f.p)(h.A h)), the
 * A-norm distance of p from the best multiple of h relative to |p|_A^2 (in [0,1],
 * invariant to the scale of h).  h is ibm_cnn_precondition's z for the same omega
 * (0: the network's map alone; in (0, 1]: the smoothed form, with the network trained
 * as its inner map M; the smoothing steps of the loss are FP64); other omega:
 * IBM_ERR_ARG.  loss_out (host) and, when
 * dw_dev != NULL, the gradient in the weights.  Synchronises the stream. */
int ibm_cnn_loss(ibm_cnn* net, ibm_ctx* ctx, const double* b_dev, const double* p_dev, double omega,
                 double* loss_out, float* dw_dev, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, FP32 moments) on that loss; loss_out
 * gets the loss before the update.  Synchronises the stream. */
int ibm_cnn_train_step(ibm_cnn* net, ibm_ctx* ctx, const double* b_dev, const double* p_dev, float lr,
                       double omega, double* loss_out, void* stream);
/* z = D^-1 r + s net(r/s) on the context's grid and geometry (r, z: cells floats,
 * 16-byte aligned).  omega in (0, 1]: that map M between two damped Jacobi steps
 * S = omega D^-1,  z1 = S r,  z2 = z1 + M(r - A z1),  z = z2 + S (r - A z2)  (symmetric,
 * positive definite for omega < 1; needs nx % 4 == 0); omega = 0: M itself.  Other
 * omega: IBM_ERR_ARG. */
int ibm_cnn_precondition(ibm_cnn* net, ibm_ctx* ctx, const float* r_dev, float* z_dev, double omega, void* stream);
/* Preconditioner used by IBM_SOLVER_FCG_CNN on this context (NULL detaches); the network
 * must cover the grid and outlive its use.  Attaching is set-up: it sizes the network's
 * per-grid partial sums (a device allocation when the grid is larger than any it was
 * attached to before), so ibm_step and ibm_poisson_solve allocate nothing; a solve on a
 * grid the network was not attached to fails with IBM_ERR_ARG. */
int ibm_ctx_set_preconditioner(ibm_ctx* ctx, ibm_cnn* net);

/* Building-cube grid (Sec. 2.2): the domain is tiled by K[0] x K[1] x K[2] coarse cubes
 * of n^3 cells of size dx0 (n even); a coarse cube with refine_host[kx + K0 (ky + K1 kz)]
 * != 0 is replaced by 8 fine cubes of n^3 cells of size dx0/2 (two fixed levels, a
 * factor of two apart).  Cube order: coarse cubes in z, y, x order, a refined one
 * contributing its 8 fine cubes in z, y, x order.  Each cube is stored as (n + 4)^3
 * doubles (two halo layers per face, x fastest); cube q starts at q (n + 4)^3.
 * Allocates the halo tables on the current device (host memory is read once); the
 * exchange, operator and SOR calls must run with that device current, else they return
 * IBM_ERR_ARG.  A failed create leaves *out untouched and frees what it allocated. */
typedef struct ibm_bcm ibm_bcm;
int ibm_bcm_create(const int32_t K[3], int32_t n, double dx0, const double origin[3], const uint8_t* refine_host,
                   ibm_bcm** out);
int ibm_bcm_destroy(ibm_bcm* grid);
/* Counts (any of the outputs may be NULL): cubes, values of the storage, face-halo
 * cells; levels_host[ncubes] (0 coarse, 1 fine) and origins_host[3 ncubes] (x, y, z of
 * each cube's first cell in fine-cell units). */
int ibm_bcm_info(const ibm_bcm* grid, int64_t* ncubes, int64_t* size, int64_t* nhalo, int32_t* levels_host,
                 int32_t* origins_host);
/* Fills the face halos (both layers; edges and corners untouched) of every cube of
 * data_dev in place: from a cube of the same or a coarser level the cell containing the
 * halo cell's centre (a copy, the paper's zero-order interpolation), from finer cubes the
 * mean of the 8 fine cells inside it (averaging), at the domain boundary the mirror of
 * the cube's own cells (layer l takes interior cell l - 1 from the face). */
int ibm_bcm_exchange(const ibm_bcm* grid, double* data_dev, void* stream);
/* y = L x on every cube interior: (sum of the six axis neighbours - 6 x_c) / dx^2 with the
 * cube's own dx, neighbours read from its storage (exchange first); halos of y are not
 * written; x and y distinct. */
int ibm_bcm_laplacian(const ibm_bcm* grid, const double* x_dev, double* y_dev, void* stream);
/* Red-black SOR on the cubes (Sec. 2.1's alternative solver on this grid): `sweeps`
 * sweeps, each two half sweeps of an exchange of x followed by the update of every
 * interior cell of one colour (parity of its cube-local i + j + k) by
 * x_c += omega (b_c - (L x)_c) / (-6 / dx^2).  b_dev (cube storage; interiors read) and
 * x_dev (in/out) distinct; 0 < omega < 2.  Asynchronous on the stream. */
int ibm_bcm_sor(const ibm_bcm* grid, const double* b_dev, double* x_dev, double omega, int32_t sweeps,
                void* stream);

/* Immersed geometry on the cubes: blocked_dev holds the blocked bits (one byte per cell,
 * bit d = direction d, as ibm_tag_geometry writes them) of the uniform grid of one level
 * over the whole domain: level 0 has K[a] n cells per axis of size dx0, level 1 twice as
 * many of size dx0 / 2, cell c = i + nx (j + ny k).  Every cube of that level takes the
 * bits of its own cells; a cube cell's face is blocked as the segment of its level's
 * grid, also toward a cube of the other level.  From then on ibm_bcm_laplacian and
 * ibm_bcm_sor give blocked faces the pressure ghost p_GC = p_c (Neumann, Sec. 2.3.2) and
 * SOR divides by the open-face count (a cell without open faces keeps its value).  The
 * first call allocates one byte per cube cell (set-up); call once per level. */
int ibm_bcm_set_blocked(ibm_bcm* grid, int32_t level, const uint8_t* blocked_dev, void* stream);

/* The pressure solve on the cubes: L x = b over the cube interiors (Sec. 2.1 names
 * BiCGStab and red-black SOR for the Poisson equation; Sec. 2.2 puts it on this grid),
 * L = ibm_bcm_exchange followed by ibm_bcm_laplacian (with the geometry of
 * ibm_bcm_set_blocked, if set).  b_dev and x_dev are cube storage (interiors read; x in/out:
 * its interiors are the initial guess and the result, its face halos are left as last
 * exchanged); distinct.
 *  kind IBM_BCM_BICGSTAB: unpreconditioned BiCGStab from x (van der Vorst 1992); stops
 *    when ||r|| <= tol ||b|| at the start of an iteration or ||s|| <= tol ||b|| halfway
 *    (then x += alpha p only); max_iter iterations; the scalars stay on the device and
 *    the host reads them every check_every iterations (launches issued after the stop
 *    do nothing).  b = 0 gives x = 0.  A breakdown (r0.r = 0, r0.v = 0, t.s = 0 or
 *    t.t = 0) returns IBM_NOT_CONVERGED with x as it stands.
 *  kind IBM_BCM_SOR: red-black SOR sweeps with relaxation omega (0 < omega < 2), the true
 *    residual checked before the first sweep and after every check_every sweeps; stops
 *    at the first check with ||b - L x|| <= tol ||b||, or after max_iter sweeps.
 * Norms are over the interiors (sums in a fixed block order).  iters_out: iterations or
 * sweeps made; rel_residual_out: the true residual ||b - L x|| / ||b|| of the returned x
 * (0 for b = 0).  Returns IBM_OK, IBM_NOT_CONVERGED, IBM_ERR_NAN (non-finite residual).
 * The first call allocates the workspace, kept by the grid until ibm_bcm_destroy:
 * partial sums and a small state, and for BiCGStab six vectors of the storage size;
 * solves on one grid share it, so they must not overlap.  Synchronises the stream. */
enum { IBM_BCM_BICGSTAB = 0, IBM_BCM_SOR = 1 };
int ibm_bcm_solve(ibm_bcm* grid, int32_t kind, const double* b_dev, double* x_dev, double omega, double tol,
                  int32_t max_iter, int32_t check_every, int32_t* iters_out, double* rel_residual_out,
                  void* stream);

/* Measurement support (not part of the method).  When enabled, launches of the
 * pressure solve are bracketed by HIP events on its stream and the elapsed times are
 * collected at the end of each solve.  Slots: 0 = CG pass A (SpMV, <d,q>; for the
 * learned solve: the whole preconditioner application), 1 = CG pass B (update, <r,r>,
 * <r,z>; for the learned solve: passes A and B), 2 = the dominant kernel of the
 * learned preconditioner (its fused forward half, the input scaling and both forward
 * convolutions).  ibm_timing_read fills out[0..2] =
 * accumulated milliseconds per slot, out[3..5] = launches per slot, out[6] =
 * iterations that did work (launches after convergence exit at once), out[7] =
 * cells, out[8] = cuts, out[9] = precision; reset != 0 zeroes the accumulators.
 * Enabling creates the events once (host objects, no device memory). */
int ibm_timing_enable(ibm_ctx* ctx, int32_t on);
/* Progress hook (measurement support): when set, the pressure solve calls
 * fn(user, iterations so far in this solve, current <r,r> of the recursive residual)
 * from the calling thread at each of its host convergence polls, and for the mixed kinds
 * fn(user, iterations so far, -(relative FP64 residual)) at each FP64 residual check
 * (a negative third argument).  NULL removes it. */
typedef void (*ibm_progress_fn)(void* user, int64_t iterations, double rr);
int ibm_set_progress(ibm_ctx* ctx, ibm_progress_fn fn, void* user);
int ibm_timing_read(ibm_ctx* ctx, double out[10], int32_t reset);
/* One timed slot: out[0] = accumulated milliseconds, out[1] = launches; reset != 0 zeroes
 * that slot.  Slots 0-2 as above, 3 = the near-field force kernel, 4-8 = the five
 * BiCGStab passes of the Crank-Nicolson predictor (4: new direction p; 5: v = A p;
 * 6: s = r - alpha v; 7: t = A s; 8: update of x and r), 9 = the momentum predictor
 * kernel of ibm_step (right-hand side H with its face values, and the AB2 update or
 * the Crank-Nicolson right-hand side). */
int ibm_timing_slot(ibm_ctx* ctx, int32_t slot, double out[2], int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* IBM_H */
