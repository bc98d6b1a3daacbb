/*
 * wwbi.h -- C ABI of the MI355X boundary-integral water-wave solver.
 *
 * The method is the one of Ambrose, Camassa, Marzuola, McLaughlin, Robinson
 * and Wilkening, "Numerical algorithms for water waves with background flow
 * over obstacles and topography" (arXiv 2108.01786).  Given the free surface
 * zeta_0, the bottom zeta_1 and obstacles zeta_2..zeta_N (Sec. 2), the
 * surface potential phi~ (velocity-potential method, Sec. 3) or the vortex
 * sheet strength gamma_0 (Sec. 4.1), and the multi-valued flow data V1, a_j,
 * z_j (Sec. 3, decomposition of Phi), the library returns the normal
 * velocity U = dphi/dn on the free surface.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Boundary k is sampled at alpha_km = 2 pi m / M_k, m = 0..M_k-1
 *    (Sec. 3.3).  Node arrays are concatenated boundary by boundary:
 *    surface (k = 0), bottom (k = 1), obstacles (k = 2..nb-1).
 *  - The surface and bottom run left to right with
 *    zeta(alpha + 2 pi) = zeta(alpha) + 2 pi; obstacles are closed curves
 *    traversed clockwise (fluid on the left, Sec. 2).
 *  - Every node, and every point given for evaluation inside the fluid, has
 *    |y| <= 30 (WWBI_EINVAL_RANGE otherwise).
 *  - Pointers marked (device) are HIP device pointers; (host) are host
 *    pointers.  The caller owns every input and output buffer.  The context
 *    owns its workspace, which grows to the largest problem seen and is then
 *    reused (a call on an already-seen size allocates nothing).
 *  - All work is enqueued on the context's stream; every call returns after
 *    its results are complete.  A context must not be used by two threads
 *    at once.
 *  - Return value: 0 = OK; < 0 = invalid input or runtime failure, outputs
 *    untouched; > 0 = numerical warning, outputs hold the best iterate.  No
 *    C++ exception crosses this interface.  The report, when given, is
 *    always filled.
 */
#ifndef WWBI_H
#define WWBI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define WWBI_OK                   0
#define WWBI_EINVAL_NULL         -1  /* a required pointer is NULL                     */
#define WWBI_EINVAL_SIZE         -2  /* nb < 2, nb > WWBI_MAX_BOUNDARIES, M_k odd or < 8 */
#define WWBI_EINVAL_NONFINITE    -3  /* NaN or Inf in the node data or the potential   */
#define WWBI_EINVAL_ORIENTATION  -4  /* an obstacle is not clockwise, or the surface or
                                        bottom does not run left to right             */
#define WWBI_ECAPACITY           -5  /* workspace allocation failed                    */
#define WWBI_EHIP                -6  /* a HIP runtime call failed                      */
#define WWBI_EINVAL_OPTS         -7  /* option out of range                            */
#define WWBI_EINVAL_RANGE        -8  /* a node has |y| > 30: far pairs use e^{-y} in
                                        FP32 intermediate steps, whose range this keeps */
#define WWBI_ESCRATCH            -9  /* wwbi_solve_phi_noalloc: the problem's workspace
                                        exceeds the static scratch array               */
#define WWBI_NOT_CONVERGED        1  /* iteration budget spent before the tolerance    */
#define WWBI_STAGNATED            2  /* a restart cycle made no progress               */
#define WWBI_REFINE_STALLED       3  /* iterative refinement stopped contracting       */
#define WWBI_WARN_UNDERRESOLVED   4  /* omega's Fourier tail (report.tail_ratio) is above
                                        max(1e-12, 10 tol) on some boundary, at the scale
                                        of the solution: the grid does not resolve it
                                        (Sec. 7.1's test)                               */

#define WWBI_MAX_BOUNDARIES      64

/* ---- option values ----------------------------------------------------- */
#define WWBI_FP64                 0  /* FP64 matrix and matvecs                          */
#define WWBI_FP32_REFINED         1  /* FP32 matrix/matvec (FP32 accumulation) inside
                                        FP64 iterative refinement                      */
#define WWBI_MATVEC_AUTO          0  /* stored matrix                                    */
#define WWBI_MATVEC_STORED        1  /* assemble once, stream the matrix per matvec      */
#define WWBI_MATVEC_ON_THE_FLY    2  /* recompute entries inside every matvec            */
#define WWBI_FLAG_PROFILE         1  /* time every launch of the dominant matvec kernel  */
#define WWBI_FLAG_NO_CORRECTION   2  /* drop the E_m rank-one blocks (singular system;
                                        for failure-detection tests only)              */
#define WWBI_FLAG_NO_RECYCLE      4  /* FP32_REFINED: every inner solve builds its own
                                        Krylov space (by default the later inner solves
                                        of a refinement deflate the space of the first:
                                        fewer Arnoldi steps, same FP64 stopping test)  */

/* spectral operators on one uniform periodic grid (Sec. 3.4), Nyquist mode zeroed */
#define WWBI_OP_D                 0  /* d/dalpha, symbol i k                             */
#define WWBI_OP_D2                1  /* d2/dalpha2, symbol -k^2                          */
#define WWBI_OP_H                 2  /* Hilbert transform, symbol -i sgn k               */
#define WWBI_OP_ABSD              3  /* |d| = H D, symbol |k|                            */

/* matrices exported by wwbi_debug_matrix */
/* surface representation of an evolution stage (wwbi_stage_rhs, wwbi_rk_step) */
#define WWBI_SURF_GRAPH           0  /* xi = alpha, state eta (Sec. 2.1)                 */
#define WWBI_SURF_HLS             1  /* tangent angle, state P theta (Sec. 2.2)          */

#define WWBI_MAT_A                0  /* velocity-potential system (Sec. 3.3)             */
#define WWBI_MAT_WALL             1  /* vortex-sheet wall system (Sec. 4.1)              */
#define WWBI_MAT_T                2  /* normal-velocity map T on the surface rows
                                        (Sec. 3.4): s U = u_mv + H gamma_0 / 2 + T gamma */

typedef struct wwbi_ctx wwbi_ctx;

/* Geometry and multi-valued flow data (Sec. 2; Sec. 3 decomposition of Phi). */
typedef struct {
    int32_t nb;               /* number of boundaries N+1, 2 <= nb <= 64             */
    const int32_t *M;         /* (host) nb node counts; each even and >= 8            */
    const double *x, *y;      /* (device) sum(M): zeta = x + i y                      */
    const double *dx, *dy;    /* (device) sum(M): zeta'                               */
    const double *ddx, *ddy;  /* (device) sum(M): zeta''                              */
    const double *zc;         /* (host) 2*(nb-2): (re, im) of z_j inside obstacle j   */
    const double *a;          /* (host) nb-2: circulation parameters a_j              */
    double V1;                /* background-flow strength                             */
    const double *psi_wall;   /* (device) sum(M)-M_0 stream-function data on the walls,
                                 or NULL for zero (the paper's problem)               */
} wwbi_geom;

typedef struct {
    double tol;          /* stop when ||b - A x||_2 <= tol ||b||_2 (true FP64 residual)   */
    double inner_tol;    /* FP32_REFINED: relative tolerance of each inner FP32 solve     */
    int32_t restart;     /* GMRES restart length, 1..WWBI_MAX_RESTART                      */
    int32_t max_iter;    /* budget of Arnoldi steps (all cycles, all refinement steps)     */
    int32_t precision;   /* WWBI_FP64 or WWBI_FP32_REFINED                                 */
    int32_t matvec;      /* WWBI_MATVEC_*                                                  */
    int32_t poll_every;  /* Arnoldi steps between host checks for the end of a cycle      */
    int32_t max_refine;  /* FP32_REFINED: maximum refinement steps                         */
    int32_t band;        /* FP32: same-boundary pairs with cyclic |l-m| <= band are
                            evaluated in FP64 and rounded (near-singular kernel)          */
    int32_t flags;       /* WWBI_FLAG_*                                                    */
    const double *x0;    /* (device) sum(M) warm start for omega, or NULL for zero        */
} wwbi_opts;

#define WWBI_MAX_RESTART 256
#define WWBI_HIST_MAX 32

typedef struct {
    int32_t status;
    int32_t iters;         /* Arnoldi steps taken (all cycles and refinement steps)       */
    int32_t restarts;      /* restart cycles                                              */
    int32_t refine_steps;  /* FP32_REFINED: inner solves                                  */
    double rel_resid;      /* final ||b - A x|| / ||b|| with the FP64 operator            */
    double ms_prep, ms_assemble, ms_solve, ms_U, ms_total;   /* HIP-event phase times     */
    int32_t n_matvec;      /* launches of the dominant matvec kernel (FLAG_PROFILE)       */
    int32_t pad0;
    double ms_matvec;      /* their summed HIP-event duration (FLAG_PROFILE)              */
    double bytes_matvec;   /* algorithmic bytes moved by one such launch                  */
    double tail_ratio;     /* wwbi_solve_phi: max over boundaries k of the root of the
                              energy of omega_k in its modes |k| >= 3 M_k / 8 over M_k^2
                              times the largest mean square of omega on any boundary
                              (Parseval: the tail's share at the solution's scale; 0
                              for other entry points)                                   */
    int32_t n_hist;        /* entries of resid_hist written (at most WWBI_HIST_MAX)       */
    int32_t pad1;
    double resid_hist[WWBI_HIST_MAX];
                           /* ||b - A x|| / ||b|| in the order measured: at the start of
                              every restart cycle of an FP64 GMRES solve (the true
                              residual) and after every step of an iterative refinement
                              (the FP64 residual; the largest over the systems of a
                              multi-RHS solve); the first WWBI_HIST_MAX values          */
} wwbi_report;

/* Fill *o with defaults: tol 1e-13, inner_tol 1e-7, restart 100, max_iter 2000,
 * FP64, stored matvec, poll every 2 steps, max_refine 8, band 16, no flags. */
void wwbi_default_opts(wwbi_opts *o);

/* Human-readable name of a status code (static string). */
const char *wwbi_status_str(int status);

/* Create a context on HIP device `device` bound to `hip_stream` (a hipStream_t;
 * NULL = the null stream).  Allocates only small bookkeeping buffers.
 * Returns WWBI_EHIP if the device cannot be used. */
int wwbi_create(wwbi_ctx **ctx, int32_t device, void *hip_stream);

/* Rebind the context to another stream (e.g. the caller's current stream). */
int wwbi_set_stream(wwbi_ctx *ctx, void *hip_stream);

/* Release every buffer and the context itself.  NULL is accepted. */
int wwbi_destroy(wwbi_ctx *ctx);

/* Pre-size the workspace for up to `max_unknowns` nodes, restart length
 * `max_restart`, and a stored matrix of the given precision (WWBI_FP64 or
 * WWBI_FP32_REFINED; -1 = no stored matrix).  Optional: a solve allocates
 * (hipMalloc, after freeing a smaller buffer) every part of the workspace
 * that is missing or too small for it, inside the call; after wwbi_reserve
 * for the largest problem, solves of that size or smaller allocate nothing,
 * except the FP64 matrix copy of a refined multi-RHS solve
 * (wwbi_solve_phi_multi).  For no allocation at all, see
 * wwbi_solve_phi_noalloc. */
int wwbi_reserve(wwbi_ctx *ctx, int64_t max_unknowns, int32_t max_restart, int32_t precision);

/* Velocity-potential solve (Sec. 3.2-3.4).
 *   phi    (device) M_0: surface potential phi~ at the surface nodes.
 * Assembles A (Sec. 3.3: K, G blocks with weights 1/M_j, -I/2 / +I/2 on the
 * diagonal blocks, self limits Im{zeta''/(2 zeta')}, rank-one blocks
 * E_m = e e^T / M_m for m >= 2) and b (b_0 = phi~, b_k = psi_wall - psi_mv),
 * solves A omega = b by restarted GMRES, and evaluates
 *   U = [Re{Phi_mv'(zeta) i zeta'} - |d| omega_0 / 2 - G_00^T D omega_0 / M_0
 *        + sum_j K_j0^T D omega_j / M_j] / |zeta'|                  (Sec. 3.4).
 * Outputs:
 *   U      (device) M_0;
 *   omega  (device) sum(M), or NULL;
 *   psi_k  (host)   nb-2 stream-function constants psi|_k = mean(omega_k), or NULL.
 * Resolution check (the paper's Fourier-tail test, Sec. 7.1): the solve also
 * measures, on every boundary, the root of the energy of omega_k in its
 * modes |k| >= 3 M_k / 8 over M_k^2 times the largest mean square of omega on
 * any boundary, i.e. the tail at the solution's scale (report.tail_ratio holds
 * the largest).  Above
 * max(1e-12, 10 tol) a solve that otherwise succeeded returns
 * WWBI_WARN_UNDERRESOLVED, with its outputs as usual: typically a boundary
 * comes too close to another for its grid.
 */
int wwbi_solve_phi(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi, const wwbi_opts *o,
                   double *U, double *omega, double *psi_k, wwbi_report *rep);

/* Allocation-free variant of wwbi_solve_phi, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same solve, with the same inputs,
 * outputs, report and status codes, under these limits:
 *   - the matvec must be WWBI_MATVEC_ON_THE_FLY (precision WWBI_FP64 or
 *     WWBI_FP32_REFINED); no matrix is stored;
 *   - the whole per-solve workspace (Krylov basis, partial sums, node data,
 *     cycle state) lives in one static device array of
 *     WWBI_NOALLOC_SCRATCH_BYTES per GPU, which the library holds until the
 *     process ends.  It needs about (restart + 302) * 8 * round_up(n, 64)
 *     bytes for n = sum(M) unknowns (restart counted as at least 8): n up to
 *     15552 fits at restart 100 and up to 14528 at restart 128.  A larger
 *     problem returns WWBI_ESCRATCH before any work, outputs untouched;
 *   - o->max_iter + o->max_refine <= 4088 (host bookkeeping reserved by
 *     wwbi_create), else WWBI_EINVAL_OPTS.
 * The call allocates nothing: no hipMalloc, hipFree or host allocation.  The
 * context must have been created by wwbi_create beforehand.  Every call on
 * one GPU shares that GPU's array, which keeps the last call's contents (each
 * call clears the part it uses first): calls that overlap on one GPU (other
 * streams, other threads, other contexts) race and must not be issued.  The
 * context's own workspace is neither used nor changed.  The call returns
 * after its work on the context's stream has completed. */
#define WWBI_NOALLOC_SCRATCH_BYTES (48LL * 1024 * 1024)
int wwbi_solve_phi_noalloc(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi,
                           const wwbi_opts *o, double *U, double *omega, double *psi_k,
                           wwbi_report *rep);

/* Vortex-sheet solve (Sec. 4.1).
 *   gamma0 (device) M_0: vortex sheet strength gamma_0 = -omega_0'.
 * Solves the wall system (-I/2 + K^dagger) gamma_w = -G_0k^dagger gamma_0
 * - s dphi_mv/dn (zero normal velocity on every wall) by GMRES and returns
 *   U = [H gamma_0 / 2 + G_00^dagger gamma_0 + sum_j K_j0^dagger gamma_j
 *        + s dphi_mv/dn] / |zeta'|.
 * Outputs: U (device) M_0; gamma_wall (device) sum(M)-M_0 or NULL.
 * Precision: FP64, or with a stored matvec and WWBI_FP32_REFINED, FP32
 * products of the wall operator (entries evaluated in FP64, stored rounded)
 * inside FP64 refinement with on-the-fly FP64 residuals; an on-the-fly
 * matvec always runs in FP64.  o->x0 warm-starts gamma_wall. */
int wwbi_solve_gamma(wwbi_ctx *ctx, const wwbi_geom *g, const double *gamma0, const wwbi_opts *o,
                     double *U, double *gamma_wall, wwbi_report *rep);

/* Tangential velocity on every boundary and the energy, from a
 * velocity-potential solution (no solve is run).
 *   phi    (device) M_0: the phi~ passed to wwbi_solve_phi; needed only for
 *          the energy (may be NULL when energy is NULL).
 *   omega  (device) sum(M): the densities returned by wwbi_solve_phi.
 *   tau, grav: surface tension and gravity of the energy (rho = 1).
 * Outputs (each may be NULL, not both):
 *   dphids (device) sum(M): the tangential derivative dphi/ds at every node,
 *          from gamma = (-D omega_0, D omega_j) by the Sec. 5.1 formulas:
 *          s dphi/ds_k = s dphi_mv/ds_k + [k = 0] gamma_0/2
 *             + sum_l K_0k(beta_l, alpha) gamma_0,l / M_0
 *             + sum_{j>=1} ( -[k = j] (H gamma_j)/2 - sum_l G_jk(beta_l, alpha) gamma_j,l / M_j ),
 *          with the surface on its fluid (lower) side.  With dphi/dn (U on the
 *          surface, 0 on the walls) it gives the velocity u - i v =
 *          (dphi/ds - i dphi/dn) |zeta'| / zeta'.
 *   energy (host) 1: E of Sec. 5.2, the trapezoid mean over the surface of
 *          tau s + g eta^2 xi' / 2 + psi phi_alpha / 2, plus sum_j a_j psi|_j / 2,
 *          with psi on the surface from the Plemelj limits of the Cauchy
 *          integrals and phi_alpha = D phi~ + d phi_mv / d alpha.
 * Errors: WWBI_EINVAL_NULL (omega, or both outputs, or phi with energy),
 * WWBI_EINVAL_NONFINITE (tau, grav, geometry or phi), and the geometry
 * checks of wwbi_solve_phi.  The report carries the timings only. */
int wwbi_tangential_energy(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi,
                           const double *omega, double tau, double grav, double *dphids,
                           double *energy, wwbi_report *rep);

/* Time derivative of the vortex sheet strengths (Sec. 4.2): the gamma_0,t
 * equation stacked on the wall equations,
 *   (I/2 + K_00^dagger) gamma_0,t - sum_j G_j0^dagger gamma_j,t = d/dalpha(e_0),
 *   G_0k^dagger gamma_0,t + (-I/2 + K_kk^dagger) gamma_k,t + sum_{j!=k} K_jk^dagger gamma_j,t
 *       = -d/dalpha(F_k0 gamma_0)                                   (k >= 1),
 *   e_0 = -W.W/2 + (V - W.t) gamma_0/(2s) - gamma_0^2/(8 s^2) + tau theta_alpha/s
 *         - grav eta - F_00 gamma_0,
 * where gamma = (-D omega_0, D omega_j), U and W (the Birkhoff-Rott velocity
 * plus grad phi_mv on the surface) come from a velocity-potential solve at
 * the state (geometry, phi~), and F_00, F_k0 take the regularised form with
 * zeta_t = (V + iU) zeta'/s.
 *   phi    (device) M_0: phi~ of the state.
 *   V      (device) M_0: tangential velocity of the surface parameterisation.
 *   tau, grav: surface tension and gravity.
 *   o: tol, restart, max_iter, matvec and precision apply to both solves, x0
 *      (an omega warm start) to the velocity-potential solve only.  The gamma_t
 *      system is solved in FP64 (stored or on the fly) or, with a stored matvec
 *      and WWBI_FP32_REFINED, by FP32 products (entries evaluated in FP64,
 *      stored rounded) inside FP64 refinement with on-the-fly FP64 residuals.
 * Outputs: gamma_t (device) sum(M), concatenated boundary by boundary;
 *   U (device) M_0 or NULL: the normal velocity of the state;
 *   rep_phi / rep (either may be NULL): reports of the velocity-potential
 *   solve and of the gamma_t stage (right-hand side, assembly, GMRES).
 * Returns the first error, else the gamma_t solve's warning, else the
 * velocity-potential solve's. */
int wwbi_solve_gamma_t(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi, const double *V,
                       double tau, double grav, const wwbi_opts *o, double *gamma_t, double *U,
                       wwbi_report *rep_phi, wwbi_report *rep);

/* One Runge-Kutta stage of the velocity-potential evolution: the time
 * derivatives of the surface variable q and of phi~ at the state (q, phi~)
 * with the walls of g held fixed.
 *   mode WWBI_SURF_GRAPH: q = eta on xi = alpha (Sec. 2.1); the surface is
 *     zeta = alpha + i eta with spectral derivatives; V = eta_alpha U and
 *     q_t = eta_t = sqrt(1 + eta_alpha^2) U.
 *   mode WWBI_SURF_HLS: q = P theta, the zero-mean tangent angle (Sec. 2.2);
 *     the curve is reconstructed with C, S = means of cos, sin P theta,
 *     P_0 theta = arg(C - iS), s_alpha = (C^2 + S^2)^(-1/2), and zero-mean
 *     antiderivatives shifted to xi(0) = 0 and zero mean height;
 *     V = antiderivative of theta_alpha U minus its mean with V(0) =
 *     U(0) eta'(0)/xi'(0) (Sec. 5); q_t = P[(U_alpha + V theta_alpha)/s_alpha].
 *   In both modes phi~_t = (phi~_alpha/s) V + (dphi~/dn) U - |grad phi|^2/2
 *     - grav eta + tau theta_alpha/s (Sec. 3.5, C(t) = 0).
 * g: the first M_0 entries of x, y, dx, dy, ddx, ddy must be writable device
 *    memory: the surface of the stage is written there (the walls are read).
 * q, phi (device) M_0: the state.  o: options of the velocity-potential
 *    solve (precision, tolerance, ...).
 * Outputs (device, M_0): q_t, phi_t; U and V may be NULL.
 * rep: the velocity-potential solve's report. */
int wwbi_stage_rhs(wwbi_ctx *ctx, const wwbi_geom *g, int32_t mode, const double *q,
                   const double *phi, double tau, double grav, const wwbi_opts *o, double *q_t,
                   double *phi_t, double *U, double *V, wwbi_report *rep);

/* One explicit Runge-Kutta step of the same evolution with the tableau
 * A (host, nstage x nstage row-major; entries on and above the diagonal are
 * ignored) and weights b (host, nstage), 1 <= nstage <= 16:
 *   stage i: (q_i, phi_i) = (q, phi) + h sum_{j<i} A_ij k_j, k_i = stage_rhs(q_i, phi_i);
 *   then (q, phi) += h sum_i b_i k_i, followed (filter != 0) by the 36th-order
 *   filter exp(-36 (|k| / (M_0/2))^36) on both (Sec. 5).
 * q, phi (device, M_0) are updated in place; g as for wwbi_stage_rhs.
 * rep: iterations summed over the stages, ms_solve = their solve time,
 * ms_total = wall time of the step. */
int wwbi_rk_step(wwbi_ctx *ctx, const wwbi_geom *g, int32_t mode, int32_t nstage,
                 const double *A, const double *b, double h, double *q, double *phi, double tau,
                 double grav, int32_t filter, const wwbi_opts *o, wwbi_report *rep);

/* Velocity on every boundary node from the densities omega of a
 * velocity-potential solve: u and v (device, sum(M)) with
 *   u - i v = (dphi/ds - i dphi/dn) |zeta'| / zeta'     (Sec. 5.1),
 * dphi/ds from the Sec. 5.1 formulas and dphi/dn from the Sec. 4.1 formulas
 * for every boundary (U on the surface; zero on the walls of the physical
 * problem up to the discretization error). */
int wwbi_boundary_velocity(wwbi_ctx *ctx, const wwbi_geom *g, const double *omega, double *u,
                           double *v);

/* Values inside the fluid of a periodic function analytic there, from its
 * values on every boundary node (the Helsing-Ojala rule of the appendix to
 * Sec. 5.1):
 *   f(z) = sum_km lam_km f_km / sum_km lam_km,
 *   lam_km = sigma_k / M_k * (1/2) cot((zeta_km - z)/2) zeta'_km,
 * sigma_0 = -1 (the positively oriented boundary runs along the free surface
 * against its parameter), sigma_k = +1 for the bottom and the obstacles.
 * Spectrally accurate up to and on the boundary; a point equal to a node
 * (or a period image of one) takes that node's value.
 *   f_re, f_im (device) sum(M); zx, zy (device) npts points inside the fluid;
 *   out_re, out_im (device) npts.
 * The points are checked first (here, in wwbi_interior_velocity and in
 * wwbi_pressure): WWBI_EINVAL_NONFINITE for a non-finite coordinate,
 * WWBI_EINVAL_RANGE for |y| > 30, outputs untouched. */
int wwbi_interior_eval(wwbi_ctx *ctx, const wwbi_geom *g, const double *f_re,
                       const double *f_im, int32_t npts, const double *zx, const double *zy,
                       double *out_re, double *out_im);

/* Fluid velocity (u, v) at npts points inside the fluid from the densities
 * omega: the boundary values of u - i v (wwbi_boundary_velocity), which is
 * analytic and periodic in the fluid, carried inside by the Helsing-Ojala rule.
 *   zx, zy, u, v (device) npts. */
int wwbi_interior_velocity(wwbi_ctx *ctx, const wwbi_geom *g, const double *omega,
                           int32_t npts, const double *zx, const double *zy, double *u,
                           double *v);

/* Pressure inside the fluid (Sec. 5.1): p / rho = C - phi_t - |grad phi|^2/2 - grav y.
 * phi_t - C is harmonic with the Dirichlet data tau kappa - |grad phi|^2/2 -
 * grav eta on the surface (Laplace-Young: p = -tau kappa there) and zero
 * normal derivative on the walls: the matrix A of the velocity-potential
 * solve (assembled once, used for both solves) with b_0 = that data and
 * b_k = 0.  Its Cauchy integrals take their fluid-side boundary values from
 * the Plemelj formulas and are carried inside by the Helsing-Ojala rule, as
 * is u - i v.
 *   phi (device) M_0; tau, grav; o as for wwbi_solve_phi.
 *   zx, zy (device) npts points inside the fluid; p (device) npts.
 * rep: the velocity-potential solve's report with the second solve's
 * iterations added. */
int wwbi_pressure(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi, double tau,
                  double grav, const wwbi_opts *o, int32_t npts, const double *zx,
                  const double *zy, double *p, wwbi_report *rep);

/* Adjoint of the velocity-potential solve.  With omega from wwbi_solve_phi on
 * the same inputs and dJdU = dJ/dU (device, M_0), returns the gradient of J
 * with respect to the surface samples (walls held fixed):
 *   g_phi, g_x, g_y, g_dx, g_dy, g_ddx, g_ddy  (device, M_0 each; overwritten).
 * Uses one transpose GMRES solve A^T lambda = c with the options' precision
 * and the derivative of every kernel entry that touches the surface. */
int wwbi_adjoint_phi(wwbi_ctx *ctx, const wwbi_geom *g, const double *omega, const double *dJdU,
                     const wwbi_opts *o, double *g_phi, double *g_x, double *g_y, double *g_dx,
                     double *g_dy, double *g_ddx, double *g_ddy, wwbi_report *rep);

/* Tangent-linear model of the velocity-potential solve (Sec. 3.2-3.4
 * differentiated; the forward-mode counterpart of wwbi_adjoint_phi), walls
 * fixed.  For nd directions of the surface's node data and phi~, the
 * directional derivatives of U:
 *   d omega_i = A^{-1} (dphi~_i e_0 - (dA_i) omega),
 *   dU_i = (d u_mv + (dT_i) gamma + T d gamma_i + H d gamma_0,i / 2 - U ds_i) / s,
 * with gamma = (-D omega_0, D omega_j).  The nd systems share A and are
 * solved together by the multi-RHS solver (wwbi_solve_phi_multi's, with the
 * matrix read once per Arnoldi step for all of them).
 *   omega  (device) sum(M): the solution at this geometry and phi~ (from
 *          wwbi_solve_phi); phi~ itself enters only through its directions.
 *   nd     1..32 directions.
 *   dirs   (device) 7 x nd x M_0: component c of direction i at offset
 *          (c * nd + i) * M_0, the components being x, y, x', y', x'', y''
 *          of the surface nodes and phi~ (a displacement of the surface
 *          comes with its own derivatives x', x'', ...).
 *   dU     (device) nd x M_0, direction i at offset i * M_0.
 *   domega (device) nd x sum(M), or NULL.
 * Options as for wwbi_solve_phi_multi (a stored matrix, no warm start).
 * Errors: WWBI_EINVAL_OPTS for nd outside 1..32, an on-the-fly matvec or a
 * warm start; WWBI_EINVAL_NONFINITE for a non-finite direction entry;
 * WWBI_EINVAL_SIZE when 7 * nd * M_0 exceeds 2^31 - 1. */
int wwbi_tangent_phi(wwbi_ctx *ctx, const wwbi_geom *g, const double *omega, int32_t nd,
                     const double *dirs, const wwbi_opts *o, double *dU, double *domega,
                     wwbi_report *rep);

/* Several right-hand sides against one matrix: solves A omega_i = rhs_i,
 * i < n, with the matrix read once per Arnoldi step for all i (matrix-core
 * product).  rhs, omega: (device) sum(M) x n, column i at offset i*sum(M).
 * With WWBI_FP32_REFINED the context also allocates and assembles an FP64
 * copy of the matrix (8 bytes per entry beside the FP32 one: 839 MB at 10240
 * unknowns, 13.4 GB at 40960), kept until wwbi_destroy, from which the
 * residuals of all systems are formed in one matrix-core pass; when that copy
 * cannot be allocated they are formed on the fly, one system at a time.
 * report.bytes_matvec counts the FP32 matrix of the inner products.
 * Errors: WWBI_EINVAL_OPTS for n outside 1..32, an on-the-fly matvec or a
 * warm start; WWBI_EINVAL_NONFINITE for a non-finite right-hand side entry
 * (omega untouched); the geometry is checked as for wwbi_solve_phi.
 * The lockstep path pays off from a few systems on; a single system solves
 * faster through wwbi_solve_phi (at 10240 unknowns, refined: 3.3 ms against
 * 5.9 ms here; 32 systems take 8.9 ms here). */
int wwbi_solve_phi_multi(wwbi_ctx *ctx, const wwbi_geom *g, const double *rhs, int32_t n,
                         const wwbi_opts *o, double *omega, wwbi_report *rep);

/* out = alpha * Op(f) + beta * out on one uniform periodic grid of n points
 * (n even, >= 8); f, out (device) n, may not alias. */
int wwbi_spectral(wwbi_ctx *ctx, int32_t n, const double *f, int32_t op, double alpha,
                  double beta, double *out);

/* Surface samples from periodic displacements: zeta = alpha + xt + i yt with
 * spectral zeta', zeta'' (x = alpha_m + xt_m, x' = 1 + D xt, x'' = D2 xt,
 * likewise for y).  All pointers (device) n.  The outputs may point into the
 * concatenated geometry arrays. */
int wwbi_surface_fill(wwbi_ctx *ctx, int32_t n, const double *xt, const double *yt, double *x,
                      double *y, double *dx, double *dy, double *ddx, double *ddy);

/* Chain rule of wwbi_surface_fill: g_xt = g_x - D g_dx + D2 g_ddx and likewise
 * for y (D is antisymmetric, D2 symmetric).  All pointers (device) n. */
int wwbi_surface_fill_adjoint(wwbi_ctx *ctx, int32_t n, const double *g_x, const double *g_y,
                              const double *g_dx, const double *g_dy, const double *g_ddx,
                              const double *g_ddy, double *g_xt, double *g_yt);

/* Export a matrix for inspection: `which` = WWBI_MAT_A (sum(M)^2),
 * WWBI_MAT_WALL ((sum(M)-M_0)^2) or WWBI_MAT_T (M_0 x sum(M); FP64 only),
 * row-major, FP64 (precision WWBI_FP64) or
 * FP32 (WWBI_FP32_REFINED, with the FP64 band of width `band`).
 * out (device) must hold n*n elements of that type.  The matrix is assembled
 * in the context's matrix workspace (padded rows) and copied out. */
int wwbi_debug_matrix(wwbi_ctx *ctx, const wwbi_geom *g, int32_t which, int32_t precision,
                      int32_t band, void *out);

/* One product with the velocity-potential matrix: y = A x (transpose = 0) or
 * y = A^T x (transpose = 1), with the given precision and matvec mode.  x, y
 * (device) sum(M).  For tests and benchmarks of the matvec kernels. */
int wwbi_matvec(wwbi_ctx *ctx, const wwbi_geom *g, const double *x, double *y, int32_t precision,
                int32_t mode, int32_t transpose, int32_t band, wwbi_report *rep);

#ifdef __cplusplus
}
#endif
#endif /* WWBI_H */
