// Internal declarations shared by the HIP translation units of libwwbi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wwbi.h"

namespace wwbi {

constexpr int kMaxB = WWBI_MAX_BOUNDARIES;

// Largest |y| of a node.  Far pairs work with E = e^{i zeta}, |E| = e^{-y}:
// the FP32 assembly forms |E_q - E_p|^2 and the FP64 far tiles seed their
// reciprocal of it in FP32, so e^{+-2|y|} and the products of two such
// quantities must stay inside the FP32 normal range.  |y| <= 30 keeps them
// within it for every pair at least 1e-6 apart.
constexpr double kMaxAbsY = 30.0;

// Boundary layout: node p of boundary k has global index off[k] + m.
struct Layout {
    int nb;
    int n;                 // total nodes sum(M)
    int off[kMaxB + 1];
};

// Multi-valued flow data (Sec. 3): V1, a_j and z_j for obstacles j = 2..nb-1.
struct Flow {
    double V1;
    int nobs;
    double a[kMaxB];
    double zx[kMaxB], zy[kMaxB];
};

// Device view of the prepared nodes.  x..dy are the caller's arrays; the rest
// is derived once per call by k_prep_nodes.
struct Nodes {
    const double *x, *y, *dx, *dy, *ddx, *ddy;
    const double *ex, *ey;   // E = e^{i zeta} = e^{-y} (cos x, sin x), leading part
    const double *exl, *eyl; // trailing part: E = (ex + exl) + i (ey + eyl) to ~1e-30
    const int *bid;        // boundary index of each node
    const int *loc;        // index m within its boundary
    const int *Mk;         // node count M_k of its boundary
    const double *w;       // quadrature weight 1/M_k of the node's boundary
    const double *s;       // |zeta'|
    const double *lre;     // Re{zeta''/(2 zeta')}
    const double *lim;     // Im{zeta''/(2 zeta')}
    // per cell of kCellNodes consecutive nodes: centre (2), radius of a disc
    // holding their E values, and the largest |E| (k_cells)
    const double *cell;
    const int *nlist;      // per cell: its near-pair list (kNearStride ints)
    int n;
    int near;              // the geometry has near pairs outside the band (set-up)
};

// Krylov vectors an FP32 inner solve may hand on to the later inner solves of
// its refinement (recycled space); the basis array keeps room for them in
// front of the Arnoldi basis.
constexpr int kRecycleMax = 64;

constexpr int kCellNodes = 64;
// Near-pair cut: a pair with |E_q - E_p| < max(|E_p|, |E_q|) / kNearCut takes
// the exact-difference cotangent (kappa64 and the on-the-fly near-pair fix).
constexpr double kNearCut = 64.0;
// Near-pair list of a cell (k_near_cells): its count (-1 when more than
// kNearList cells hold near pairs with it), then the cells in increasing order.
constexpr int kNearList = 31;
constexpr int kNearStride = kNearList + 1;

// sum_{k < ns} part[k * stride + i], added in increasing k; eight loads are
// issued before their additions (the slices are streamed from HBM/L2).
__device__ __forceinline__ double sum_slices(const double *part, int ns, long stride, long i) {
    double acc = 0.0;
    int k = 0;
    for (; k + 8 <= ns; k += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(long)(k + u) * stride + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; k < ns; ++k) acc += part[(long)k * stride + i];
    return acc;
}

// The same sum over the W waves of a block whose 64 lanes are 64 outputs:
// wave w sums slices [ns w / W, ns (w + 1) / W) in increasing k, and the W
// sums are added in wave order.  Every thread of the block calls it (it holds
// a barrier); the result is valid in wave 0.  One lane alone would sum all ns
// slices in dependent rounds of loads.
template <int W>
__device__ __forceinline__ double sum_slices_waves(const double *part, int ns, long stride,
                                                   long i, bool live, double (*red)[64]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k0 = (int)((long)ns * wv / W), k1 = (int)((long)ns * (wv + 1) / W);
    red[wv][lane] = live ? sum_slices(part + (long)k0 * stride, k1 - k0, stride, i) : 0.0;
    __syncthreads();
    double s = 0.0;
    if (wv == 0)
        for (int w = 0; w < W; ++w) s += red[w][lane];
    return s;
}
constexpr int kSliceWaves = 8;

// Device-resident GMRES cycle state (one per Krylov solve in flight).
struct GState {
    int active;        // 1 while the current restart cycle runs
    int jdone;         // Arnoldi steps completed in the current cycle
    int breakdown;
    int its;           // Arnoldi steps since the solve began (all cycles)
    double bnorm;      // ||b||
    double tol_abs;    // tol * ||b||
    double beta;       // residual norm at the start of the cycle
    double resid;      // current residual estimate |g_{j+1}|
    int cyc;           // host-visible copy only: the cycle whose end it records
    int pad;
};

// Strides of a batch of Krylov solves run in lockstep (system = blockIdx.y).
// A single solve uses nsys = 1 and zero strides.
struct Bat {
    int nsys;
    long v;      // Krylov basis V (doubles)
    long v32;    // FP32 copy of the newest basis vector (floats)
    long vec;    // length-n vectors: x, r, w, b
    long p;      // partial sums
    long h;      // Hessenberg matrix
    long rot;    // Givens cosines/sines, g and y
};
constexpr Bat kSingle{1, 0, 0, 0, 0, 0, 0};

// circulant row (1/2) cot(pi n / M) of the Hilbert regulariser h (n != 0)
constexpr int kOpHalfCot = 100;

struct Ctx;   // host context (api.hip)

// ---- kernels_geom.hip --------------------------------------------------------
void launch_prep_nodes(const Layout &L, const double *x, const double *y, const double *dx,
                       const double *dy, const double *ddx, const double *ddy, int *bid,
                       int *loc, int *Mk, double *w, double *s, double *lre, double *lim,
                       double *ex, double *ey, double *exl, double *eyl, hipStream_t st);
void launch_cells(const Nodes &N, double *cell, hipStream_t st);
void launch_near_cells(const Nodes &N, int *lists, double *count, hipStream_t st);
// Input checks: per boundary k, out[4k..4k+3] = (non-finite samples, signed
// area, mean x', samples beyond the height limit); out[4 nb + 1] = 0 (the
// near-pair count, added by launch_near_cells); out[4 nb + 2 + b] for
// b < validate_data_blocks(nphi): non-finite entries of the data array.
constexpr int kValidateBlocks = 64;
int validate_data_blocks(int nphi);
void launch_validate(const Layout &L, const Nodes &N, const double *phi, int nphi,
                     double *out, hipStream_t st);
void launch_rhs_phi(const Layout &L, const Nodes &N, const Flow &F, const double *phi,
                    const double *psi_wall, double *b, hipStream_t st);
void launch_umv(const Nodes &N, const Flow &F, int first, int count, double *out,
                hipStream_t st);
void launch_tmv(const Nodes &N, const Flow &F, int first, int count, double *out,
                hipStream_t st);
void launch_tangential_finalize(int n, int n0, const double *s, const double *tmv,
                                const double *gamma, const double *hg, const double *part,
                                int nsplit, double *out, hipStream_t st);
// gamma_t right-hand side pieces on the surface: fV = V gamma_0 / s, fU = U gamma_0 / s
void launch_gt_vectors(int n0, const double *V, const double *U, const double *gamma,
                       const double *s, double *fV, double *fU, hipStream_t st);
// surface term e = -W.W/2 + (V - W.t) gamma_0/(2s) - gamma_0^2/(8s^2) + tau theta_a/s - g y - F00
// with W.t = (tmv + sum of the nsq partials of Q gamma)/s and F00 = -H(fU)/2 + KS fV + GS fU
void launch_gt_surface(int n0, const Nodes &N, double tau, double grav, const double *V,
                       const double *U, const double *gamma, const double *tmv,
                       const double *pq, int nsq, const double *hfu, const double *kfv,
                       const double *gfu, double *e, hipStream_t st);
// energy density terms and the fixed-order mean (psi_k: nb-2 obstacle constants)
void launch_energy(int n0, const Nodes &N, const Flow &F, double tau, double grav,
                   const double *hw, const double *part, int nsplit, const double *dphi,
                   const double *tmv, const double *psi_k, double *e, double *E, hipStream_t st);
// op: WWBI_OP_D, WWBI_OP_H or kOpHalfCot, one row per boundary laid out like the nodes
void launch_circulant_rows(const Layout &L, int op, double *rows, hipStream_t st);
// Fourier-tail measure of f on every boundary (Sec. 7.1's resolution test):
// out[2k] = energy in the modes ceil(3 M_k / 8) .. M_k / 2 (both signs),
// out[2k+1] = total energy; modes holds tail_modes_total(L) doubles.
int tail_modes_total(const Layout &L);
void launch_tail_monitor(const Layout &L, const double *f, double *modes, double *out,
                         hipStream_t st);
// out = alpha C_k f + beta out on boundaries first..last (one launch);
// launch_circulant_apply2 scales boundary 0 by alpha0 and the others by alpha
void launch_circulant_apply(const Layout &L, const double *rows, const double *f, double *out,
                            double alpha, double beta, int first_block, int last_block,
                            hipStream_t st);
void launch_circulant_apply2(const Layout &L, const double *rows, const double *f, double *out,
                             double alpha0, double alpha, double beta, int first_block,
                             int last_block, hipStream_t st);
// the same for nv vectors at once: vector v reads f + v fs and writes out + v os
void launch_circulant_batched(const Layout &L, const double *rows, const double *f, long fs,
                              double *out, long os, int nv, double alpha0, double alpha,
                              double beta, int first_block, int last_block, hipStream_t st);
void launch_circ_row1(int M, int op, double *row, hipStream_t st);
void launch_circ_apply1(int M, const double *row, const double *f, double *out, double alpha,
                        double beta, hipStream_t st);
void launch_block_means(const Layout &L, const double *v, double *out, hipStream_t st);
void launch_U_finalize(int n0, const double *s, const double *umv, const double *hg,
                       const double *part, int nsplit, double *U, hipStream_t st);
void launch_wall_rhs_finalize(int nw, const double *umv_w, const double *part, int nsplit,
                              double *rhs, hipStream_t st);
void launch_surface_base(int n, const double *xt, const double *yt, double *x, double *y,
                         hipStream_t st);
void launch_add_scalar(int n, double *v, double c, hipStream_t st);

// ---- kernels_evolve.hip ------------------------------------------------------
constexpr int kMaxStages = 16;   // Runge-Kutta stages per step
struct RkCoef {
    int ns;
    double h;
    double c[kMaxStages];
};
// filter symbol (sigma, M/2) and the circulant rows of the zero-mean
// antiderivative and of the 36th-order filter on an M-point grid
void launch_evolve_rows(int M, double *sigma, double *rint, double *rfil, hipStream_t st);
void launch_graph_base(int M, const double *eta, double *x, double *y, double *dx, double *ddx,
                       hipStream_t st);
void launch_mean_cs(int M, const double *a, double *out, hipStream_t st);
void launch_mean_prod(int M, const double *a, const double *b, double *out, hipStream_t st);
void launch_hls_slope(int M, const double *Pt, const double *cs, double *dx, double *dy,
                      double *xm1, hipStream_t st);
void launch_hls_xy(int M, const double *xa, const double *ya, const double *mean_yx, double *x,
                   double *y, hipStream_t st);
void launch_hls_curv(int M, const double *ta, const double *dx, const double *dy, double *ddx,
                     double *ddy, hipStream_t st);
void launch_graph_rates(int M, const double *U, const double *dy, double *V, double *qt,
                        hipStream_t st);
void launch_mul(int M, const double *a, const double *b, double *out, hipStream_t st);
void launch_hls_V(int M, const double *Vi, const double *U, const double *dx, const double *dy,
                  double *V, hipStream_t st);
void launch_hls_f(int M, const double *dU, const double *V, const double *ta, const double *dx,
                  const double *dy, double *f, hipStream_t st);
void launch_sub_mean(int M, const double *f, const double *mean, double *out, hipStream_t st);
void launch_phit(int M, const Nodes &N, const Flow &F, const double *dphi, const double *U,
                 const double *V, double tau, double grav, double *out, hipStream_t st);
void launch_rk_combine(int M, const double *base, const double *K, long ld, const RkCoef &co,
                       double *out, hipStream_t st);

// ---- kernels_interior.hip ----------------------------------------------------
// Helsing-Ojala rule at P points from boundary values f (partial slices in
// part: 4 * ho_slices * P doubles; hit: ho_slices * P ints)
int ho_slices(int P, int n);
// out[0] = points with a non-finite coordinate, out[1] = finite points with
// |y| > kMaxAbsY (2 doubles, device)
void launch_check_points(int P, const double *zx, const double *zy, double *out,
                         hipStream_t st);
void launch_helsing_ojala(const Nodes &N, int n, int n0, int P, const double *zx,
                          const double *zy, const double *fr, const double *fi, double *part,
                          int *hit, bool neg_im, double *outr, double *outi, hipStream_t st);
void launch_boundary_velocity(int n, const double *dx, const double *dy, const double *sds,
                              const double *sdn, bool phi_prime, double *u, double *v,
                              hipStream_t st);
// s dphi/dn = s dphi_mv/dn + local + T gamma partials (local: H gamma_0/2 on
// the surface, -gamma_k/2 on wall k)
void launch_normal_finalize(int n, int n0, const double *umv, const double *gamma,
                            const double *hg, const double *part, int nsplit, double *out,
                            hipStream_t st);

void launch_pressure_data(int n0, const Nodes &N, const double *sds, const double *sdn,
                          double tau, double grav, double *b, hipStream_t st);
void launch_phi_aux_values(int n, int n0, const double *data, const double *ps,
                           const double *rw, const double *hw, const int *bid,
                           const double *means, double *fr, double *fi, hipStream_t st);
void launch_pressure_final(int P, const double *phit, const double *wr, const double *wi,
                           const double *zy, double grav, double *out, hipStream_t st);

// ---- kernels_matrix.hip ------------------------------------------------------
// `active` (device, may be null): when it points to 0 the product is skipped.
void launch_assemble64(const Layout &L, const Nodes &N, int flags, double *A, long ld,
                       hipStream_t st);
void launch_assemble32(const Layout &L, const Nodes &N, int flags, int band, float *A, long ld,
                       hipStream_t st);
// the transpose A^T in the same layout (row q = source q), for products with
// A^T by the forward stored matvec
void launch_assemble32_T(const Layout &L, const Nodes &N, int flags, int band, float *AT,
                         long ld, hipStream_t st);
void launch_assemble64_T(const Layout &L, const Nodes &N, int flags, double *AT, long ld,
                         hipStream_t st);
// operator of the gamma_t system (Sec. 4.2), n x n FP64
void launch_assemble_gt64(const Layout &L, const Nodes &N, double *B, long ld, hipStream_t st);
// the same entries, evaluated in FP64 and stored rounded to FP32 (refined solves)
void launch_assemble_gt32(const Layout &L, const Nodes &N, float *B, long ld, hipStream_t st);
void launch_assemble_wall64(const Layout &L, const Nodes &N, const double *hrow, double *W, long ld,
                            hipStream_t st);
// the same entries, evaluated in FP64 and stored rounded to FP32 (refined solves)
void launch_assemble_wall32(const Layout &L, const Nodes &N, const double *hrow, float *W, long ld,
                            hipStream_t st);
// the normal-velocity map T (surface rows, all columns), FP64
void launch_assemble_T64(const Layout &L, const Nodes &N, const double *hrow, double *T, long ld,
                         hipStream_t st);
// y = c - A x, or y = A x when c is null, accumulated in FP64 for either
// matrix type (FP32 entries and x widened one by one)
void launch_gemv64(const double *A, long ld, int n, const double *x, const double *c, double *y,
                   const int *active, hipStream_t st);
void launch_gemv32(const float *A, long ld, int n, const float *x, const double *c, double *y,
                   const int *active, hipStream_t st);
// Number of per-block partials of the fused Arnoldi product below.
int gemv_partials(int n);
// y = A x (FP32 matrix and x, FP64 accumulation) fused with the first
// Gram-Schmidt dots: P[i * gemv_partials(n) + b] (i <= j < 64) and the squared
// norm partials P3[b] of y, per block b, summed later in a fixed order.
void launch_gemv32_dots(const float *A, long ld, int n, const float *x, double *y,
                        const int *active, const double *V, long ldv, int j, double *P,
                        double *P3, hipStream_t st);
// the same for an FP64 matrix
void launch_gemv64_dots(const double *A, long ld, int n, const double *x, double *y,
                        const int *active, const double *V, long ldv, int j, double *P,
                        double *P3, hipStream_t st);
void launch_otf_matvec(const Layout &L, const Nodes &N, int flags, int fp32, int band,
                       int transpose, const double *x, const double *c, double *y, double *part,
                       const int *active, hipStream_t st);
// target-flavour products over rows [r0, r0+nr) and columns [c0, c0+nc):
// mode 2 = T (normal-velocity map / G^dagger), mode 3 = wall operator T - I/2,
// mode 4 = stream-function map P (surface rows), mode 5 = tangential map Q.
// Forward: part[s][r] over column chunks; transpose: part[s][c] over row chunks.
void launch_rflavour(const Layout &L, const Nodes &N, const double *hrow, int mode, int transpose,
                     int r0, int nr, int c0, int nc, const double *x, double *part,
                     const int *active, hipStream_t st);
// partial slices (far chunks + the near band) of a product over nr rows and
// nc columns, forward or transposed; at most 257, each of length nr
// (forward) or nc (transposed)
int rflavour_nsplit(const Nodes &N, int nr, int nc, int transpose);
void launch_reduce_partials(int n, const double *part, int nsplit, const double *c, double scale,
                            double *y, const int *active, hipStream_t st);
int otf_chunk(int n);
int otf_nsplit(int n);

// ---- kernels_adjoint.hip -----------------------------------------------------
int adjoint_nsplit(int n);
// Tangent-linear model of the velocity-potential solve (up to 32 directions
// at once; dirs 7 x nd x M_0): the source-moving parts of dA omega (pA, n per
// direction and slice) and of dT gamma (pT, M_0), from the weights W
// (tlm_weights_size(M_0) doubles), then the right-hand sides (rhs, ld ldb) and
// the surface terms of dU (um, nd x M_0).
int tlm_nsplit(int n, int n0);
size_t tlm_weights_size(int n0);
void launch_tlm_cols(const Nodes &N, int n0, int n, int nd, const double *dirs,
                     const double *omega, const double *gamma, double *W, double *pA, double *pT,
                     hipStream_t st);
void launch_tlm_rhs(const Nodes &N, const Flow &F, int n0, int n, int nd, const double *dirs,
                    const double *omega, const double *gamma, const double *U,
                    const double *prow, const double *pA, const double *pT, double *rhs, long ldb,
                    double *um, hipStream_t st);
void launch_tlm_finalize(int n0, int nd, const double *s, const double *um, const double *hg,
                         const double *tg, double *dU, hipStream_t st);
void launch_adj_c(int n0, const double *Ubar, const double *s, double *c, hipStream_t st);
void launch_adj_rows(const Nodes &N, const double *hrow, int n0, int n, const double *omega,
                     const double *gamma, double *part, hipStream_t st);
void launch_adj_cols(const Nodes &N, int n0, int n, const double *lam, const double *cvec,
                     double *part, hipStream_t st);
void launch_adj_finalize(const Nodes &N, const Flow &F, int n0, const double *Ubar,
                         const double *U, const double *omega, const double *gamma,
                         const double *lam, const double *prow, int nsr, const double *pcol,
                         int nsc, double *g_phi, double *g_x, double *g_y, double *g_dx,
                         double *g_dy, double *g_ddx, double *g_ddy, hipStream_t st);

// ---- kernels_multi.hip -------------------------------------------------------
// Y_s = c_s - A X_s (or A X_s when c is null) for s < nr on the matrix cores.
void launch_mfma_multi64(const double *A, long ld, int n, const double *X, long xs, int nr,
                         const double *c, long cs, double *y, long ys, double *part,
                         hipStream_t st);
void launch_mfma_multi32(const float *A, long ld, int n, const float *X, long xs, int nr,
                         const double *c, long cs, double *y, long ys, double *part,
                         hipStream_t st);
void launch_to_f32_batched(const double *src, long ss, float *dst, long ds, int n, int nr,
                           hipStream_t st);
void launch_copy_strided(const double *src, long ss, double *dst, long ds, int n, int nr,
                         hipStream_t st);
int multi_part_size(int n, int nr);
// the product alone: system s of slice k at part + (k * nr + s) * n, for the
// caller to sum in slice order; returns the slice count
int launch_mfma_parts64(const double *A, long ld, int n, const double *X, long xs, int nr,
                        double *part, hipStream_t st);
int launch_mfma_parts32(const float *A, long ld, int n, const float *X, long xs, int nr,
                        double *part, hipStream_t st);
// y_s = T X_s, s < nr, for an FP64 m x n matrix T (row stride ld, a multiple
// of 64 columns readable past n); part needs multi_part_size_rect64(m, n, nr).
void launch_mfma_rect64(const double *A, long ld, int m, int n, const double *X, long xs, int nr,
                        double *y, long ys, double *part, hipStream_t st);
int multi_part_size_rect64(int m, int n, int nr);

// ---- kernels_gmres.hip -------------------------------------------------------
int gmres_nblocks(int n);
void launch_norm_partial(const double *v, int n, double *P, int G, hipStream_t st,
                         const Bat &bt = kSingle);
void launch_set_tol(const double *P, int G, double tol, GState *gs, hipStream_t st,
                    const Bat &bt = kSingle);
// mirror (may be null): host-visible copy of the cycle state, written once
// per cycle, by the kernel that ends cycle `cyc` (the cycle start when there
// is nothing to do, else the Arnoldi step that converges or fills the basis)
void launch_cycle_start(const double *r, int n, const double *P, int G, double *V, float *v32,
                        double *g, int ldg, GState *gs, int cyc, GState *mirror, hipStream_t st,
                        const Bat &bt = kSingle);
// partial dots of w with V_0..V_j into P, partial |w|^2 into P3
// With part (ks slices of nr systems, as launch_mfma_parts* leave them), w is
// first written as their sum in slice order.
void launch_cgs_dot(const double *V, long ldv, double *w, int n, int j, double *P,
                    double *P3, int G, const GState *gs, hipStream_t st, const Bat &bt = kSingle,
                    const double *part = nullptr, int ks = 0, int nr = 0);
// first Gram-Schmidt pass (w -= V h; dots of V with w into P2, |w|^2 into P3)
// GP: the number of partials in P1 (0: G, the chunk count)
// hred (may be null): the coefficients already summed (launch_reduce_rows)
void launch_cgs_first(const double *V, long ldv, double *w, int n, int j, const double *P1,
                      double *P2, double *P3, int G, double *H, int ldh, const GState *gs,
                      hipStream_t st, const Bat &bt = kSingle, int GP = 0,
                      const double *hred = nullptr);
// out[r] = sum of row r of the GP per-block partials P (rows 0..nrows-1, the
// last one taken from Px when Px is given); nothing once the cycle has ended
void launch_reduce_rows(const double *P, int GP, const double *Px, int nrows, double *out,
                        const GState *gs, hipStream_t st);
// last pass fused with normalisation into V_{j+1} and the Givens step
// (add: column j of H already holds a first pass)
// GP: the number of partials in P2 and P3 (0: G, the chunk count)
// kc > 0: V points at kc recycled vectors in front of the Arnoldi basis, whose
// coefficients go to column j of B (ld ldb)
void launch_cgs_final(const double *V, long ldv, const double *w, int n, int j,
                      const double *P2, const double *P3, int G, float *v32, double *H, int ldh,
                      bool add, double *cs, double *sn, double *g, int restart_len, GState *gs,
                      int cyc, GState *mirror, hipStream_t st, const Bat &bt = kSingle,
                      int GP = 0, int kc = 0, double *B = nullptr, int ldb = 0,
                      const double *hred = nullptr);
// Recycling of an inner solve's Krylov space (k steps, basis V, rotated
// Hessenberg H, rotations cs/sn): C (k rows, orthonormal) and U with A U = C
void launch_recycle_build(const double *V, long ldv, int n, int k, const double *H, int ldh,
                          const double *cs, const double *sn, double *C, double *U,
                          hipStream_t st);
// partial dots of r with C_0..C_{kc-1} into P, partial |r|^2 into P3
void launch_recycle_dots(const double *C, long ldv, const double *r, int n, int kc, double *P,
                         double *P3, int G, hipStream_t st);
// z = C^T r, r0 = r - C z, partial |r0|^2 into P3
void launch_recycle_project(const double *C, long ldv, const double *r, int n, int kc,
                            const double *P, double *P3, int G, double *r0, double *z,
                            hipStream_t st);
// z -= B y over the solved columns
void launch_recycle_coef(double *z, const double *B, int ldb, const double *y, int kc,
                         const GState *gs, hipStream_t st);
// x = V y + U z
void launch_xupdate_recycled(double *x, const double *V, long ldv, int n, const double *y,
                             const double *U, const double *z, int kc, const GState *gs,
                             hipStream_t st);
void launch_hsolve(const double *H, int ldh, const double *g, double *y, const GState *gs,
                   hipStream_t st, const Bat &bt = kSingle);
// x += V y (x = V y when overwrite)
void launch_xupdate(double *x, const double *V, long ldv, int n, const double *y,
                    bool overwrite, const GState *gs, hipStream_t st, const Bat &bt = kSingle);
void launch_axpy(double *x, const double *d, int n, double alpha, hipStream_t st);
void launch_copy(double *dst, const double *src, int n, hipStream_t st);
void launch_fill(double *dst, double v, int n, hipStream_t st);
void launch_to_f32(const double *src, float *dst, int n, hipStream_t st);

}  // namespace wwbi
