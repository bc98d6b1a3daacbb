// Derivative contractions of the adjoint of the velocity-potential solve.
//
// Forward map (walls fixed, surface samples z, d = z', e = z'' free):
//   A(z, d, e) omega = b,  b_0 = phi~            (Sec. 3.2-3.3)
//   gamma = (-D omega_0, D omega_1, ...)
//   s U = u_mv(z, d) + H gamma_0 / 2 + T(z, d, e) gamma     (Sec. 3.4)
// With c = Ubar / s and lambda = A^{-T} omegabar, the geometric part of the
// gradient is
//   sum_m c_m [d u_mv + dT gamma]_m - sum_m c_m U_m ds_m - lambda^T dA omega.
// Every kernel entry that involves a surface node contributes through
//   d kappa / d Delta = -(1 + kappa^2)/2,  kappa = cot((z_q - z_p)/2),
// so dS/dz_q = -d_q (1 + kappa^2)/4 = -dS/dz_p, dS/dd_q = kappa/2 for the
// source flavour and dR/dz_q = d_p (1 + kappa^2)/4 = -dR/dz_p, dR/dd_p =
// -kappa/2 for the target flavour.
#include "entries.h"
#include "internal.h"

namespace wwbi {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
constexpr int kStage = 256;
constexpr int kTlmMax = 32;      // directions of one tangent-linear launch
constexpr int kTlmWaves = 4608;  // waves the column pass's source split aims at

struct Cx {
    double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cx ctimes_i(Cx a) { return {-a.im, a.re}; }
__device__ __forceinline__ Cx cscale(Cx a, double s) { return {a.re * s, a.im * s}; }

// Row pass: targets r on the surface, all sources q != r.
//   out[0] = sum_q omega_q dA_rq/dx_r        out[1] = ... /dy_r
//   out[2] = sum_q gamma_q dT_rq/dx_r        out[3] = ... /dy_r
//   out[4] = sum_q gamma_q dT_rq/ddx_r       out[5] = ... /ddy_r
__device__ __forceinline__ void row_terms(const Tgt &t, const Src &s, double cr, double ci,
                                          double wq, double gq, double (&a)[6]) {
    const Cx kap{cr, ci};
    const Cx Q{1.0 + cr * cr - ci * ci, 2.0 * cr * ci};
    // source flavour, target derivative: dS/dz_r = +d_q Q / 4
    const Cx dS = cscale(cmul({s.dx, s.dy}, Q), 0.25 * s.w * wq);
    const Cx dSy = ctimes_i(dS);
    if (s.k == 0) { a[0] += dS.im; a[1] += dSy.im; }   // Im block (surface row, surface col)
    else { a[0] += dS.re; a[1] += dSy.re; }            // Re block (surface row, wall col)
    // target flavour: dR/dz_r = -d_r Q / 4, dR/dd_r = -kappa / 2
    const double gw = s.w * gq;
    const Cx dR = cscale(cmul({t.dx, t.dy}, Q), -0.25 * gw);
    const Cx dRy = ctimes_i(dR);
    const Cx dD = cscale(kap, -0.5 * gw);
    const Cx dDy = ctimes_i(dD);
    if (s.k == 0) { a[2] += dR.re; a[3] += dRy.re; a[4] += dD.re; a[5] += dDy.re; }
    else { a[2] += dR.im; a[3] += dRy.im; a[4] += dD.im; a[5] += dDy.im; }
}

// Column pass: sources r on the surface, all targets p != r.
//   out[0..3] = sum_p lambda_p dA_pr/d(x_r, y_r, dx_r, dy_r)
//   out[4..5] = sum_{p on surface} c_p dT_pr/d(x_r, y_r)
__device__ __forceinline__ void col_terms(const Tgt &t, const Src &s, double cr, double ci,
                                          double lp, double cp, double (&a)[6]) {
    const Cx kap{cr, ci};
    const Cx Q{1.0 + cr * cr - ci * ci, 2.0 * cr * ci};
    // source flavour, source derivative: dS/dz_r = -d_r Q / 4, dS/dd_r = kappa / 2
    const double lw = s.w * lp;
    const Cx dS = cscale(cmul({s.dx, s.dy}, Q), -0.25 * lw);
    const Cx dSy = ctimes_i(dS);
    const Cx dK = cscale(kap, 0.5 * lw);
    const Cx dKy = ctimes_i(dK);
    if (t.k == 0) {   // surface row: Im S
        a[0] += dS.im; a[1] += dSy.im; a[2] += dK.im; a[3] += dKy.im;
        // target flavour, source derivative: dR/dz_r = d_p Q / 4 (surface source: Re)
        const Cx dR = cscale(cmul({t.dx, t.dy}, Q), 0.25 * s.w * cp);
        a[4] += dR.re;
        a[5] += ctimes_i(dR).re;
    } else {          // wall row: -Re S
        a[0] -= dS.re; a[1] -= dSy.re; a[2] -= dK.re; a[3] -= dKy.re;
    }
}

__device__ __forceinline__ void store6(double *part, long st, long off, const double (&a)[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) part[k * st + off] = a[k];
}

// Far part of both passes: every pair except the surface pairs within nb
// grid steps of r (diagonal included), with kappa from E alone.  Chunk
// blockIdx.y of the other index, written as slice blockIdx.y of `part`
// (component stride st).  A staged tile that holds no near-band pair for the
// wave skips the per-pair test (CHECK = false).
template <bool CHECK>
__device__ __forceinline__ void adj_rows_tile(const Tgt &t, const Src *ss, const double *sw,
                                              const double *sg, int m, int nb, double (&a)[6]) {
    for (int i = 0; i < m; ++i) {
        const Src &s = ss[i];
        if (CHECK && in_band(t, s, nb)) continue;
        double cr, ci;
        kappa64_far(t, s, cr, ci);
        row_terms(t, s, cr, ci, sw[i], sg[i], a);
    }
}

template <bool CHECK>
__device__ __forceinline__ void adj_cols_tile(const Src &s, const Tgt *ts, const double *sl,
                                              const double *sc, int m, int nb, double (&a)[6]) {
    for (int i = 0; i < m; ++i) {
        const Tgt &t = ts[i];
        if (CHECK && in_band(t, s, nb)) continue;
        double cr, ci;
        kappa64_far(t, s, cr, ci);
        col_terms(t, s, cr, ci, sl[i], sc[i], a);
    }
}

__global__ __launch_bounds__(256) void k_adj_rows(Nodes N, int n0, int n, int chunk, int nb,
                                                  const double *__restrict__ omega,
                                                  const double *__restrict__ gamma,
                                                  double *__restrict__ part, long st) {
    __shared__ Src ss[kStage];
    __shared__ double sw[kStage], sg[kStage];
    const int wb = wave_base();
    const int r = blockIdx.x * 256 + threadIdx.x;
    const bool live = r < n0;
    Tgt t;
    if (live) t = load_tgt(N, r);
    const int qb = blockIdx.y * chunk, qe = min(n, qb + chunk);
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int qq = qb; qq < qe; qq += kStage) {
        const int q = qq + threadIdx.x;
        if (q < qe) {
            ss[threadIdx.x] = load_src(N, q);
            sw[threadIdx.x] = omega[q];
            sg[threadIdx.x] = gamma[q];
        }
        __syncthreads();
        const int m = min(kStage, qe - qq);
        const bool apart = wave_apart<false>(N, 0, blockIdx.x * 256 + wb, n0, qq, m, nb);
        if (live) {
            if (apart)
                adj_rows_tile<false>(t, ss, sw, sg, m, nb, a);
            else
                adj_rows_tile<true>(t, ss, sw, sg, m, nb, a);
        }
        __syncthreads();
    }
    if (live) store6(part, st, (long)blockIdx.y * n0 + r, a);
}

__global__ __launch_bounds__(256) void k_adj_cols(Nodes N, int n0, int n, int chunk, int nb,
                                                  const double *__restrict__ lam,
                                                  const double *__restrict__ cvec,
                                                  double *__restrict__ part, long st) {
    __shared__ Tgt ts[kStage];
    __shared__ double sl[kStage], sc[kStage];
    const int wb = wave_base();
    const int r = blockIdx.x * 256 + threadIdx.x;
    const bool live = r < n0;
    Src s;
    if (live) s = load_src(N, r);
    const int pb = blockIdx.y * chunk, pe = min(n, pb + chunk);
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int pp = pb; pp < pe; pp += kStage) {
        const int p = pp + threadIdx.x;
        if (p < pe) {
            ts[threadIdx.x] = load_tgt(N, p);
            sl[threadIdx.x] = lam[p];
            sc[threadIdx.x] = p < n0 ? cvec[p] : 0.0;
        }
        __syncthreads();
        const int m = min(kStage, pe - pp);
        const bool apart = wave_apart<true>(N, 0, blockIdx.x * 256 + wb, n0, pp, m, nb);
        if (live) {
            if (apart)
                adj_cols_tile<false>(s, ts, sl, sc, m, nb, a);
            else
                adj_cols_tile<true>(s, ts, sl, sc, m, nb, a);
        }
        __syncthreads();
    }
    if (live) store6(part, st, (long)blockIdx.y * n0 + r, a);
}

// Near part of both passes: the surface partners of r within nb grid steps
// (the whole surface when it has at most 2 nb + 1 nodes), diagonal excluded,
// with the exact-difference kappa; written as slice `slice`.
template <bool COLS>
__global__ __launch_bounds__(256) void k_adj_near(Nodes N, int n0, int nb,
                                                  const double *__restrict__ v1,
                                                  const double *__restrict__ v2,
                                                  double *__restrict__ part, long st, int slice) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n0) return;
    const bool whole = 2 * nb + 1 >= n0;
    const int d0 = whole ? -r : -nb, d1 = whole ? n0 - 1 - r : nb;
    double a[6] = {0, 0, 0, 0, 0, 0};
    const Tgt tr = load_tgt(N, r);
    const Src sr = load_src(N, r);
    for (int d = d0; d <= d1; ++d) {
        if (d == 0) continue;
        int l = r + d;
        if (l < 0) l += n0;
        if (l >= n0) l -= n0;
        double cr, ci;
        if (!COLS) {
            const Src s = load_src(N, l);
            kappa64(N, tr, s, cr, ci);
            row_terms(tr, s, cr, ci, v1[l], v2[l], a);
        } else {
            const Tgt t = load_tgt(N, l);
            kappa64(N, t, sr, cr, ci);
            col_terms(t, sr, cr, ci, v1[l], v2[l], a);
        }
    }
    store6(part, st, (long)slice * n0 + r, a);
}

// Derivatives of u_mv = -(V1 + sum a / 2) y' + sum_j a_j Re{cot((z - z_j)/2) z' / 2}
// with respect to x, y, x', y' of one surface node.
__device__ __forceinline__ void umv_derivs(const Flow &F, double x, double y, double dx, double dy,
                                           double &ux, double &uy, double &udx, double &udy) {
    double asum = 0.0;
    for (int j = 0; j < F.nobs; ++j) asum += F.a[j];
    ux = 0.0;
    uy = 0.0;
    udx = 0.0;
    udy = -(F.V1 + 0.5 * asum);
    for (int j = 0; j < F.nobs; ++j) {
        double cr, ci;
        cot_half64(x - F.zx[j], y - F.zy[j], cr, ci);
        const Cx kap{cr, ci};
        const Cx Q{1.0 + cr * cr - ci * ci, 2.0 * cr * ci};
        const Cx dz = cscale(cmul({dx, dy}, Q), -0.25 * F.a[j]);   // d/dz of a kappa z'/2
        ux += dz.re;
        uy += ctimes_i(dz).re;
        udx += 0.5 * F.a[j] * kap.re;
        udy += 0.5 * F.a[j] * ctimes_i(kap).re;
    }
}

// The diagonal limit L = e / (2 d) (d = z', e = z'') of a surface node and its
// complex derivatives dL/dd = -L / d and dL/de = 1 / (2 d); A_rr = -1/2 + w Im L
// and T_rr = w Re L.
__device__ __forceinline__ void diag_limit_derivs(double dx, double dy, double ex, double ey,
                                                  Cx &dLdd, Cx &dLde) {
    const double d2 = dx * dx + dy * dy;
    const Cx inv_d{dx / d2, -dy / d2};                 // 1/d
    const Cx L{(ex * dx + ey * dy) / (2.0 * d2), (ey * dx - ex * dy) / (2.0 * d2)};
    dLdd = cscale(cmul(L, inv_d), -1.0);
    dLde = cscale(inv_d, 0.5);
}

// Combine every term on the surface nodes.
__global__ void k_adj_finalize(Nodes N, Flow F, int n0, const double *__restrict__ Ubar,
                               const double *__restrict__ U, const double *__restrict__ omega,
                               const double *__restrict__ gamma, const double *__restrict__ lam,
                               const double *__restrict__ prow, int nsr,
                               const double *__restrict__ pcol, int nsc, double *g_phi,
                               double *g_x, double *g_y, double *g_dx, double *g_dy, double *g_ddx,
                               double *g_ddy) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n0) return;
    double R[6] = {0, 0, 0, 0, 0, 0}, Cc[6] = {0, 0, 0, 0, 0, 0};
    const long sr = (long)nsr * n0, sc = (long)nsc * n0;
    for (int k = 0; k < 6; ++k) {
        for (int b = 0; b < nsr; ++b) R[k] += prow[k * sr + (long)b * n0 + r];
        for (int b = 0; b < nsc; ++b) Cc[k] += pcol[k * sc + (long)b * n0 + r];
    }
    const double x = N.x[r], y = N.y[r], dx = N.dx[r], dy = N.dy[r];
    const double ex = N.ddx[r], ey = N.ddy[r];
    const double s = N.s[r], w = N.w[r];
    const double c = Ubar[r] / s;
    const double lr = lam[r], wr = omega[r], gr = gamma[r];
    double ux, uy, udx, udy;
    umv_derivs(F, x, y, dx, dy, ux, uy, udx, udy);
    // diagonal limits L = e/(2d): A_rr = -1/2 + w Im L, T_rr = w Re L
    Cx dLdd, dLde;
    diag_limit_derivs(dx, dy, ex, ey, dLdd, dLde);
    const Cx dLdd_y = ctimes_i(dLdd);
    const Cx dLde_y = ctimes_i(dLde);
    const double la = -lr * wr * w, tc = c * gr * w;   // weights of Im (A) and Re (T) parts
    g_phi[r] = lr;
    g_x[r] = c * ux + c * R[2] + gr * Cc[4] - lr * R[0] - wr * Cc[0];
    g_y[r] = c * uy + c * R[3] + gr * Cc[5] - lr * R[1] - wr * Cc[1];
    g_dx[r] = c * udx - c * U[r] * dx / s + c * R[4] - wr * Cc[2] + la * dLdd.im + tc * dLdd.re;
    g_dy[r] = c * udy - c * U[r] * dy / s + c * R[5] - wr * Cc[3] + la * dLdd_y.im + tc * dLdd_y.re;
    g_ddx[r] = la * dLde.im + tc * dLde.re;
    g_ddy[r] = la * dLde_y.im + tc * dLde_y.re;
}

// ---------------------------------------------------------------------------
// Tangent-linear model (forward mode) of the same chain, for up to kTlmMax
// directions at once.  A direction moves the surface's node data (x, y, x',
// y', x'', y'') and phi~; dirs holds 7 x nd x M_0 values, component c of
// direction i at (c * nd + i) * M_0.  With d omega = A^{-1} (d phi~ e_0 -
// dA omega) and dU = (d u_mv + dT gamma + T d gamma + H d gamma_0 / 2 - U ds) / s,
// the terms of dA omega and dT gamma that move with the target node are the
// adjoint's row sums (k_adj_rows) times the direction at that node; the terms
// that move with the source node come from k_tlm_cols (matrix cores).
// ---------------------------------------------------------------------------

// Weights of the column part: W[(q * 6 + c) * kTlmMax + i] is direction i's
// change of source q's x, y, x', y' times omega_q (c = 0..3) and of its x, y
// times gamma_q (c = 4, 5); zero for i >= nd.
__global__ void k_tlm_weights(int n0, int nd, const double *__restrict__ dirs,
                              const double *__restrict__ omega, const double *__restrict__ gamma,
                              double *__restrict__ W) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n0 * 6 * kTlmMax) return;
    const int i = (int)(e % kTlmMax), c = (int)((e / kTlmMax) % 6), q = (int)(e / (6 * kTlmMax));
    double v = 0.0;
    if (i < nd) {
        const int cc = c < 4 ? c : c - 4;
        v = dirs[((long)cc * nd + i) * n0 + q] * (c < 4 ? omega[q] : gamma[q]);
    }
    W[e] = v;
}

// Column part on the matrix cores: for targets p and directions i,
//   colA_i[p] = sum_{q != p on the surface} sum_c dA_pq/dc_q W_c(q, i)   (c = x, y, x', y')
//   colT_i[p] = sum_{q != p on the surface} sum_c dT_pq/dc_q W_{4+c}(q, i) (c = x, y; p on the surface)
// a contraction over (q, c) of the derivative coefficients with the weights.
// A wave owns 16 targets and all directions (two 16-wide tiles when nd > 16)
// over one chunk of sources (blockIdx.y), 4 sources per step: lane l takes
// the pair (p0 + l % 16, q0 + l / 16), which is exactly the A operand it
// supplies to v_mfma_f64_16x16x4f64 (row l % 16, k slot l / 16), forms kappa
// once (kappa64: near pairs from the exact difference) and one coefficient
// per component c, and the B operand is W_c(q0 + l / 16, 16 t + l % 16).
// With S = (w/2) z'_q kappa and R = -(1/2) z'_p kappa:
//   dS/dz_q = -(w/4) z'_q (1 + kappa^2), dS/dz'_q = (w/2) kappa (surface rows
//   take Im S, wall rows -Re S), dR/dz_q = (w/4) z'_p (1 + kappa^2) (Re R).
// Result element r of lane l is target p0 + l / 16 + 4 r, direction l % 16.
__global__ __launch_bounds__(256) void k_tlm_cols(Nodes N, int n0, int n, int nd, int chunk,
                                                  const double *__restrict__ W,
                                                  double *__restrict__ pA,
                                                  double *__restrict__ pT) {
    typedef double v4d __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int p0 = (blockIdx.x * 4 + wv) * 16;
    if (p0 >= n) return;                        // whole waves; no barriers below
    const int il = lane & 15, kq = lane >> 4;
    const int p = p0 + il;
    const bool live = p < n;
    const Tgt t = load_tgt(N, live ? p : n - 1);
    const bool surf = t.k == 0;
    const bool tpart = p0 < n0;                 // the tile holds surface targets
    const bool two = nd > 16;
    const int qb = blockIdx.y * chunk, qe = min(n0, qb + chunk);
    v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0, t0 = a0, t1 = a0;
    // the step's source and weights, loaded one step ahead
    auto weights = [&](int qc, double (&wo)[12]) __attribute__((always_inline)) {
        const double *w = W + (long)qc * 6 * kTlmMax + il;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            wo[2 * c] = w[c * kTlmMax];
            wo[2 * c + 1] = w[c * kTlmMax + 16];
        }
    };
    Src s = load_src(N, min(qb + kq, n0 - 1));
    double wc[12];
    weights(min(qb + kq, n0 - 1), wc);
    for (int qs = qb; qs < qe; qs += 4) {
        const int q = qs + kq;
        const int qn = min(qs + 4 + kq, n0 - 1);
        const Src sn = load_src(N, qn);
        double wn[12];
        weights(qn, wn);
        double ca[4] = {0.0, 0.0, 0.0, 0.0}, ct[2] = {0.0, 0.0};
        if (live && q < qe && q != p) {
            double cr, ci;
            kappa64(N, t, s, cr, ci);
            const Cx Q{1.0 + cr * cr - ci * ci, 2.0 * cr * ci};
            const Cx dz = cscale(cmul({s.dx, s.dy}, Q), -0.25 * s.w);
            const Cx dd = cscale({cr, ci}, 0.5 * s.w);
            if (surf) {
                ca[0] = dz.im; ca[1] = dz.re; ca[2] = dd.im; ca[3] = dd.re;
                const Cx dr = cscale(cmul({t.dx, t.dy}, Q), 0.25 * s.w);
                ct[0] = dr.re; ct[1] = -dr.im;
            } else {
                ca[0] = -dz.re; ca[1] = dz.im; ca[2] = -dd.re; ca[3] = dd.im;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[c], wc[2 * c], a0, 0, 0, 0);
            if (two) a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[c], wc[2 * c + 1], a1, 0, 0, 0);
        }
        if (tpart) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                t0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ct[c], wc[8 + 2 * c], t0, 0, 0, 0);
                if (two)
                    t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ct[c], wc[9 + 2 * c], t1, 0, 0, 0);
            }
        }
        s = sn;
#pragma unroll
        for (int e = 0; e < 12; ++e) wc[e] = wn[e];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = p0 + kq + 4 * r;
        const long sa = (long)blockIdx.y * nd;
        if (row < n) {
            if (il < nd) pA[(sa + il) * n + row] = a0[r];
            if (two && il + 16 < nd) pA[(sa + il + 16) * n + row] = a1[r];
        }
        if (tpart && row < n0) {
            if (il < nd) pT[(sa + il) * n0 + row] = t0[r];
            if (two && il + 16 < nd) pT[(sa + il + 16) * n0 + row] = t1[r];
        }
    }
}

// Right-hand sides of the nd tangent systems (rhs, system i at i * ldb) and
// the surface terms of dU (um, direction i at i * n0):
//   rhs_i = [p on the surface] (dphi~_i - row terms of dA omega) - colA_i,
//   um_i = d u_mv + row terms of dT gamma + colT_i - U ds,
// the row terms being the adjoint's row sums times the direction at the node
// plus the diagonal limits' derivatives.
__global__ void k_tlm_rhs(Nodes N, Flow F, int n0, int n, int nd, const double *__restrict__ dirs,
                          const double *__restrict__ omega, const double *__restrict__ gamma,
                          const double *__restrict__ U, const double *__restrict__ prow, int nsr,
                          const double *__restrict__ pA, const double *__restrict__ pT, int nsc,
                          double *rhs, long ldb, double *um) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (r >= n) return;
    double colA = 0.0;
    for (int b = 0; b < nsc; ++b) colA += pA[((long)b * nd + i) * n + r];
    if (r >= n0) {
        rhs[i * ldb + r] = -colA;
        return;
    }
    double R[6] = {0, 0, 0, 0, 0, 0};
    const long sr = (long)nsr * n0;
    for (int k = 0; k < 6; ++k)
        for (int b = 0; b < nsr; ++b) R[k] += prow[k * sr + (long)b * n0 + r];
    double colT = 0.0;
    for (int b = 0; b < nsc; ++b) colT += pT[((long)b * nd + i) * n0 + r];
    double d[7];
    for (int c = 0; c < 7; ++c) d[c] = dirs[((long)c * nd + i) * n0 + r];
    const double x = N.x[r], y = N.y[r], dx = N.dx[r], dy = N.dy[r];
    const double s = N.s[r], w = N.w[r];
    Cx dLdd, dLde;
    diag_limit_derivs(dx, dy, N.ddx[r], N.ddy[r], dLdd, dLde);
    const Cx a = cmul(dLdd, {d[2], d[3]}), b2 = cmul(dLde, {d[4], d[5]});
    const Cx dL{a.re + b2.re, a.im + b2.im};
    double ux, uy, udx, udy;
    umv_derivs(F, x, y, dx, dy, ux, uy, udx, udy);
    const double dArow = R[0] * d[0] + R[1] * d[1] + w * omega[r] * dL.im;
    rhs[i * ldb + r] = d[6] - dArow - colA;
    const double dumv = ux * d[0] + uy * d[1] + udx * d[2] + udy * d[3];
    const double dTrow = R[2] * d[0] + R[3] * d[1] + R[4] * d[2] + R[5] * d[3] + w * gamma[r] * dL.re;
    const double ds = (dx * d[2] + dy * d[3]) / s;
    um[(long)i * n0 + r] = dumv + dTrow + colT - U[r] * ds;
}

// dU_i = (um_i + H d gamma_0,i / 2 + T d gamma_i) / s for every direction
// (blockIdx.y), all three terms at stride n0.
__global__ void k_tlm_finalize(int n0, const double *__restrict__ s, const double *__restrict__ um,
                               const double *__restrict__ hg, const double *__restrict__ tg,
                               double *__restrict__ dU) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n0) return;
    const long o = (long)blockIdx.y * n0 + r;
    dU[o] = (um[o] + 0.5 * hg[o] + tg[o]) / s[r];
}

// c = Ubar / s on the surface
__global__ void k_adj_c(int n0, const double *Ubar, const double *s, double *c) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n0) c[r] = Ubar[r] / s[r];
}

}  // namespace

// partial slices per component: far chunks plus the near slice
int adjoint_nsplit(int n) { return cdiv(n, otf_chunk(n)) + 1; }

// slices of the tangent-linear column pass over the M_0 surface sources:
// about kTlmWaves waves for n targets in tiles of 16, chunks of a multiple of
// 4 sources
static int tlm_chunk(int n, int n0) {
    const int ks = std::max(1, std::min(16, cdiv(kTlmWaves, cdiv(n, 16))));
    return cdiv(cdiv(n0, ks), 4) * 4;
}
int tlm_nsplit(int n, int n0) { return cdiv(n0, tlm_chunk(n, n0)); }
size_t tlm_weights_size(int n0) { return (size_t)n0 * 6 * kTlmMax; }

void launch_tlm_cols(const Nodes &N, int n0, int n, int nd, const double *dirs,
                     const double *omega, const double *gamma, double *W, double *pA, double *pT,
                     hipStream_t st) {
    const long nw = (long)tlm_weights_size(n0);
    hipLaunchKernelGGL(k_tlm_weights, dim3(cdiv(nw, 256)), dim3(256), 0, st, n0, nd, dirs, omega,
                       gamma, W);
    const int chunk = tlm_chunk(n, n0);
    hipLaunchKernelGGL(k_tlm_cols, dim3(cdiv(n, 64), cdiv(n0, chunk)), dim3(256), 0, st, N, n0, n,
                       nd, chunk, W, pA, pT);
}

void launch_tlm_rhs(const Nodes &N, const Flow &F, int n0, int n, int nd, const double *dirs,
                    const double *omega, const double *gamma, const double *U,
                    const double *prow, const double *pA, const double *pT, double *rhs, long ldb,
                    double *um, hipStream_t st) {
    hipLaunchKernelGGL(k_tlm_rhs, dim3(cdiv(n, 256), nd), dim3(256), 0, st, N, F, n0, n, nd, dirs,
                       omega, gamma, U, prow, adjoint_nsplit(n), pA, pT, tlm_nsplit(n, n0), rhs, ldb,
                       um);
}

void launch_tlm_finalize(int n0, int nd, const double *s, const double *um, const double *hg,
                         const double *tg, double *dU, hipStream_t st) {
    hipLaunchKernelGGL(k_tlm_finalize, dim3(cdiv(n0, 256), nd), dim3(256), 0, st, n0, s, um, hg,
                       tg, dU);
}

void launch_adj_c(int n0, const double *Ubar, const double *s, double *c, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_c, dim3(cdiv(n0, 256)), dim3(256), 0, st, n0, Ubar, s, c);
}

void launch_adj_rows(const Nodes &N, const double *hrow, int n0, int n, const double *omega,
                     const double *gamma, double *part, hipStream_t st) {
    (void)hrow;
    const int chunk = otf_chunk(n);
    const int ns = cdiv(n, chunk);
    const long cs = (long)(ns + 1) * n0;
    hipLaunchKernelGGL(k_adj_rows, dim3(cdiv(n0, 256), ns), dim3(256), 0, st, N, n0, n, chunk,
                       kNearBand, omega, gamma, part, cs);
    hipLaunchKernelGGL((k_adj_near<false>), dim3(cdiv(n0, 256)), dim3(256), 0, st, N, n0,
                       kNearBand, omega, gamma, part, cs, ns);
}

void launch_adj_cols(const Nodes &N, int n0, int n, const double *lam, const double *cvec,
                     double *part, hipStream_t st) {
    const int chunk = otf_chunk(n);
    const int ns = cdiv(n, chunk);
    const long cs = (long)(ns + 1) * n0;
    hipLaunchKernelGGL(k_adj_cols, dim3(cdiv(n0, 256), ns), dim3(256), 0, st, N, n0, n, chunk,
                       kNearBand, lam, cvec, part, cs);
    hipLaunchKernelGGL((k_adj_near<true>), dim3(cdiv(n0, 256)), dim3(256), 0, st, N, n0,
                       kNearBand, lam, cvec, part, cs, ns);
}

void launch_adj_finalize(const Nodes &N, const Flow &F, int n0, const double *Ubar,
                         const double *U, const double *omega, const double *gamma,
                         const double *lam, const double *prow, int nsr, const double *pcol,
                         int nsc, double *g_phi, double *g_x, double *g_y, double *g_dx,
                         double *g_dy, double *g_ddx, double *g_ddy, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_finalize, dim3(cdiv(n0, 256)), dim3(256), 0, st, N, F, n0, Ubar, U,
                       omega, gamma, lam, prow, nsr, pcol, nsc, g_phi, g_x, g_y, g_dx, g_dy,
                       g_ddx, g_ddy);
}

}  // namespace wwbi
