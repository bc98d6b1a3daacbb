// Node preparation, validation, right-hand side, multi-valued terms, spectral
// circulants and the final assembly of the normal velocity.
#include <algorithm>

#include "ddmath.h"
#include "entries.h"
#include "internal.h"

namespace wwbi {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ int find_block(const Layout &L, int p) {
    int k = 0;
    while (k + 1 < L.nb && p >= L.off[k + 1]) ++k;
    return k;
}

// Per-node data derived once per call: boundary index, local index, M_k,
// weight 1/M_k, s = |zeta'| and the self limit zeta''/(2 zeta').
__global__ void k_prep_nodes(Layout L, const double *x, const double *y, const double *dx,
                             const double *dy, const double *ddx, const double *ddy, int *bid,
                             int *loc, int *Mk, double *w, double *s, double *lre, double *lim,
                             double *eR, double *eI, double *eRl, double *eIl) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= L.n) return;
    const int k = find_block(L, p);
    const int M = L.off[k + 1] - L.off[k];
    bid[p] = k;
    loc[p] = p - L.off[k];
    Mk[p] = M;
    w[p] = 1.0 / (double)M;
    const double a = dx[p], b = dy[p], ex = ddx[p], ey = ddy[p];
    const double d2 = a * a + b * b;
    s[p] = sqrt(d2);
    // zeta''/(2 zeta') = (ex + i ey)(a - i b) / (2 |zeta'|^2)
    lre[p] = (ex * a + ey * b) / (2.0 * d2);
    lim[p] = (ey * a - ex * b) / (2.0 * d2);
    // E = e^{i zeta} = e^{-y} (cos x + i sin x) as a double-double, so that
    // differences of E between nodes keep their relative accuracy
    DD er, ei;
    dd_expi(x[p], y[p], er, ei);
    eR[p] = er.hi;
    eI[p] = ei.hi;
    eRl[p] = er.lo;
    eIl[p] = ei.lo;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    return t;
}

// One block per boundary: count of non-finite samples, signed area
// (1/2) sum (x y' - y x') 2pi/M (negative = clockwise) and the mean of x'.
// Block nb checks the potential.
__global__ __launch_bounds__(1024) void k_validate(Layout L, Nodes N, const double *phi,
                                                  int nphi, int pb, double *out) {
    __shared__ double sh[16];
    const int k = blockIdx.x;
    if (k >= L.nb) {
        // the data array: block b of pb counts its share (grid-stride) into
        // out[4 nb + 2 + b], for the host to add
        const int b = k - L.nb;
        double bad = 0.0;
        for (long i = (long)b * blockDim.x + threadIdx.x; i < nphi; i += (long)pb * blockDim.x)
            bad += isfinite(phi[i]) ? 0.0 : 1.0;
        bad = block_sum(bad, sh);
        if (threadIdx.x == 0) {
            out[4 * L.nb + 2 + b] = bad;
            if (b == 0) out[4 * L.nb + 1] = 0.0;   // the near-pair count, added next
        }
        return;
    }
    const int p0 = L.off[k], p1 = L.off[k + 1];
    const double M = (double)(p1 - p0);
    double bad = 0.0, area = 0.0, mdx = 0.0, far = 0.0;
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const double v[6] = {N.x[p], N.y[p], N.dx[p], N.dy[p], N.ddx[p], N.ddy[p]};
        bool fin = true;
        for (int i = 0; i < 6; ++i) fin = fin && isfinite(v[i]);
        bad += fin ? 0.0 : 1.0;
        far += fabs(v[1]) > kMaxAbsY ? 1.0 : 0.0;
        area += 0.5 * (v[0] * v[3] - v[1] * v[2]) * (2.0 * M_PI / M);
        mdx += v[2] / M;
    }
    bad = block_sum(bad, sh);
    area = block_sum(area, sh);
    mdx = block_sum(mdx, sh);
    far = block_sum(far, sh);
    if (threadIdx.x == 0) {
        out[4 * k + 0] = bad;
        out[4 * k + 1] = area;
        out[4 * k + 2] = mdx;
        out[4 * k + 3] = far;
    }
}

// ln|1 - e^{i w}| with |1 - e^{iw}|^2 = expm1(-v)^2 + 4 e^{-v} sin^2(u/2)
__device__ __forceinline__ double log_abs_1m_eiw(double u, double v) {
    const double em = expm1(-v);
    const double su = sin(0.5 * u);
    return 0.5 * log(em * em + 4.0 * (em + 1.0) * su * su);
}

// psi_mv(z) = V1 Im z - sum_j a_j ln|1 - e^{i(z - z_j)}|   (Sec. 3, 3.1)
__device__ __forceinline__ double psi_mv(const Flow &F, double x, double y) {
    double v = F.V1 * y;
    for (int j = 0; j < F.nobs; ++j) v -= F.a[j] * log_abs_1m_eiw(x - F.zx[j], y - F.zy[j]);
    return v;
}

// b_0 = phi~ on the surface, b_k = psi_wall - psi_mv(zeta_k) on the walls (Sec. 3.2).
__global__ void k_rhs_phi(Layout L, Nodes N, Flow F, const double *phi, const double *psi_wall,
                          double *b) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= L.n) return;
    if (p < L.off[1]) {
        b[p] = phi[p];
        return;
    }
    const double g = psi_wall ? psi_wall[p - L.off[1]] : 0.0;
    b[p] = g - psi_mv(F, N.x[p], N.y[p]);
}

// s dphi_mv/dn = -(V1 + sum a_j / 2) y' + sum_j a_j Re{(1/2) cot((z - z_j)/2) z'}  (Sec. 3.4)
__global__ void k_umv(Nodes N, Flow F, int first, int count, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int p = first + i;
    const double dx = N.dx[p], dy = N.dy[p];
    double asum = 0.0;
    for (int j = 0; j < F.nobs; ++j) asum += F.a[j];
    double v = -(F.V1 + 0.5 * asum) * dy;
    for (int j = 0; j < F.nobs; ++j) {
        double cr, ci;
        cot_half64(N.x[p] - F.zx[j], N.y[p] - F.zy[j], cr, ci);
        v += F.a[j] * 0.5 * (cr * dx - ci * dy);
    }
    out[i] = v;
}

// Circulant rows on each boundary's grid (Sec. 3.4 symbols, Nyquist zeroed):
//   D: c(n) = (1/2)(-1)^n cot(pi n / M), c(0) = 0
//   H: c(n) = (2/M) cot(pi n / M) for odd n, 0 for even n
//   h (the Hilbert regulariser of the kernels): c(n) = (1/2) cot(pi n / M)
__global__ void k_circ_rows(Layout L, int op, double *rows) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= L.n) return;
    const int k = find_block(L, p);
    const int M = L.off[k + 1] - L.off[k];
    const int nn = p - L.off[k];
    double v = 0.0;
    if (nn != 0) {
        const double th = (double)nn / (double)M;
        const double ct = cospi(th) / sinpi(th);
        if (op == kOpHalfCot)
            v = 0.5 * ct;
        else if (op == WWBI_OP_D)
            v = (nn & 1) ? -0.5 * ct : 0.5 * ct;
        else if (nn & 1)
            v = 2.0 * ct / (double)M;
    }
    rows[p] = v;
}

__global__ void k_circ_row1(int M, int op, double *row) {
    const int nn = blockIdx.x * blockDim.x + threadIdx.x;
    if (nn >= M) return;
    double v = 0.0;
    if (nn != 0) {
        const double th = (double)nn / (double)M;
        const double ct = cospi(th) / sinpi(th);
        if (op == kOpHalfCot)
            v = 0.5 * ct;
        else if (op == WWBI_OP_D)
            v = (nn & 1) ? -0.5 * ct : 0.5 * ct;
        else if (nn & 1)
            v = 2.0 * ct / (double)M;
    }
    row[nn] = v;
}

// Circulant product on one periodic grid of M points:
//   out_m = alpha sum_l c((m - l) mod M) f_l + beta out_m.
// A block owns 64 outputs; its 16 waves split the sources into interleaved
// tiles of 64.  Each wave stages its tile of f and the 127 row entries the
// tile needs in a private LDS region (no block barrier: one wave's LDS
// operations complete in issue order), loads the next tile's values into
// registers while it sums the current one, and keeps four partial sums to
// shorten the dependent chain.  The 16 waves' sums are added in a fixed
// order at the end.
constexpr int kCT = 64;
constexpr int kCW = 16;

// keeps the compiler from moving one wave's LDS accesses across this point
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wrap_index(int d, int M) {
    d %= M;
    return d < 0 ? d + M : d;
}

// out[m0 .. m0+63] of one boundary of M nodes (see above).
__device__ __forceinline__ void circ_tile(int M, int m0, const double *__restrict__ row,
                                          const double *__restrict__ f, double *out,
                                          double alpha, double beta) {
    __shared__ double fs[kCW][kCT];
    __shared__ double rs[kCW][2 * kCT];
    __shared__ double red[kCW][kCT];
    const int lane = threadIdx.x % kCT, wv = threadIdx.x / kCT;
    const int ntiles = (M + kCT - 1) / kCT;
    // tile values: f_l (zero past M) and the row entries c(d) for
    // d = m0 - l0 - 63 + t, t in [0, 126], at t = lane and t = 64 + lane
    double fv = 0.0, r0 = 0.0, r1 = 0.0;
    auto load = [&](int tile) {
        const int l0 = tile * kCT, l = l0 + lane;
        fv = l < M ? f[l] : 0.0;
        const int base = m0 - l0 - (kCT - 1);
        r0 = row[wrap_index(base + lane, M)];
        r1 = lane < kCT - 1 ? row[wrap_index(base + kCT + lane, M)] : 0.0;
    };
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (wv < ntiles) load(wv);
    for (int tile = wv; tile < ntiles; tile += kCW) {
        wave_lds_order();          // the previous tile's reads come first
        fs[wv][lane] = fv;
        rs[wv][lane] = r0;
        rs[wv][kCT + lane] = r1;
        wave_lds_order();
        if (tile + kCW < ntiles) load(tile + kCW);
        // c(m - l) for output m = m0 + lane and l = l0 + i sits at t = lane + 63 - i
        const double *rw = &rs[wv][lane + kCT - 1];
#pragma unroll
        for (int i = 0; i < kCT; i += 4) {
            a0 += rw[-i] * fs[wv][i];
            a1 += rw[-i - 1] * fs[wv][i + 1];
            a2 += rw[-i - 2] * fs[wv][i + 2];
            a3 += rw[-i - 3] * fs[wv][i + 3];
        }
    }
    red[wv][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (wv == 0) {
        double s = 0.0;
        for (int w = 0; w < kCW; ++w) s += red[w][lane];
        const int m = m0 + lane;
        if (m < M) out[m] = alpha * s + (beta != 0.0 ? beta * out[m] : 0.0);
    }
}

__global__ __launch_bounds__(kCT * kCW) void k_circ_tile(int M, const double *__restrict__ row,
                                                         const double *__restrict__ f,
                                                         double *out, double alpha,
                                                         double beta) {
    circ_tile(M, blockIdx.x * kCT, row, f, out, alpha, beta);
}

// The same for boundaries first..last of a layout in one launch (their tiles
// run side by side): block b takes the tile of the boundary its index falls
// in; alpha0 scales boundary 0, alpha every other one.  blockIdx.y selects
// one of several vectors, at strides fs (input) and os (output).
__global__ __launch_bounds__(kCT * kCW) void k_circ_tiles(Layout L, int first, int last,
                                                          const double *__restrict__ rows,
                                                          const double *__restrict__ f, long fs,
                                                          double *out, long os, double alpha0,
                                                          double alpha, double beta) {
    f += blockIdx.y * fs;
    out += blockIdx.y * os;
    int b = blockIdx.x, k = first;
    for (; k < last; ++k) {
        const int t = (L.off[k + 1] - L.off[k] + kCT - 1) / kCT;
        if (b < t) break;
        b -= t;
    }
    const int o = L.off[k], M = L.off[k + 1] - o;
    circ_tile(M, b * kCT, rows + o, f + o, out + o, k == 0 ? alpha0 : alpha, beta);
}

// psi|_k = (1/M_k) sum_m omega_(k,m) for k >= 2 (Sec. 3.2); one block per boundary.
__global__ void k_block_means(Layout L, const double *v, double *out) {
    __shared__ double sh[16];
    const int k = blockIdx.x + 2;
    const int p0 = L.off[k], p1 = L.off[k + 1];
    double acc = 0.0;
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) acc += v[p];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = acc / (double)(p1 - p0);
}

// Fourier-tail resolution measure (the test the paper applies before it
// refines its grids, Sec. 7.1).  Boundary k of M nodes has the tail modes
// n = ceil(3M/8) .. M/2 of its real sample vector f; mode n holds
// |f^_n|^2, f^_n = sum_m f_m e^{-2 pi i n m / M}, counted twice for n < M/2
// (with its negative) and once for n = M/2.  Parseval gives the total energy
// M sum_m f_m^2.
__host__ __device__ __forceinline__ int tail_lo(int M) { return (3 * M + 7) / 8; }
__host__ __device__ __forceinline__ int tail_count(int M) { return M / 2 - tail_lo(M) + 1; }

// One wave per tail mode of every boundary, in boundary order (four modes per
// block).  Lane l takes the samples m = l, l + 64, ...; its phase advances by
// the rotation e^{-2 pi i 64 n / M} and is set exactly every 16 samples, so
// the twiddles stay within a few ulp (far below the 1e-12 test level).
constexpr int kTailWaves = 4;

__device__ __forceinline__ double wave_sum64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(64 * kTailWaves) void k_tail_modes(Layout L, int total,
                                                                const double *__restrict__ f,
                                                                double *__restrict__ modes) {
    const int gid = blockIdx.x * kTailWaves + (threadIdx.x >> 6);
    if (gid >= total) return;                  // whole waves only
    const int lane = threadIdx.x & 63;
    int b = gid, k = 0;
    for (; k < L.nb - 1; ++k) {
        const int t = tail_count(L.off[k + 1] - L.off[k]);
        if (b < t) break;
        b -= t;
    }
    const int M = L.off[k + 1] - L.off[k];
    const int n = tail_lo(M) + b;
    const double *fk = f + L.off[k];
    double sr, cr;                             // rotation by 64 samples
    sincospi(2.0 * (double)(((long)n * 64) % M) / (double)M, &sr, &cr);
    double re = 0.0, im = 0.0, c = 1.0, s = 0.0;
    // eight samples per lane are loaded before they are used
    for (int m0 = lane, i = 0; m0 < M; m0 += 64 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = m0 + 64 * u < M ? fk[m0 + 64 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u, ++i) {
            const int m = m0 + 64 * u;
            if ((i & 15) == 0) {
                sincospi(2.0 * (double)(((long)n * m) % M) / (double)M, &s, &c);
            } else {
                const double c2 = c * cr - s * sr;
                s = s * cr + c * sr;
                c = c2;
            }
            re += v[u] * c;
            im -= v[u] * s;
        }
    }
    re = wave_sum64(re);
    im = wave_sum64(im);
    if (lane == 0) modes[gid] = (2 * n == M ? 1.0 : 2.0) * (re * re + im * im);
}

// One block per boundary: out[2k] = tail energy, out[2k+1] = total energy.
__global__ __launch_bounds__(256) void k_tail_finish(Layout L, const double *__restrict__ f,
                                                     const double *__restrict__ modes,
                                                     double *__restrict__ out) {
    __shared__ double sh[8];
    const int k = blockIdx.x;
    int m0 = 0;
    for (int j = 0; j < k; ++j) m0 += tail_count(L.off[j + 1] - L.off[j]);
    const int M = L.off[k + 1] - L.off[k];
    const int cnt = tail_count(M);
    double t = 0.0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) t += modes[m0 + i];
    double e = 0.0;
    for (int m = threadIdx.x; m < M; m += blockDim.x) e += f[L.off[k] + m] * f[L.off[k] + m];
    t = block_sum(t, sh);
    e = block_sum(e, sh);
    if (threadIdx.x == 0) {
        out[2 * k] = t;
        out[2 * k + 1] = (double)M * e;
    }
}

// U_m = (u_mv + (1/2) H gamma_0 + sum over split partials of T gamma) / s_m
// (64 targets per block, the slices shared by kSliceWaves waves)
__global__ __launch_bounds__(64 * kSliceWaves) void k_U_finalize(int n0, const double *s,
                                                                 const double *umv,
                                                                 const double *hg,
                                                                 const double *part, int nsplit,
                                                                 double *U) {
    __shared__ double red[kSliceWaves][64];
    const int m = blockIdx.x * 64 + (threadIdx.x & 63);
    const double acc = sum_slices_waves<kSliceWaves>(part, nsplit, n0, m, m < n0, red);
    if (threadIdx.x >= 64 || m >= n0) return;
    U[m] = (umv[m] + 0.5 * hg[m] + acc) / s[m];
}

// wall rhs = -(sum of G_0k^dagger gamma_0 partials) - s dphi_mv/dn
__global__ __launch_bounds__(64 * kSliceWaves) void k_wall_rhs_finalize(int nw,
                                                                        const double *umv_w,
                                                                        const double *part,
                                                                        int nsplit, double *rhs) {
    __shared__ double red[kSliceWaves][64];
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const double acc = sum_slices_waves<kSliceWaves>(part, nsplit, nw, i, i < nw, red);
    if (threadIdx.x >= 64 || i >= nw) return;
    rhs[i] = -acc - umv_w[i];
}

// s dphi_mv/ds = (V1 + sum a_j / 2) x' + sum_j a_j Im{(1/2) cot((z - z_j)/2) z'}
// on every node (Sec. 5.1, the tangential companion of the normal formula).
__global__ void k_tmv(Nodes N, Flow F, int first, int count, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int p = first + i;
    const double dx = N.dx[p], dy = N.dy[p];
    double asum = 0.0;
    for (int j = 0; j < F.nobs; ++j) asum += F.a[j];
    double v = (F.V1 + 0.5 * asum) * dx;
    for (int j = 0; j < F.nobs; ++j) {
        double cr, ci;
        cot_half64(N.x[p] - F.zx[j], N.y[p] - F.zy[j], cr, ci);
        v += F.a[j] * 0.5 * (cr * dy + ci * dx);
    }
    out[i] = v;
}

// dphi/ds = (s dphi_mv/ds + local + sum of the split partials of Q gamma) / s
// (s dphi/ds when s is null),
// local = gamma_0 / 2 on the surface and -(H gamma_k)/2 on wall k.
__global__ __launch_bounds__(64 * kSliceWaves) void k_tangential_finalize(
    int n, int n0, const double *s, const double *tmv, const double *gamma, const double *hg,
    const double *part, int nsplit, double *out) {
    __shared__ double red[kSliceWaves][64];
    const int p = blockIdx.x * 64 + (threadIdx.x & 63);
    const double acc = sum_slices_waves<kSliceWaves>(part, nsplit, n, p, p < n, red);
    if (threadIdx.x >= 64 || p >= n) return;
    const double loc = p < n0 ? 0.5 * gamma[p] : -0.5 * hg[p];
    out[p] = s ? (tmv[p] + loc + acc) / s[p] : tmv[p] + loc + acc;
}

// fV = V gamma_0 / s and fU = U gamma_0 / s on the surface (Sec. 4.2 F operators)
__global__ void k_gt_vectors(int n0, const double *V, const double *U, const double *gamma,
                             const double *s, double *fV, double *fU) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n0) return;
    const double g = gamma[m] / s[m];
    fV[m] = V[m] * g;
    fU[m] = U[m] * g;
}

// The bracket of the gamma_0,t equation (Sec. 4.2) before d/dalpha:
//   e = -W.W/2 + (V - W.t) gamma_0/(2 s) - gamma_0^2/(8 s^2) + tau theta_a/s - g y - F_00,
// W.t = (s dphi_mv/ds + sum_q Q gamma)/s (the principal value, without the
// jump), W.n = U, theta_a = Im(zeta''/zeta') = 2 Im L,
// F_00 = -H(fU)/2 + KS fV + GS fU.
__global__ __launch_bounds__(64 * kSliceWaves) void k_gt_surface(
    int n0, Nodes N, double tau, double grav, const double *V, const double *U,
    const double *gamma, const double *tmv, const double *pq, int nsq, const double *hfu,
    const double *kfv, const double *gfu, double *e) {
    __shared__ double red[kSliceWaves][64];
    const int m = blockIdx.x * 64 + (threadIdx.x & 63);
    const double acc = sum_slices_waves<kSliceWaves>(pq, nsq, n0, m, m < n0, red);
    if (threadIdx.x >= 64 || m >= n0) return;
    const double s = N.s[m], g0 = gamma[m], u = U[m];
    const double wt = (tmv[m] + acc) / s;
    const double F00 = -0.5 * hfu[m] + kfv[m] + gfu[m];
    e[m] = -0.5 * (wt * wt + u * u) + (V[m] - wt) * g0 / (2.0 * s) - g0 * g0 / (8.0 * s * s) +
           tau * 2.0 * N.lim[m] / s - grav * N.y[m] - F00;
}

// Per surface node of the energy density (Sec. 5.2, rho = 1):
//   e = tau s + g y^2 x' / 2 + psi phi_alpha / 2,
//   psi = psi_mv + (H omega_0)/2 + sum of the split partials of P omega,
//   phi_alpha = D phi~ + s dphi_mv/ds.
__global__ __launch_bounds__(64 * kSliceWaves) void k_energy_terms(
    int n0, Nodes N, Flow F, double tau, double grav, const double *hw, const double *part,
    int nsplit, const double *dphi, const double *tmv, double *e) {
    __shared__ double red[kSliceWaves][64];
    const int m = blockIdx.x * 64 + (threadIdx.x & 63);
    const double acc = sum_slices_waves<kSliceWaves>(part, nsplit, n0, m, m < n0, red);
    if (threadIdx.x >= 64 || m >= n0) return;
    const double x = N.x[m], y = N.y[m];
    const double psi = psi_mv(F, x, y) + 0.5 * hw[m] + acc;
    const double pa = dphi[m] + tmv[m];
    e[m] = tau * N.s[m] + 0.5 * grav * y * y * N.dx[m] + 0.5 * psi * pa;
}

// E = mean(e) + sum_{j>=2} a_j psi|_j / 2, one block, fixed summation order.
__global__ void k_energy_final(int n0, const double *e, Flow F, const double *psi_k,
                               double *E) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int m = threadIdx.x; m < n0; m += blockDim.x) acc += e[m];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        double v = acc / (double)n0;
        for (int j = 0; j < F.nobs; ++j) v += 0.5 * F.a[j] * psi_k[j];
        *E = v;
    }
}

__global__ void k_surface_base(int n, const double *xt, const double *yt, double *x, double *y) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    x[m] = 2.0 * M_PI * (double)m / (double)n + xt[m];
    y[m] = yt[m];
}

__global__ void k_add_scalar(int n, double *v, double c) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) v[m] += c;
}

}  // namespace

void launch_prep_nodes(const Layout &L, const double *x, const double *y, const double *dx,
                       const double *dy, const double *ddx, const double *ddy, int *bid,
                       int *loc, int *Mk, double *w, double *s, double *lre, double *lim,
                       double *ex, double *ey, double *exl, double *eyl, hipStream_t st) {
    hipLaunchKernelGGL(k_prep_nodes, dim3(cdiv(L.n, 256)), dim3(256), 0, st, L, x, y, dx, dy, ddx,
                       ddy, bid, loc, Mk, w, s, lre, lim, ex, ey, exl, eyl);
}

int validate_data_blocks(int nphi) {
    return std::max(1, std::min(kValidateBlocks, cdiv(nphi, 8192)));
}

void launch_validate(const Layout &L, const Nodes &N, const double *phi, int nphi, double *out,
                     hipStream_t st) {
    const int pb = validate_data_blocks(nphi);
    // 1024 threads: a block walks its boundary (or share of the data) in few
    // rounds of loads (12 -> 9 us at M = 10240 against 256 threads)
    hipLaunchKernelGGL(k_validate, dim3(L.nb + pb), dim3(1024), 0, st, L, N, phi, nphi, pb, out);
}

void launch_rhs_phi(const Layout &L, const Nodes &N, const Flow &F, const double *phi,
                    const double *psi_wall, double *b, hipStream_t st) {
    hipLaunchKernelGGL(k_rhs_phi, dim3(cdiv(L.n, 256)), dim3(256), 0, st, L, N, F, phi, psi_wall,
                       b);
}

void launch_umv(const Nodes &N, const Flow &F, int first, int count, double *out,
                hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_umv, dim3(cdiv(count, 256)), dim3(256), 0, st, N, F, first, count, out);
}

void launch_tmv(const Nodes &N, const Flow &F, int first, int count, double *out,
                hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_tmv, dim3(cdiv(count, 256)), dim3(256), 0, st, N, F, first, count, out);
}

void launch_tangential_finalize(int n, int n0, const double *s, const double *tmv,
                                const double *gamma, const double *hg, const double *part,
                                int nsplit, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_tangential_finalize, dim3(cdiv(n, 64)), dim3(64 * kSliceWaves), 0, st,
                       n, n0, s, tmv, gamma, hg, part, nsplit, out);
}

void launch_gt_vectors(int n0, const double *V, const double *U, const double *gamma,
                       const double *s, double *fV, double *fU, hipStream_t st) {
    hipLaunchKernelGGL(k_gt_vectors, dim3(cdiv(n0, 256)), dim3(256), 0, st, n0, V, U, gamma, s,
                       fV, fU);
}

void launch_gt_surface(int n0, const Nodes &N, double tau, double grav, const double *V,
                       const double *U, const double *gamma, const double *tmv,
                       const double *pq, int nsq, const double *hfu, const double *kfv,
                       const double *gfu, double *e, hipStream_t st) {
    hipLaunchKernelGGL(k_gt_surface, dim3(cdiv(n0, 64)), dim3(64 * kSliceWaves), 0, st, n0, N,
                       tau, grav, V, U, gamma, tmv, pq, nsq, hfu, kfv, gfu, e);
}

void launch_energy(int n0, const Nodes &N, const Flow &F, double tau, double grav,
                   const double *hw, const double *part, int nsplit, const double *dphi,
                   const double *tmv, const double *psi_k, double *e, double *E, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_terms, dim3(cdiv(n0, 64)), dim3(64 * kSliceWaves), 0, st, n0, N,
                       F, tau, grav, hw, part, nsplit, dphi, tmv, e);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(1024), 0, st, n0, e, F, psi_k, E);
}

void launch_circulant_rows(const Layout &L, int op, double *rows, hipStream_t st) {
    hipLaunchKernelGGL(k_circ_rows, dim3(cdiv(L.n, 256)), dim3(256), 0, st, L, op, rows);
}

void launch_circulant_batched(const Layout &L, const double *rows, const double *f, long fs,
                              double *out, long os, int nv, double alpha0, double alpha,
                              double beta, int first_block, int last_block, hipStream_t st) {
    int tiles = 0;
    for (int k = first_block; k <= last_block; ++k) tiles += cdiv(L.off[k + 1] - L.off[k], kCT);
    if (tiles == 0 || nv < 1) return;
    hipLaunchKernelGGL(k_circ_tiles, dim3(tiles, nv), dim3(kCT * kCW), 0, st, L, first_block,
                       last_block, rows, f, fs, out, os, alpha0, alpha, beta);
}

void launch_circulant_apply2(const Layout &L, const double *rows, const double *f, double *out,
                             double alpha0, double alpha, double beta, int first_block,
                             int last_block, hipStream_t st) {
    launch_circulant_batched(L, rows, f, 0, out, 0, 1, alpha0, alpha, beta, first_block,
                             last_block, st);
}

void launch_circulant_apply(const Layout &L, const double *rows, const double *f, double *out,
                            double alpha, double beta, int first_block, int last_block,
                            hipStream_t st) {
    launch_circulant_apply2(L, rows, f, out, alpha, alpha, beta, first_block, last_block, st);
}

void launch_circ_row1(int M, int op, double *row, hipStream_t st) {
    hipLaunchKernelGGL(k_circ_row1, dim3(cdiv(M, 256)), dim3(256), 0, st, M, op, row);
}

void launch_circ_apply1(int M, const double *row, const double *f, double *out, double alpha,
                        double beta, hipStream_t st) {
    hipLaunchKernelGGL(k_circ_tile, dim3(cdiv(M, kCT)), dim3(kCT * kCW), 0, st, M, row, f, out,
                       alpha, beta);
}

int tail_modes_total(const Layout &L) {
    int t = 0;
    for (int k = 0; k < L.nb; ++k) t += tail_count(L.off[k + 1] - L.off[k]);
    return t;
}

void launch_tail_monitor(const Layout &L, const double *f, double *modes, double *out,
                         hipStream_t st) {
    const int total = tail_modes_total(L);
    hipLaunchKernelGGL(k_tail_modes, dim3((total + kTailWaves - 1) / kTailWaves),
                       dim3(64 * kTailWaves), 0, st, L, total, f, modes);
    hipLaunchKernelGGL(k_tail_finish, dim3(L.nb), dim3(256), 0, st, L, f, modes, out);
}

void launch_block_means(const Layout &L, const double *v, double *out, hipStream_t st) {
    if (L.nb <= 2) return;
    hipLaunchKernelGGL(k_block_means, dim3(L.nb - 2), dim3(256), 0, st, L, v, out);
}

void launch_U_finalize(int n0, const double *s, const double *umv, const double *hg,
                       const double *part, int nsplit, double *U, hipStream_t st) {
    hipLaunchKernelGGL(k_U_finalize, dim3(cdiv(n0, 64)), dim3(64 * kSliceWaves), 0, st, n0, s,
                       umv, hg, part, nsplit, U);
}

void launch_wall_rhs_finalize(int nw, const double *umv_w, const double *part, int nsplit,
                              double *rhs, hipStream_t st) {
    hipLaunchKernelGGL(k_wall_rhs_finalize, dim3(cdiv(nw, 64)), dim3(64 * kSliceWaves), 0, st,
                       nw, umv_w, part, nsplit, rhs);
}

void launch_surface_base(int n, const double *xt, const double *yt, double *x, double *y,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_surface_base, dim3(cdiv(n, 256)), dim3(256), 0, st, n, xt, yt, x, y);
}

void launch_add_scalar(int n, double *v, double c, hipStream_t st) {
    hipLaunchKernelGGL(k_add_scalar, dim3(cdiv(n, 256)), dim3(256), 0, st, n, v, c);
}

}  // namespace wwbi
