// Device work of one Runge-Kutta stage of the free-surface evolution
// (Sec. 2.1 graph surfaces, Sec. 2.2 the HLS reconstruction from P theta,
// Sec. 3.5 the phi~ equation, Sec. 5 the tangential velocity V and the
// 36th-order filter) and the combination of stage derivatives.
//
// Every surface array has M = M_0 entries on the uniform grid alpha_m =
// 2 pi m / M.  Means are one-block reductions in a fixed order.
#include "entries.h"
#include "internal.h"

namespace wwbi {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

constexpr int kRB = 1024;   // threads of the one-block reductions

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

// sigma_k = exp(-36 (k / (M/2))^36), the filter's symbol for 0 <= k < M/2
__global__ void k_filter_sigma(int M, double *sigma) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M / 2) return;
    const double r = (double)k / (0.5 * (double)M);
    sigma[k] = exp(-36.0 * pow(r, 36.0));
}

// Circulant rows on the M-point grid (Nyquist mode zeroed, like D and H):
//   antiderivative 1/(ik), k != 0:  c(n) = (2/M) sum_{k=1}^{M/2-1} sin(2 pi k n / M) / k
//   filter sigma_k:                  c(n) = (1 + 2 sum_{k=1}^{M/2-1} sigma_k cos(2 pi k n / M)) / M
// The angle 2 k n / M (in units of pi) is reduced exactly in integers.
__global__ void k_evolve_rows(int M, const double *sigma, double *rint, double *rfil) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= M) return;
    const long twoM = 2L * M;
    double si = 0.0, sf = 0.0;
    for (int k = 1; k < M / 2; ++k) {
        const double t = (double)((2L * k * n) % twoM) / (double)M;
        si += sinpi(t) / (double)k;
        sf += sigma[k] * cospi(t);
    }
    rint[n] = 2.0 * si / (double)M;
    rfil[n] = (1.0 + 2.0 * sf) / (double)M;
}

// graph surface zeta = alpha + i eta: x = alpha, y = eta, x' = 1, x'' = 0
__global__ void k_graph_base(int M, const double *eta, double *x, double *y, double *dx,
                             double *ddx) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    x[m] = 2.0 * M_PI * (double)m / (double)M;
    y[m] = eta[m];
    dx[m] = 1.0;
    ddx[m] = 0.0;
}

// out[0] = mean(cos a), out[1] = mean(sin a)   (one block)
__global__ void k_mean_cs(int M, const double *a, double *out) {
    __shared__ double sh[kRB / 64];
    double c = 0.0, s = 0.0;
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        double sv, cv;
        sincos(a[m], &sv, &cv);
        c += cv;
        s += sv;
    }
    c = block_sum(c, sh);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        out[0] = c / (double)M;
        out[1] = s / (double)M;
    }
}

// out[0] = mean(a b) (b may be null: mean(a))   (one block)
__global__ void k_mean_prod(int M, const double *a, const double *b, double *out) {
    __shared__ double sh[kRB / 64];
    double t = 0.0;
    for (int m = threadIdx.x; m < M; m += blockDim.x) t += b ? a[m] * b[m] : a[m];
    t = block_sum(t, sh);
    if (threadIdx.x == 0) out[0] = t / (double)M;
}

// theta = P theta + arg(C - iS), s_alpha = (C^2 + S^2)^(-1/2),
// zeta' = s_alpha e^{i theta}; xm1 = x' - 1 (the antiderivative's argument)
__global__ void k_hls_slope(int M, const double *Pt, const double *cs, double *dx, double *dy,
                            double *xm1) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double C = cs[0], S = cs[1];
    const double th0 = atan2(-S, C);
    const double sa = 1.0 / sqrt(C * C + S * S);
    double sv, cv;
    sincos(Pt[m] + th0, &sv, &cv);
    dx[m] = sa * cv;
    dy[m] = sa * sv;
    xm1[m] = sa * cv - 1.0;
}

// xi = alpha + xa - xa(0), eta = ya - <ya xi'>
__global__ void k_hls_xy(int M, const double *xa, const double *ya, const double *mean_yx,
                         double *x, double *y) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    x[m] = 2.0 * M_PI * (double)m / (double)M + xa[m] - xa[0];
    y[m] = ya[m] - mean_yx[0];
}

// zeta'' = i theta_alpha zeta' (s_alpha does not depend on alpha)
__global__ void k_hls_curv(int M, const double *ta, const double *dx, const double *dy,
                           double *ddx, double *ddy) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    ddx[m] = -ta[m] * dy[m];
    ddy[m] = ta[m] * dx[m];
}

// graph: V = eta_alpha U, eta_t = sqrt(1 + eta_alpha^2) U
__global__ void k_graph_rates(int M, const double *U, const double *dy, double *V, double *qt) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double ea = dy[m];
    V[m] = ea * U[m];
    qt[m] = sqrt(1.0 + ea * ea) * U[m];
}

__global__ void k_mul(int M, const double *a, const double *b, double *out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) out[m] = a[m] * b[m];
}

// V = Vi - Vi(0) + U(0) eta'(0) / xi'(0), so that xi(0) stays 0
__global__ void k_hls_V(int M, const double *Vi, const double *U, const double *dx,
                        const double *dy, double *V) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    V[m] = Vi[m] - Vi[0] + U[0] * dy[0] / dx[0];
}

// f = (U_alpha + V theta_alpha) / s_alpha
__global__ void k_hls_f(int M, const double *dU, const double *V, const double *ta,
                        const double *dx, const double *dy, double *f) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double sa = sqrt(dx[m] * dx[m] + dy[m] * dy[m]);
    f[m] = (dU[m] + V[m] * ta[m]) / sa;
}

__global__ void k_sub_mean(int M, const double *f, const double *mean, double *out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) out[m] = f[m] - mean[0];
}

// phi~_t = (phi~_alpha / s) V + (U - s dphi_mv/dn / s) U - |grad phi|^2 / 2 - g eta
//          + tau theta_alpha / s,  |grad phi|^2 = (phi_alpha / s)^2 + U^2,
// phi_alpha = phi~_alpha + s dphi_mv/ds, theta_alpha = Im(zeta''/zeta') = 2 Im L.
__global__ void k_phit(int M, Nodes N, Flow F, const double *dphi, const double *U,
                       const double *V, double tau, double grav, double *out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double dx = N.dx[m], dy = N.dy[m];
    double asum = 0.0;
    for (int j = 0; j < F.nobs; ++j) asum += F.a[j];
    double un = -(F.V1 + 0.5 * asum) * dy;   // s dphi_mv/dn
    double ut = (F.V1 + 0.5 * asum) * dx;    // s dphi_mv/ds
    for (int j = 0; j < F.nobs; ++j) {
        double cr, ci;
        cot_half64(N.x[m] - F.zx[j], N.y[m] - F.zy[j], cr, ci);
        un += F.a[j] * 0.5 * (cr * dx - ci * dy);
        ut += F.a[j] * 0.5 * (cr * dy + ci * dx);
    }
    const double s = N.s[m], u = U[m];
    const double pa = dphi[m] + ut;
    const double grad2 = (pa / s) * (pa / s) + u * u;
    out[m] = dphi[m] / s * V[m] + (u - un / s) * u - 0.5 * grad2 - grav * N.y[m] +
             tau * 2.0 * N.lim[m] / s;
}

// out = base + h sum_j c_j K_j, K_j = K + j ld, the sum in increasing j
__global__ void k_rk_combine(int M, const double *base, const double *K, long ld, RkCoef co,
                             double *out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    double acc = 0.0;
    for (int j = 0; j < co.ns; ++j)
        if (co.c[j] != 0.0) acc += co.c[j] * K[(long)j * ld + m];
    out[m] = base[m] + co.h * acc;
}

}  // namespace

void launch_evolve_rows(int M, double *sigma, double *rint, double *rfil, hipStream_t st) {
    hipLaunchKernelGGL(k_filter_sigma, dim3(cdiv(M / 2, 256)), dim3(256), 0, st, M, sigma);
    hipLaunchKernelGGL(k_evolve_rows, dim3(cdiv(M, 64)), dim3(64), 0, st, M, sigma, rint, rfil);
}

void launch_graph_base(int M, const double *eta, double *x, double *y, double *dx, double *ddx,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_graph_base, dim3(cdiv(M, 256)), dim3(256), 0, st, M, eta, x, y, dx, ddx);
}

void launch_mean_cs(int M, const double *a, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_mean_cs, dim3(1), dim3(kRB), 0, st, M, a, out);
}

void launch_mean_prod(int M, const double *a, const double *b, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_mean_prod, dim3(1), dim3(kRB), 0, st, M, a, b, out);
}

void launch_hls_slope(int M, const double *Pt, const double *cs, double *dx, double *dy,
                      double *xm1, hipStream_t st) {
    hipLaunchKernelGGL(k_hls_slope, dim3(cdiv(M, 256)), dim3(256), 0, st, M, Pt, cs, dx, dy, xm1);
}

void launch_hls_xy(int M, const double *xa, const double *ya, const double *mean_yx, double *x,
                   double *y, hipStream_t st) {
    hipLaunchKernelGGL(k_hls_xy, dim3(cdiv(M, 256)), dim3(256), 0, st, M, xa, ya, mean_yx, x, y);
}

void launch_hls_curv(int M, const double *ta, const double *dx, const double *dy, double *ddx,
                     double *ddy, hipStream_t st) {
    hipLaunchKernelGGL(k_hls_curv, dim3(cdiv(M, 256)), dim3(256), 0, st, M, ta, dx, dy, ddx, ddy);
}

void launch_graph_rates(int M, const double *U, const double *dy, double *V, double *qt,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_graph_rates, dim3(cdiv(M, 256)), dim3(256), 0, st, M, U, dy, V, qt);
}

void launch_mul(int M, const double *a, const double *b, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_mul, dim3(cdiv(M, 256)), dim3(256), 0, st, M, a, b, out);
}

void launch_hls_V(int M, const double *Vi, const double *U, const double *dx, const double *dy,
                  double *V, hipStream_t st) {
    hipLaunchKernelGGL(k_hls_V, dim3(cdiv(M, 256)), dim3(256), 0, st, M, Vi, U, dx, dy, V);
}

void launch_hls_f(int M, const double *dU, const double *V, const double *ta, const double *dx,
                  const double *dy, double *f, hipStream_t st) {
    hipLaunchKernelGGL(k_hls_f, dim3(cdiv(M, 256)), dim3(256), 0, st, M, dU, V, ta, dx, dy, f);
}

void launch_sub_mean(int M, const double *f, const double *mean, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sub_mean, dim3(cdiv(M, 256)), dim3(256), 0, st, M, f, mean, out);
}

void launch_phit(int M, const Nodes &N, const Flow &F, const double *dphi, const double *U,
                 const double *V, double tau, double grav, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_phit, dim3(cdiv(M, 256)), dim3(256), 0, st, M, N, F, dphi, U, V, tau,
                       grav, out);
}

void launch_rk_combine(int M, const double *base, const double *K, long ld, const RkCoef &co,
                       double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_rk_combine, dim3(cdiv(M, 256)), dim3(256), 0, st, M, base, K, ld, co,
                       out);
}

}  // namespace wwbi
