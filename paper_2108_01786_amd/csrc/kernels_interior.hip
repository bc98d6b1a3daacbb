// Values inside the fluid from boundary values (Sec. 5.1 and the
// Helsing-Ojala appendix): for z in the fluid,
//   f(z) = sum_km lam_km f_km / sum_km lam_km,
//   lam_km = sigma_k / M_k * (1/2) cot((zeta_km - z)/2) zeta'_km,
// the trapezoid sums of contour integrals over the positively oriented
// boundary of the fluid: the free surface against its parameter
// (sigma_0 = -1), the bottom and the clockwise obstacles along theirs.
// A point that coincides with a node takes that node's value.
//
// Also the boundary velocity u - i v = (dphi/ds - i dphi/dn) |zeta'| / zeta'.
#include "ddmath.h"
#include "entries.h"
#include "internal.h"

namespace wwbi {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

constexpr int kHoStage = 256;

struct HoNode {
    double ex, ey, exl, eyl, x, y, dx, dy, w, fr, fi;
    int neg;   // free-surface node (sigma = -1)
};

// Partial sums over chunk blockIdx.y of the nodes, one point per thread:
// part[c][s][p] for c = Re num, Im num, Re den, Im den; hit[s][p] = the first
// node of the chunk that coincides with the point, or -1.
__global__ __launch_bounds__(256) void k_ho_partial(Nodes N, int n, int n0, int P,
                                                    const double *__restrict__ zx,
                                                    const double *__restrict__ zy,
                                                    const double *__restrict__ fr,
                                                    const double *__restrict__ fi, int chunk,
                                                    double *__restrict__ part,
                                                    int *__restrict__ hit) {
    __shared__ HoNode sn[kHoStage];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool live = p < P;
    const double x = live ? zx[p] : 0.0, y = live ? zy[p] : 0.0;
    // E_z = e^{i z} as a double-double, like the nodes' E: the difference
    // E_zeta - E_z then keeps its relative accuracy for nearby points
    DD ezr, ezi;
    dd_expi(x, y, ezr, ezi);
    const double er = ezr.hi, ei = ezi.hi, erl = ezr.lo, eil = ezi.lo;
    const double ee = er * er + ei * ei;
    double nr = 0.0, ni = 0.0, dr = 0.0, di = 0.0;
    int h = -1;
    const int qb = blockIdx.y * chunk, qe = min(n, qb + chunk);
    for (int qq = qb; qq < qe; qq += kHoStage) {
        const int q = qq + threadIdx.x;
        if (q < qe) {
            HoNode v;
            v.ex = N.ex[q]; v.ey = N.ey[q]; v.exl = N.exl[q]; v.eyl = N.eyl[q];
            v.x = N.x[q]; v.y = N.y[q];
            v.dx = N.dx[q]; v.dy = N.dy[q]; v.w = N.w[q]; v.fr = fr[q]; v.fi = fi[q];
            v.neg = q < n0 ? 1 : 0;
            sn[threadIdx.x] = v;
        }
        __syncthreads();
        const int m = min(kHoStage, qe - qq);
        if (live) {
            for (int i = 0; i < m; ++i) {
                const HoNode &v = sn[i];
                const double ddr = (v.ex - er) + (v.exl - erl);
                const double ddi = (v.ey - ei) + (v.eyl - eil);
                const double den = ddr * ddr + ddi * ddi;
                double kr, ki;
                if (den == 0.0) {       // the point is this node (or a period image)
                    if (h < 0) h = qq + i;
                    continue;
                }
                if (den * 4096.0 < ee) {
                    const double u = v.x - x, w = v.y - y;
                    if (u == 0.0 && w == 0.0) {   // the node itself
                        if (h < 0) h = qq + i;
                        continue;
                    }
                    cot_half64(u, w, kr, ki);
                } else {
                    // cot((zeta - z)/2) = i (E_zeta + E_z) / (E_zeta - E_z)
                    const double sr = v.ex + er, si = v.ey + ei;
                    const double inv = 1.0 / den;
                    const double pr = (sr * ddr + si * ddi) * inv;
                    const double pi = (si * ddr - sr * ddi) * inv;
                    kr = -pi;
                    ki = pr;
                }
                // lam = sigma w (1/2) kappa zeta'
                const double sw = (v.neg ? -0.5 : 0.5) * v.w;
                const double lr = sw * (kr * v.dx - ki * v.dy);
                const double li = sw * (kr * v.dy + ki * v.dx);
                nr += lr * v.fr - li * v.fi;
                ni += lr * v.fi + li * v.fr;
                dr += lr;
                di += li;
            }
        }
        __syncthreads();
    }
    if (live) {
        const long st = (long)gridDim.y * P;
        const long o = (long)blockIdx.y * P + p;
        part[o] = nr;
        part[st + o] = ni;
        part[2 * st + o] = dr;
        part[3 * st + o] = di;
        hit[o] = h;
    }
}

// f(z) = num / den, or the coinciding node's value; neg_im stores -Im f
__global__ void k_ho_finalize(int P, int ns, const double *__restrict__ part,
                              const int *__restrict__ hit, const double *__restrict__ fr,
                              const double *__restrict__ fi, int neg_im,
                              double *__restrict__ outr, double *__restrict__ outi) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int h = -1;
    for (int s = 0; s < ns && h < 0; ++s) h = hit[(long)s * P + p];
    const double sg = neg_im ? -1.0 : 1.0;
    if (h >= 0) {
        outr[p] = fr[h];
        outi[p] = sg * fi[h];
        return;
    }
    const long st = (long)ns * P;
    const double nr = sum_slices(part, ns, P, p), ni = sum_slices(part + st, ns, P, p);
    const double dr = sum_slices(part + 2 * st, ns, P, p);
    const double di = sum_slices(part + 3 * st, ns, P, p);
    const double inv = 1.0 / (dr * dr + di * di);
    outr[p] = (nr * dr + ni * di) * inv;
    outi[p] = sg * (ni * dr - nr * di) * inv;
}

// u - i v on every node from s dphi/ds and s dphi/dn:
// (dphi/ds - i dphi/dn) |zeta'| / zeta' = (sds - i sdn) / zeta';
// stores (u, v), or (Re, Im) of u - i v when phi_prime is set
__global__ void k_boundary_velocity(int n, const double *dx, const double *dy, const double *sds,
                                    const double *sdn, int phi_prime, double *u, double *v) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double a = dx[p], b = dy[p];
    const double inv = 1.0 / (a * a + b * b);
    // (sds - i sdn) (a - i b) / |zeta'|^2
    const double re = (sds[p] * a - sdn[p] * b) * inv;
    const double im = (-sds[p] * b - sdn[p] * a) * inv;
    u[p] = re;
    v[p] = phi_prime ? im : -im;
}

// s dphi/dn = s dphi_mv/dn + local + sum of the split partials of T gamma,
// local = H gamma_0 / 2 on the surface and -gamma_k / 2 on wall k
__global__ __launch_bounds__(64 * kSliceWaves) void k_normal_finalize(
    int n, int n0, const double *umv, const double *gamma, const double *hg, const double *part,
    int nsplit, double *out) {
    __shared__ double red[kSliceWaves][64];
    const int p = blockIdx.x * 64 + (threadIdx.x & 63);
    const double acc = sum_slices_waves<kSliceWaves>(part, nsplit, n, p, p < n, red);
    if (threadIdx.x >= 64 || p >= n) return;
    const double loc = p < n0 ? 0.5 * hg[p] : -0.5 * gamma[p];
    out[p] = umv[p] + loc + acc;
}

// Dirichlet data of phi_t - C on the surface (Sec. 5.1, Laplace-Young):
// tau kappa - |grad phi|^2 / 2 - g eta, kappa = Im(zeta''/zeta')/s = 2 Im L / s
__global__ void k_pressure_data(int n0, Nodes N, const double *sds, const double *sdn,
                                double tau, double grav, double *b) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n0) return;
    const double s = N.s[m];
    const double a = sds[m] / s, c = sdn[m] / s;
    b[m] = tau * 2.0 * N.lim[m] / s - 0.5 * (a * a + c * c) - grav * N.y[m];
}

// Fluid-side boundary values of the auxiliary Cauchy integrals:
// surface Re = the data, Im = P omega + H(omega_0)/2; wall k Re = KS omega_0 +
// GS omega_w - H(omega_k)/2, Im = psi|_k (mean of omega_k for k >= 2, 0 on
// the bottom).
__global__ void k_phi_aux_values(int n, int n0, const double *data, const double *ps,
                                 const double *rw, const double *hw, const int *bid,
                                 const double *means, double *fr, double *fi) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (p < n0) {
        fr[p] = data[p];
        fi[p] = ps[p] + 0.5 * hw[p];
    } else {
        const int k = bid[p];
        fr[p] = rw[p - n0] - 0.5 * hw[p];
        fi[p] = k >= 2 ? means[k - 2] : 0.0;
    }
}

// p = -(phi_t - C) - |u - i v|^2 / 2 - g y
__global__ void k_pressure_final(int P, const double *phit, const double *wr, const double *wi,
                                 const double *zy, double grav, double *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    out[p] = -phit[p] - 0.5 * (wr[p] * wr[p] + wi[p] * wi[p]) - grav * zy[p];
}

}  // namespace

void launch_pressure_data(int n0, const Nodes &N, const double *sds, const double *sdn,
                          double tau, double grav, double *b, hipStream_t st) {
    hipLaunchKernelGGL(k_pressure_data, dim3(cdiv(n0, 256)), dim3(256), 0, st, n0, N, sds, sdn,
                       tau, grav, b);
}

void launch_phi_aux_values(int n, int n0, const double *data, const double *ps,
                           const double *rw, const double *hw, const int *bid,
                           const double *means, double *fr, double *fi, hipStream_t st) {
    hipLaunchKernelGGL(k_phi_aux_values, dim3(cdiv(n, 256)), dim3(256), 0, st, n, n0, data, ps, rw,
                       hw, bid, means, fr, fi);
}

void launch_pressure_final(int P, const double *phit, const double *wr, const double *wi,
                           const double *zy, double grav, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_pressure_final, dim3(cdiv(P, 256)), dim3(256), 0, st, P, phit, wr, wi, zy,
                       grav, out);
}

static int ho_chunk(int P, int n) {
    int ns = cdiv(2048, cdiv(P, 256));
    ns = ns < 1 ? 1 : (ns > 64 ? 64 : ns);
    int c = cdiv(n, ns);
    c = cdiv(c, 32) * 32;
    return c < 32 ? 32 : c;
}

int ho_slices(int P, int n) { return cdiv(n, ho_chunk(P, n)); }

namespace {
// out[0] = points with a non-finite coordinate, out[1] = points with |y| above
// the node height limit (one block; the counts are exact small integers)
__global__ __launch_bounds__(256) void k_check_points(int P, const double *__restrict__ zx,
                                                      const double *__restrict__ zy,
                                                      double *__restrict__ out) {
    __shared__ double sh[8];
    double bad = 0.0, far = 0.0;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        const double x = zx[p], y = zy[p];
        const bool fin = isfinite(x) && isfinite(y);
        bad += fin ? 0.0 : 1.0;
        far += fin && fabs(y) > kMaxAbsY ? 1.0 : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        bad += __shfl_xor(bad, o, 64);
        far += __shfl_xor(far, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[2 * w] = bad;
        sh[2 * w + 1] = far;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0, f = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            b += sh[2 * i];
            f += sh[2 * i + 1];
        }
        out[0] = b;
        out[1] = f;
    }
}
}  // namespace

void launch_check_points(int P, const double *zx, const double *zy, double *out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_check_points, dim3(1), dim3(256), 0, st, P, zx, zy, out);
}

void launch_helsing_ojala(const Nodes &N, int n, int n0, int P, const double *zx,
                          const double *zy, const double *fr, const double *fi, double *part,
                          int *hit, bool neg_im, double *outr, double *outi, hipStream_t st) {
    const int chunk = ho_chunk(P, n);
    const int ns = cdiv(n, chunk);
    hipLaunchKernelGGL(k_ho_partial, dim3(cdiv(P, 256), ns), dim3(256), 0, st, N, n, n0, P, zx, zy,
                       fr, fi, chunk, part, hit);
    hipLaunchKernelGGL(k_ho_finalize, dim3(cdiv(P, 64)), dim3(64), 0, st, P, ns, part, hit, fr, fi,
                       neg_im ? 1 : 0, outr, outi);
}

void launch_boundary_velocity(int n, const double *dx, const double *dy, const double *sds,
                              const double *sdn, bool phi_prime, double *u, double *v,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_boundary_velocity, dim3(cdiv(n, 256)), dim3(256), 0, st, n, dx, dy, sds,
                       sdn, phi_prime ? 1 : 0, u, v);
}

void launch_normal_finalize(int n, int n0, const double *umv, const double *gamma,
                            const double *hg, const double *part, int nsplit, double *out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_normal_finalize, dim3(cdiv(n, 64)), dim3(64 * kSliceWaves), 0, st, n,
                       n0, umv, gamma, hg, part, nsplit, out);
}

}  // namespace wwbi
