// Device-resident restarted GMRES: Arnoldi with classical Gram-Schmidt applied
// twice (CGS2), Givens rotations on the Hessenberg column, triangular solve and
// solution update.  Every reduction has a fixed order (partials per block, then
// a sequential sum over blocks), so results are bitwise reproducible.
//
// G blocks each own one contiguous chunk of the vectors.  Every block reduces
// the G partials itself (in the same order), which avoids a separate launch
// per reduction.  Kernels of an iteration return at once when the cycle has
// ended (gs->active == 0), so the host may enqueue several steps between
// reads of the flag.
#include <cstddef>

#include "internal.h"

namespace wwbi {

namespace {

constexpr int kT = 256;       // threads per block
constexpr int kMaxG = 64;     // max blocks of the vector kernels

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// system index of a batched launch (gridDim.y systems in lockstep)
__device__ __forceinline__ long sys() { return (long)blockIdx.y; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void chunk_of(int n, int G, int b, int &c0, int &c1) {
    const int len = (n + G - 1) / G;
    c0 = b * len;
    c1 = min(n, c0 + len);
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kT / 64; ++i) t += sh[i];
    return t;
}

// (active, jdone) of a cycle state as one 8-byte word.  The Hessenberg block
// of k_cgs_final may end the cycle while vector blocks of the same launch
// still read the flag: a block of step j runs when the cycle is active or was
// ended by step j itself (jdone = j + 1 only then), whichever word it sees.
static_assert(offsetof(GState, active) == 0 && offsetof(GState, jdone) == 4,
              "active and jdone share one aligned 8-byte word");
__device__ __forceinline__ bool step_runs(const GState *gs, int j) {
    const unsigned long long v =
        __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<GState *>(gs)),
                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (unsigned)(v & 0xffffffffu) != 0u || (int)(unsigned)(v >> 32) == j + 1;
}
__device__ __forceinline__ void store_step(GState *gs, int active, int jdone) {
    const unsigned long long v =
        (unsigned long long)(unsigned)active | ((unsigned long long)(unsigned)jdone << 32);
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(gs), v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Copy of the state at the end of cycle `cyc` into host-visible memory (m may
// be null), written through volatile stores that bypass the caches, so that
// the host reads it without a copy once the kernel has completed.  The write
// crosses to host memory and delays the kernel's completion by a few
// microseconds, so it happens once per cycle, not per step.
__device__ __forceinline__ void publish(GState *m, const GState *gs, int cyc) {
    if (!m) return;
    volatile GState *d = m;
    d->its = gs->its;
    d->jdone = gs->jdone;
    d->breakdown = gs->breakdown;
    d->bnorm = gs->bnorm;
    d->tol_abs = gs->tol_abs;
    d->beta = gs->beta;
    d->resid = gs->resid;
    d->active = gs->active;
    d->cyc = cyc;
}

// P[b] = sum over chunk b of v^2
__global__ __launch_bounds__(kT) void k_norm_partial(const double *v, int n, double *P, int G,
                                                     Bat bt) {
    __shared__ double sh[kT / 64];
    v += sys() * bt.vec;
    P += sys() * bt.p;
    int c0, c1;
    chunk_of(n, G, blockIdx.x, c0, c1);
    double a = 0.0;
    for (int i = c0 + threadIdx.x; i < c1; i += kT) a += v[i] * v[i];
    a = block_sum(a, sh);
    if (threadIdx.x == 0) P[blockIdx.x] = a;
}

__global__ void k_set_tol(const double *P, int G, double tol, GState *gs, Bat bt) {
    P += sys() * bt.p;
    gs += sys();
    double v = (int)threadIdx.x < G ? P[threadIdx.x] : 0.0;
    v = wave_sum(v);
    if (threadIdx.x == 0) {
        gs->bnorm = sqrt(v);
        gs->tol_abs = tol * gs->bnorm;
        gs->its = 0;
    }
}

// v_0 = r / beta (FP64 and FP32 copies), g = (beta, 0, ...), new cycle state.
__global__ __launch_bounds__(kT) void k_cycle_start(const double *r, int n, const double *P,
                                                    int G, double *V, float *v32, double *g,
                                                    int ldg, GState *gs, int cyc,
                                                    GState *mirror, Bat bt) {
    __shared__ double sb;
    r += sys() * bt.vec;
    P += sys() * bt.p;
    V += sys() * bt.v;
    if (v32) v32 += sys() * bt.v32;
    g += sys() * bt.rot;
    gs += sys();
    if (threadIdx.x < 64) {
        double v = (int)threadIdx.x < G ? P[threadIdx.x] : 0.0;
        v = wave_sum(v);
        if (threadIdx.x == 0) sb = sqrt(v);
    }
    __syncthreads();
    const double beta = sb;
    const double sc = beta > 0.0 ? 1.0 / beta : 0.0;
    int c0, c1;
    chunk_of(n, G, blockIdx.x, c0, c1);
    for (int i = c0 + threadIdx.x; i < c1; i += kT) {
        const double v = r[i] * sc;
        V[i] = v;
        if (v32) v32[i] = (float)v;
    }
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < ldg; i += kT) g[i] = (i == 0) ? beta : 0.0;
        if (threadIdx.x == 0) {
            gs->beta = beta;
            gs->resid = beta;
            gs->jdone = 0;
            gs->breakdown = 0;
            gs->active = (beta > gs->tol_abs) ? 1 : 0;
            if (!gs->active) publish(mirror, gs, cyc);
        }
    }
}

// P[i*G + b] = <V_i, w> over chunk b, i = 0..j.  Wave wv handles i = wv, wv+4, ...,
// four of them per pass so that their loads are in flight together; each sum
// keeps its own sequential order.
__device__ __forceinline__ void chunk_dots(const double *V, long ldv, const double *w, int c0,
                                           int c1, int j, double *P, int G) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int W = kT / 64;
    for (int i0 = wv; i0 <= j; i0 += 4 * W) {
        const double *vi[4];
        bool on[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            on[u] = i0 + u * W <= j;
            vi[u] = V + (long)(on[u] ? i0 + u * W : i0) * ldv;
        }
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int m = c0 + lane; m < c1; m += 64) {
            const double wm = w[m];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] += vi[u][m] * wm;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double t = wave_sum(a[u]);
            if (lane == 0 && on[u]) P[(long)(i0 + u * W) * G + blockIdx.x] = t;
        }
    }
}

// acc - sum_{i<=j} h_i V_i[m] in ascending i, sixteen loads in flight at a
// time (the last group predicated, its missing terms exact zeros)
__device__ __forceinline__ double minus_proj(double acc, const double *h, const double *V,
                                             long ldv, int m, int j) {
    for (int i = 0; i <= j; i += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = i + u <= j ? V[(long)(i + u) * ldv + m] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc -= (i + u <= j ? h[i + u] : 0.0) * v[u];
    }
    return acc;
}

// h_i = sum_b P[i*G + b] for i = 0..j into LDS: one wave per i, lanes over b
// (lane l sums b = l, l + 64, ... in order), four coefficients per wave with
// eight partials each in flight. A non-null Px is summed the same way as one
// more row, into h[j + 1], alongside the others.
__device__ __forceinline__ void reduce_coeffs(const double *P, int G, int j, double *h,
                                              const double *Px = nullptr) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int last = Px ? j + 1 : j;
    for (int i0 = wv; i0 <= last; i0 += 4 * (kT / 64)) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b0 = lane; b0 < G; b0 += 64 * 8) {
            double t[4][8];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * (kT / 64);
                const double *row = i > j ? (Px ? Px : P) : P + (long)i * G;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int b = b0 + 64 * k;
                    t[u][k] = (i <= last && b < G) ? row[b] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int k = 0; k < 8; ++k) v[u] += t[u][k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * (kT / 64);
            const double t = wave_sum(v[u]);
            if (lane == 0 && i <= last) h[i] = t;
        }
    }
}

// Row sums of the per-block partials of a fused Arnoldi product (one block
// per row): out[r] = sum_b P[r * GP + b] for the coefficient rows and, when
// Px is given, out[nrows - 1] = sum_b Px[b] (the squared norm).  Each row in
// one fixed order: thread t takes b = t, t + kT, ... (eight loads in flight),
// then the waves' butterflies and the wave sums in order.  Summed once here,
// the coefficients are then read by every block of the Gram-Schmidt kernel.
__global__ __launch_bounds__(kT) void k_reduce_rows(const double *P, int GP, const double *Px,
                                                    int nrows, double *out, const GState *gs) {
    if (gs->active == 0) return;
    __shared__ double sh[kT / 64];
    const int r = blockIdx.x;
    const double *row = (Px && r == nrows - 1) ? Px : P + (long)r * GP;
    double a = 0.0;
    for (int b0 = threadIdx.x; b0 < GP; b0 += 8 * kT) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = b0 + k * kT < GP ? row[b0 + k * kT] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) a += t[k];
    }
    a = block_sum(a, sh);
    if (threadIdx.x == 0) out[r] = a;
}

// Partial dots of w with V_0..V_j (P[i*G + b]) and the partial squared norm
// of w (P3[b]).
__global__ __launch_bounds__(kT) void k_cgs_dot(const double *V, long ldv, double *w, int n,
                                                int j, double *P, double *P3, int G,
                                                const GState *gs, Bat bt, const double *part,
                                                int ks, int nr) {
    const int s = sys();
    gs += s;
    if (gs->active == 0) return;
    V += s * bt.v;
    w += s * bt.vec;
    P += s * bt.p;
    P3 += s * bt.p;
    __shared__ double sh[kT / 64];
    int c0, c1;
    chunk_of(n, G, blockIdx.x, c0, c1);
    double nn = 0.0;
    if (part) {
        // w = the product's slices summed in order, on this block's chunk
        for (int m = c0 + threadIdx.x; m < c1; m += kT) {
            double a = 0.0;
            for (int k = 0; k < ks; ++k) a += part[((long)k * nr + s) * n + m];
            w[m] = a;
            nn += a * a;
        }
        __syncthreads();    // the chunk's w, written by this block, read below
    } else {
        for (int m = c0 + threadIdx.x; m < c1; m += kT) nn += w[m] * w[m];
    }
    nn = block_sum(nn, sh);
    if (threadIdx.x == 0) P3[blockIdx.x] = nn;
    chunk_dots(V, ldv, w, c0, c1, j, P, G);
}

// First Gram-Schmidt pass: h_i = sum_b P1[i][b] (every block, same order);
// w' = w - sum_i h_i V_i on the block's chunk; then the partial dots of w'
// with V (P2) and its partial squared norm (P3).  Block 0 stores h into
// column j of H.
__global__ __launch_bounds__(kT) void k_cgs_first(const double *V, long ldv, double *w, int n,
                                                  int j, const double *P1, double *P2,
                                                  double *P3, int G, int GP, double *H, int ldh,
                                                  const GState *gs, Bat bt, const double *hred) {
    gs += sys();
    if (gs->active == 0) return;
    V += sys() * bt.v;
    w += sys() * bt.vec;
    P1 += sys() * bt.p;
    P2 += sys() * bt.p;
    P3 += sys() * bt.p;
    H += sys() * bt.h;
    __shared__ double h[WWBI_MAX_RESTART + 1];
    __shared__ double sh[kT / 64];
    if (hred) {
        for (int i = threadIdx.x; i <= j; i += kT) h[i] = hred[i];
    } else {
        reduce_coeffs(P1, GP, j, h);
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i <= j; i += kT) H[(long)j * ldh + i] = h[i];
    int c0, c1;
    chunk_of(n, G, blockIdx.x, c0, c1);
    double nn = 0.0;
    for (int m = c0 + threadIdx.x; m < c1; m += kT) {
        const double acc = minus_proj(w[m], h, V, ldv, m, j);
        w[m] = acc;
        nn += acc * acc;
    }
    nn = block_sum(nn, sh);
    if (threadIdx.x == 0) P3[blockIdx.x] = nn;
    __syncthreads();
    chunk_dots(V, ldv, w, c0, c1, j, P2, G);
}

// Last Gram-Schmidt pass fused with the normalisation and the Givens step:
// h_i = sum_b P2[i][b]; w'' = w' - sum_i h_i V_i; ||w''||^2 = ||w'||^2 -
// ||h||^2 with ||w'||^2 from P3; V_{j+1} = w'' / ||w''|| in FP64 and FP32.
// After a first pass (add = 1) h is the re-orthogonalising correction, at
// rounding level, so the difference loses nothing; as the only pass (add = 0)
// the difference is exact to about eps (||w|| / ||w''||)^2, ample for the
// inner solves of the refinement, whose outer FP64 residual corrects them.
//
// Blocks 0..G-1 form V_{j+1} on their chunks.  Block G, beside them, adds h
// to (add = 1) or stores it into (add = 0) column j of H, applies the
// previous rotations, forms the new one and updates the residual estimate, so
// the serial rotation chain overlaps the vector update instead of following
// it.  V_{j+1} is written also by the step that ends the cycle (the recycled
// space of the refinement reads it).
//
// With kc > 0 recycled vectors C_0..C_{kc-1} sit in front of the Arnoldi
// basis (V_ points at C_0, the basis vector v_i at row kc + i): w is
// orthogonalised against all kc + j + 1 rows, the first kc coefficients go to
// column j of B (ld ldb) and only the rest into the Hessenberg column.
__global__ __launch_bounds__(kT) void k_cgs_final(const double *V_, long ldv, const double *w,
                                                  int n, int j, const double *P2,
                                                  const double *P3, int G, int GP, float *v32,
                                                  double *H, int ldh, int add, double *cs,
                                                  double *sn, double *g, int restart_len,
                                                  GState *gs, int cyc, GState *mirror,
                                                  Bat bt, int kc, double *B, int ldb,
                                                  const double *hred) {
    gs += sys();
    if (!step_runs(gs, j)) return;
    P2 += sys() * bt.p;
    P3 += sys() * bt.p;
    __shared__ double h[WWBI_MAX_RESTART + 1];
    __shared__ double sh[kT / 64];
    const int jj = kc + j;     // last row orthogonalised against
    // h[0..jj] from P2 and ||w'||^2 from P3 into h[jj + 1], in one pass (or
    // already summed into hred)
    if (hred) {
        for (int i = threadIdx.x; i <= jj + 1; i += kT) h[i] = hred[i];
    } else {
        reduce_coeffs(P2, GP, jj, h, P3);
    }
    __syncthreads();
    // ||h||^2 in one fixed order (the same in every block)
    double s2 = 0.0;
    for (int i = threadIdx.x; i <= jj; i += kT) s2 += h[i] * h[i];
    s2 = block_sum(s2, sh);
    const double q = h[jj + 1] - s2;
    const double nrm = q > 0.0 ? sqrt(q) : 0.0;
    if ((int)blockIdx.x < G) {
        double *V = const_cast<double *>(V_) + sys() * bt.v;
        w += sys() * bt.vec;
        if (v32) v32 += sys() * bt.v32;
        const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
        int c0, c1;
        chunk_of(n, G, blockIdx.x, c0, c1);
        double *vn = V + (long)(jj + 1) * ldv;
        for (int m = c0 + threadIdx.x; m < c1; m += kT) {
            const double v = minus_proj(w[m], h, V, ldv, m, jj) * sc;
            vn[m] = v;
            if (v32) v32[m] = (float)v;
        }
        return;
    }
    H += sys() * bt.h;
    cs += sys() * bt.rot;
    sn += sys() * bt.rot;
    g += sys() * bt.rot;
    __shared__ double col[WWBI_MAX_RESTART + 2], lc[WWBI_MAX_RESTART], ls[WWBI_MAX_RESTART];
    double *hc = H + (long)j * ldh;
    for (int i = threadIdx.x; i <= j; i += kT) col[i] = (add ? hc[i] : 0.0) + h[kc + i];
    for (int i = threadIdx.x; i < j; i += kT) { lc[i] = cs[i]; ls[i] = sn[i]; }
    if (kc > 0) {
        double *bc = B + (long)j * ldb;
        for (int i = threadIdx.x; i < kc; i += kT) bc[i] = (add ? bc[i] : 0.0) + h[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // rotation i mixes entries i and i + 1; the rotated entry i + 1 is
        // carried in a register into the next rotation
        double a = col[0];
        for (int i = 0; i < j; ++i) {
            const double b = col[i + 1];
            col[i] = lc[i] * a + ls[i] * b;
            a = -ls[i] * a + lc[i] * b;
        }
        const double b = nrm;
        const double r = hypot(a, b);
        double c = 1.0, s = 0.0;
        if (r > 0.0) { c = a / r; s = b / r; }
        cs[j] = c;
        sn[j] = s;
        col[j] = r;
        col[j + 1] = 0.0;
        const double gj = g[j];
        g[j] = c * gj;
        g[j + 1] = -s * gj;
        const double res = fabs(g[j + 1]);
        gs->resid = res;
        gs->its += 1;
        const bool brk = !(nrm > 0.0);           // exact invariant subspace, or NaN
        gs->breakdown = brk ? 1 : 0;
        const bool end = res <= gs->tol_abs || brk || j + 1 >= restart_len;
        store_step(gs, end ? 0 : 1, j + 1);
        if (end) publish(mirror, gs, cyc);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += kT) hc[i] = col[i];
}

// y = R^{-1} g for the k x k upper triangle (k = jdone), column-oriented.
__global__ __launch_bounds__(kT) void k_hsolve(const double *H, int ldh, const double *g,
                                               double *y, const GState *gs, Bat bt) {
    __shared__ double rhs[WWBI_MAX_RESTART + 1];
    H += sys() * bt.h;
    g += sys() * bt.rot;
    y += sys() * bt.rot;
    gs += sys();
    const int k = gs->jdone;
    for (int i = threadIdx.x; i < k; i += kT) rhs[i] = g[i];
    __syncthreads();
    for (int l = k - 1; l >= 0; --l) {
        const double rl = H[(long)l * ldh + l];
        const double yl = rl != 0.0 ? rhs[l] / rl : 0.0;
        __syncthreads();
        if (threadIdx.x == 0) y[l] = yl;
        for (int i = threadIdx.x; i < l; i += kT) rhs[i] -= H[(long)l * ldh + i] * yl;
        __syncthreads();
    }
}

// The same back substitution with the triangle staged first: the whole
// block copies columns 0..k-1 of R (rows 0..l of column l, at l (l + 1) / 2 + i
// of the dynamic LDS) in parallel, then one wave solves from LDS with no block
// barrier: one wave's LDS operations complete in issue order.
__global__ __launch_bounds__(kT) void k_hsolve_lds(const double *H, int ldh, const double *g,
                                                   double *y, const GState *gs, Bat bt) {
    extern __shared__ double tri[];
    __shared__ double sr[WWBI_MAX_RESTART + 1];
    H += sys() * bt.h;
    g += sys() * bt.rot;
    y += sys() * bt.rot;
    gs += sys();
    const int k = gs->jdone;
    const int nt = k * (k + 1) / 2;
    for (int e = threadIdx.x; e < nt; e += kT) {
        int l = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (l * (l + 1) / 2 > e) --l;
        while ((l + 1) * (l + 2) / 2 <= e) ++l;
        tri[e] = H[(long)l * ldh + (e - l * (l + 1) / 2)];
    }
    for (int i = threadIdx.x; i < k; i += kT) sr[i] = g[i];
    __syncthreads();
    if (threadIdx.x >= 64) return;
    for (int l = k - 1; l >= 0; --l) {
        const double *col = tri + l * (l + 1) / 2;
        const double rl = col[l];
        const double yl = rl != 0.0 ? sr[l] / rl : 0.0;
        if (threadIdx.x == 0) y[l] = yl;
        for (int i = threadIdx.x; i < l; i += 64) sr[i] -= col[i] * yl;
        // keep the compiler from reordering or forwarding LDS accesses across steps
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// x += sum_{i<k} y_i V_i (x = ... when overwrite is set)
__global__ void k_xupdate(double *x, const double *V, long ldv, int n, const double *y,
                          int overwrite, const GState *gs, Bat bt) {
    x += sys() * bt.vec;
    V += sys() * bt.v;
    y += sys() * bt.rot;
    gs += sys();
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int k = gs->jdone;
    double acc = overwrite ? 0.0 : x[m];
    int i = 0;
    for (; i + 8 <= k; i += 8) {          // eight loads in flight, ascending i
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = V[(long)(i + u) * ldv + m];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += y[i + u] * v[u];
    }
    for (; i < k; ++i) acc += y[i] * V[(long)i * ldv + m];
    x[m] = acc;
}

__global__ void k_axpy(double *x, const double *d, int n, double alpha) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) x[m] += alpha * d[m];
}
__global__ void k_copy(double *dst, const double *src, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) dst[m] = src[m];
}
__global__ void k_fill(double *dst, double v, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) dst[m] = v;
}
__global__ void k_to_f32(const double *src, float *dst, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) dst[m] = (float)src[m];
}

// ---------------------------------------------------------------------------
// Recycling of the first inner solve's Krylov space (GCRO-style deflation of
// the later inner solves of one refinement).  The first solve leaves the
// Arnoldi relation A V_k = V_{k+1} Hbar with Hbar = Q [R; 0], Q the product
// of its Givens rotations.  Then C = V_{k+1} Q[:, :k] has orthonormal columns
// and U = V_k R^{-1} satisfies A U = C (to the accuracy of the FP32
// products).  A later solve of A d = r projects r onto the complement of C,
// r0 = r - C (C^T r), runs Arnoldi on (I - C C^T) A, and returns
// d = V y + U (C^T r - B y), B = C^T A V the coefficients of C in its
// Gram-Schmidt; its least-squares problem and residual estimate are those
// of plain GMRES on r0.
// ---------------------------------------------------------------------------

// One thread per row m, one wave per block: the row's k + 1 basis values
// are staged in the thread's own column of LDS (sixteen loads in flight),
// then C_i[m] (the rotations applied along the row, carrying one value:
// O(k)) and U_i[m] (forward substitution through R's columns, in place over
// the staged values: O(k^2) LDS reads).  R and the rotations are uniform
// across the wave.
constexpr int kRecycleRows = 64;
__global__ __launch_bounds__(kRecycleRows) void k_recycle_build(const double *V, long ldv, int n,
                                                                int k, const double *H, int ldh,
                                                                const double *cs,
                                                                const double *sn, double *C,
                                                                double *U) {
    __shared__ double ws[kRecycleMax + 1][kRecycleRows];      // k <= kRecycleMax
    const int t = threadIdx.x;
    const int m = blockIdx.x * kRecycleRows + t;
    if (m >= n) return;                  // no barrier below: each thread keeps to its column
    for (int i0 = 0; i0 <= k; i0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = i0 + u <= k ? V[(long)(i0 + u) * ldv + m] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (i0 + u <= k) ws[i0 + u][t] = v[u];
    }
    double carry = ws[0][t];
    for (int i = 0; i < k; ++i) {
        const double nx = ws[i + 1][t];
        const double c = cs[i], s = sn[i];
        C[(long)i * ldv + m] = c * carry + s * nx;
        carry = -s * carry + c * nx;
    }
    for (int i = 0; i < k; ++i) {
        const double *rc = H + (long)i * ldh;      // column i of R
        double acc = ws[i][t];
        for (int l = 0; l < i; ++l) acc -= rc[l] * ws[l][t];
        acc /= rc[i];
        ws[i][t] = acc;
        U[(long)i * ldv + m] = acc;
    }
}

// Partial dots of r with C_0..C_{kc-1} (P[i*G + b]) and the partial squared
// norm of r (P3[b]); runs whatever the state of the previous solve.
__global__ __launch_bounds__(kT) void k_recycle_dots(const double *C, long ldv, const double *r,
                                                     int n, int kc, double *P, double *P3,
                                                     int G) {
    __shared__ double sh[kT / 64];
    int c0, c1;
    chunk_of(n, G, blockIdx.x, c0, c1);
    double nn = 0.0;
    for (int m = c0 + threadIdx.x; m < c1; m += kT) nn += r[m] * r[m];
    nn = block_sum(nn, sh);
    if (threadIdx.x == 0) P3[blockIdx.x] = nn;
    chunk_dots(C, ldv, r, c0, c1, kc - 1, P, G);
}

// h = C^T r (summed from P, every block in the same order; block 0 keeps it
// in z), r0 = r - C h and the partial squared norms of r0 (P3).
__global__ __launch_bounds__(kT) void k_recycle_project(const double *C, long ldv,
                                                        const double *r, int n, int kc,
                                                        const double *P, double *P3, int G,
                                                        double *r0, double *z) {
    __shared__ double h[WWBI_MAX_RESTART + 1];
    __shared__ double sh[kT / 64];
    reduce_coeffs(P, G, kc - 1, h);
    __syncthreads();
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < kc; i += kT) z[i] = h[i];
    int c0, c1;
    chunk_of(n, G, blockIdx.x, c0, c1);
    double nn = 0.0;
    for (int m = c0 + threadIdx.x; m < c1; m += kT) {
        const double v = minus_proj(r[m], h, C, ldv, m, kc - 1);
        r0[m] = v;
        nn += v * v;
    }
    nn = block_sum(nn, sh);
    if (threadIdx.x == 0) P3[blockIdx.x] = nn;
}

// z <- z - B y over the jdone solved columns (one block, a thread per row of
// B, columns in ascending order).
__global__ void k_recycle_coef(double *z, const double *B, int ldb, const double *y, int kc,
                               const GState *gs) {
    const int k = gs->jdone;
    for (int i = threadIdx.x; i < kc; i += blockDim.x) {
        double acc = z[i];
        for (int j = 0; j < k; ++j) acc -= B[(long)j * ldb + i] * y[j];
        z[i] = acc;
    }
}

// x = sum_{i<jdone} y_i V_i + sum_{i<kc} z_i U_i
__global__ void k_xupdate_recycled(double *x, const double *V, long ldv, int n, const double *y,
                                   const double *U, const double *z, int kc,
                                   const GState *gs) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int k = gs->jdone;
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += y[i] * V[(long)i * ldv + m];
    for (int i = 0; i < kc; ++i) acc += z[i] * U[(long)i * ldv + m];
    x[m] = acc;
}

}  // namespace

int gmres_nblocks(int n) {
    const int g = cdiv(n, kT);
    return g > kMaxG ? kMaxG : (g < 1 ? 1 : g);
}

void launch_norm_partial(const double *v, int n, double *P, int G, hipStream_t st,
                         const Bat &bt) {
    hipLaunchKernelGGL(k_norm_partial, dim3(G, bt.nsys), dim3(kT), 0, st, v, n, P, G, bt);
}
void launch_set_tol(const double *P, int G, double tol, GState *gs, hipStream_t st,
                    const Bat &bt) {
    hipLaunchKernelGGL(k_set_tol, dim3(1, bt.nsys), dim3(64), 0, st, P, G, tol, gs, bt);
}
void launch_cycle_start(const double *r, int n, const double *P, int G, double *V, float *v32,
                        double *g, int ldg, GState *gs, int cyc, GState *mirror,
                        hipStream_t st, const Bat &bt) {
    hipLaunchKernelGGL(k_cycle_start, dim3(G, bt.nsys), dim3(kT), 0, st, r, n, P, G, V, v32, g,
                       ldg, gs, cyc, mirror, bt);
}
void launch_cgs_dot(const double *V, long ldv, double *w, int n, int j, double *P,
                    double *P3, int G, const GState *gs, hipStream_t st, const Bat &bt,
                    const double *part, int ks, int nr) {
    hipLaunchKernelGGL(k_cgs_dot, dim3(G, bt.nsys), dim3(kT), 0, st, V, ldv, w, n, j, P, P3, G,
                       gs, bt, part, ks, nr);
}
void launch_cgs_first(const double *V, long ldv, double *w, int n, int j, const double *P1,
                      double *P2, double *P3, int G, double *H, int ldh, const GState *gs,
                      hipStream_t st, const Bat &bt, int GP, const double *hred) {
    hipLaunchKernelGGL(k_cgs_first, dim3(G, bt.nsys), dim3(kT), 0, st, V, ldv, w, n, j, P1, P2,
                       P3, G, GP > 0 ? GP : G, H, ldh, gs, bt, hred);
}
void launch_reduce_rows(const double *P, int GP, const double *Px, int nrows, double *out,
                        const GState *gs, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_rows, dim3(nrows), dim3(kT), 0, st, P, GP, Px, nrows, out, gs);
}
void launch_cgs_final(const double *V, long ldv, const double *w, int n, int j,
                      const double *P2, const double *P3, int G, float *v32, double *H, int ldh,
                      bool add, double *cs, double *sn, double *g, int restart_len, GState *gs,
                      int cyc, GState *mirror, hipStream_t st, const Bat &bt, int GP, int kc,
                      double *B, int ldb, const double *hred) {
    // G vector blocks and one Hessenberg block
    hipLaunchKernelGGL(k_cgs_final, dim3(G + 1, bt.nsys), dim3(kT), 0, st, V, ldv, w, n, j, P2,
                       P3, G,
                       GP > 0 ? GP : G, v32, H, ldh, add ? 1 : 0, cs, sn, g, restart_len, gs,
                       cyc, mirror, bt, kc, B, ldb, hred);
}
void launch_recycle_build(const double *V, long ldv, int n, int k, const double *H, int ldh,
                          const double *cs, const double *sn, double *C, double *U,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_recycle_build, dim3(cdiv(n, kRecycleRows)), dim3(kRecycleRows), 0, st, V,
                       ldv, n, k, H, ldh, cs, sn, C, U);
}
void launch_recycle_dots(const double *C, long ldv, const double *r, int n, int kc, double *P,
                         double *P3, int G, hipStream_t st) {
    hipLaunchKernelGGL(k_recycle_dots, dim3(G), dim3(kT), 0, st, C, ldv, r, n, kc, P, P3, G);
}
void launch_recycle_project(const double *C, long ldv, const double *r, int n, int kc,
                            const double *P, double *P3, int G, double *r0, double *z,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_recycle_project, dim3(G), dim3(kT), 0, st, C, ldv, r, n, kc, P, P3, G,
                       r0, z);
}
void launch_recycle_coef(double *z, const double *B, int ldb, const double *y, int kc,
                         const GState *gs, hipStream_t st) {
    hipLaunchKernelGGL(k_recycle_coef, dim3(1), dim3(64), 0, st, z, B, ldb, y, kc, gs);
}
void launch_xupdate_recycled(double *x, const double *V, long ldv, int n, const double *y,
                             const double *U, const double *z, int kc, const GState *gs,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_xupdate_recycled, dim3(cdiv(n, 256)), dim3(256), 0, st, x, V, ldv, n, y,
                       U, z, kc, gs);
}
void launch_hsolve(const double *H, int ldh, const double *g, double *y, const GState *gs,
                   hipStream_t st, const Bat &bt) {
    // the staged form while the triangle of the largest k (ldh - 1) fits the default
    // 64 KB launch limit beside the static right-hand side
    const size_t tri = (size_t)ldh * (ldh - 1) / 2 * sizeof(double);
    if (tri <= 60 * 1024)
        hipLaunchKernelGGL(k_hsolve_lds, dim3(1, bt.nsys), dim3(kT), tri, st, H, ldh, g, y, gs,
                           bt);
    else
        hipLaunchKernelGGL(k_hsolve, dim3(1, bt.nsys), dim3(kT), 0, st, H, ldh, g, y, gs, bt);
}
void launch_xupdate(double *x, const double *V, long ldv, int n, const double *y,
                    bool overwrite, const GState *gs, hipStream_t st, const Bat &bt) {
    hipLaunchKernelGGL(k_xupdate, dim3(cdiv(n, 256), bt.nsys), dim3(256), 0, st, x, V, ldv, n, y,
                       overwrite ? 1 : 0, gs, bt);
}
void launch_axpy(double *x, const double *d, int n, double alpha, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy, dim3(cdiv(n, 256)), dim3(256), 0, st, x, d, n, alpha);
}
void launch_copy(double *dst, const double *src, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy, dim3(cdiv(n, 256)), dim3(256), 0, st, dst, src, n);
}
void launch_fill(double *dst, double v, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(cdiv(n, 256)), dim3(256), 0, st, dst, v, n);
}
void launch_to_f32(const double *src, float *dst, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_to_f32, dim3(cdiv(n, 256)), dim3(256), 0, st, src, dst, n);
}

}  // namespace wwbi
