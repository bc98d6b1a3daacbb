// Assembly of the collocated operators and the products with them.
//
// Stored matrices are row-major with a leading dimension padded to a multiple
// of 64 elements; padding columns hold zeros.  Every product that can be
// skipped after GMRES convergence takes `active` (device flag, may be null).
#include "entries.h"
#include "internal.h"

namespace wwbi {

namespace {

constexpr int kRowsPerAsmBlock = 32;

// ---------------------------------------------------------------------------
// assembly: one thread per column (coalesced row writes), a tile of rows per
// block with the target data staged in LDS (read as broadcasts).
// ---------------------------------------------------------------------------
template <bool FP32, bool WALL>
__global__ __launch_bounds__(256) void k_assemble(Nodes N, const double *hrow, int r0, int nr,
                                                  int c0, int nc, int corr, int band, void *out,
                                                  long ld) {
    __shared__ Tgt tg[kRowsPerAsmBlock];
    const int col = blockIdx.x * 256 + threadIdx.x;           // column within the output
    const int rbase = blockIdx.y * kRowsPerAsmBlock;
    if (threadIdx.x < kRowsPerAsmBlock) {
        const int r = rbase + threadIdx.x;
        if (r < nr) tg[threadIdx.x] = load_tgt(N, r0 + r);
    }
    __syncthreads();
    if (col >= ld) return;
    const bool live = col < nc;
    Src s;
    if (live) s = load_src(N, c0 + col);
    const int rend = min(kRowsPerAsmBlock, nr - rbase);
    for (int i = 0; i < rend; ++i) {
        const long idx = (long)(rbase + i) * ld + col;
        if (WALL) {
            double v = 0.0;
            if (live) {
                v = t_val64(N, tg[i], s, hrow);
                if (tg[i].k == s.k && tg[i].loc == s.loc) v -= 0.5;
            }
            __builtin_nontemporal_store(v, static_cast<double *>(out) + idx);
        } else if (FP32) {
            __builtin_nontemporal_store(live ? a_val32(N, tg[i], s, corr != 0, band) : 0.0f,
                                        static_cast<float *>(out) + idx);
        } else {
            __builtin_nontemporal_store(live ? a_val64(N, tg[i], s, corr != 0) : 0.0,
                                        static_cast<double *>(out) + idx);
        }
    }
}

// ---------------------------------------------------------------------------
// stored product y = c - A x (or y = A x): one wave per R rows, 16-byte loads
// along the row, x converted to the accumulation type, wave-level reduction.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// 16-byte vectors of the matrix element type, read with a non-temporal hint:
// the matrix is streamed once per product, and without the hint the stream
// reaches only about half the HBM bandwidth (measured on MI355X).
template <typename TA> struct Vec16;
template <> struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <> struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};

template <typename TA>
__device__ __forceinline__ typename Vec16<TA>::type stream_load(const TA *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const typename Vec16<TA>::type *>(p));
}

template <typename TACC, typename TX, int VW>
__device__ __forceinline__ void load_x(const TX *x, int col, TACC (&xv)[VW]) {
#pragma unroll
    for (int v = 0; v < VW; ++v) xv[v] = (TACC)x[col + v];
}

// y = c - A x (or A x): each wave owns R rows and walks them in steps of
// 64 lanes x 16 bytes, U steps in flight; FP32 matrices accumulate in FP32.
template <typename TA, typename TX, typename TACC, int R, int U>
__global__ __launch_bounds__(256) void k_gemv(const TA *__restrict__ A, long ld, int n,
                                              const TX *__restrict__ x,
                                              const double *__restrict__ c,
                                              double *__restrict__ y, const int *active) {
    if (active && *active == 0) return;
    using V = typename Vec16<TA>::type;
    constexpr int VW = Vec16<TA>::n;
    constexpr int STEP = 64 * VW;
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const long r0 = wave * R;
    if (r0 >= n) return;
    const TA *rowp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rowp[r] = A + (r0 + r < n ? r0 + r : n - 1) * ld;
    TACC acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = (TACC)0;
    const int nbig = (n / (STEP * U)) * (STEP * U);
    for (int c0 = 0; c0 < nbig; c0 += STEP * U) {
        V a[U][R];
        TACC xv[U][VW];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int col = c0 + u * STEP + lane * VW;
#pragma unroll
            for (int r = 0; r < R; ++r) a[u][r] = stream_load(rowp[r] + col);
            load_x<TACC, TX, VW>(x, col, xv[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int v = 0; v < VW; ++v) acc[r] += (TACC)a[u][r][v] * xv[u][v];
    }
    const int nstep = (n / STEP) * STEP;
    for (int c0 = nbig; c0 < nstep; c0 += STEP) {
        const int col = c0 + lane * VW;
        TACC xv[VW];
        load_x<TACC, TX, VW>(x, col, xv);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const V a = stream_load(rowp[r] + col);
#pragma unroll
            for (int v = 0; v < VW; ++v) acc[r] += (TACC)a[v] * xv[v];
        }
    }
    for (int col = nstep + lane; col < n; col += 64) {
        const TACC xv = (TACC)x[col];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += (TACC)rowp[r][col] * xv;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const TACC s = wave_sum(acc[r]);
        if (lane == 0 && r0 + r < n) {
            const double v = (double)s;
            y[r0 + r] = c ? c[r0 + r] - v : v;
        }
    }
}

// transpose product, split over row chunks: part[s][q] = sum_{p in chunk s} A[p][q] x[p]
template <typename TA, typename TACC>
__global__ __launch_bounds__(256) void k_gemvT(const TA *__restrict__ A, long ld, int n,
                                               const double *__restrict__ x,
                                               double *__restrict__ part, int rows_per,
                                               const int *active) {
    if (active && *active == 0) return;
    using V = typename Vec16<TA>::type;
    constexpr int VW = Vec16<TA>::n;
    const int col = (blockIdx.x * 256 + threadIdx.x) * VW;
    const int p0 = blockIdx.y * rows_per;
    const int p1 = min(n, p0 + rows_per);
    if (col >= n) return;
    TACC acc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[v] = (TACC)0;
    for (int p = p0; p < p1; ++p) {
        const TACC xp = (TACC)x[p];
        const V a = stream_load(A + (long)p * ld + col);
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] += (TACC)a[v] * xp;
    }
    double *out = part + (long)blockIdx.y * n;
#pragma unroll
    for (int v = 0; v < VW; ++v)
        if (col + v < n) out[col + v] = (double)acc[v];
}

__global__ void k_reduce_partials(int n, const double *__restrict__ part, int nsplit,
                                  const double *__restrict__ c, double scale,
                                  double *__restrict__ y, const int *active) {
    if (active && *active == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(long)k * n + i];
    s *= scale;
    y[i] = c ? c[i] - s : s;
}

// ---------------------------------------------------------------------------
// on-the-fly products: entries recomputed in registers, never stored.
// Forward: one thread per target row, a chunk of sources per grid.y staged in
// LDS.  Transpose: one thread per source column, a chunk of targets staged.
// Mode selects the entry: 0 = A in FP64, 1 = A in FP32 (with FP64 band),
// 2 = target-flavour T, 3 = target-flavour wall operator (T - I/2).
// ---------------------------------------------------------------------------
constexpr int kStage = 256;

template <int MODE>
__device__ __forceinline__ double entry(const Nodes &N, const Tgt &t, const Src &s, bool corr,
                                        int band, const double *hrow) {
    if (MODE == 0) return a_val64(N, t, s, corr);
    if (MODE == 1) return (double)a_val32(N, t, s, corr, band);
    double v = t_val64(N, t, s, hrow);
    if (MODE == 3 && t.k == s.k && t.loc == s.loc) v -= 0.5;
    return v;
}

// Forward product: each thread owns kTPT target rows (rows t, t + 256, ... of
// the block's 256 * kTPT), so every source staged in LDS is read once for
// kTPT entries.
constexpr int kTPT = 2;

template <int MODE, bool ACC32>
__global__ __launch_bounds__(256) void k_otf_rows(Nodes N, const double *hrow, int r0, int nr,
                                                  int c0, int nc,
                                                  int chunk, int corr, int band,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ part,
                                                  const int *active) {
    if (active && *active == 0) return;
    __shared__ Src ss[kStage];
    __shared__ double sx[kStage];
    Tgt t[kTPT];
    bool live[kTPT];
#pragma unroll
    for (int u = 0; u < kTPT; ++u) {
        const int r = blockIdx.x * 256 * kTPT + u * 256 + threadIdx.x;
        live[u] = r < nr;
        t[u] = load_tgt(N, r0 + (live[u] ? r : 0));
    }
    const int cb = blockIdx.y * chunk;
    const int ce = min(nc, cb + chunk);
    double acc[kTPT];
    float acc32[kTPT];
#pragma unroll
    for (int u = 0; u < kTPT; ++u) { acc[u] = 0.0; acc32[u] = 0.0f; }
    for (int cc = cb; cc < ce; cc += kStage) {
        const int q = cc + threadIdx.x;
        if (q < ce) {
            ss[threadIdx.x] = load_src(N, c0 + q);
            sx[threadIdx.x] = x[q];
        }
        __syncthreads();
        const int m = min(kStage, ce - cc);
        for (int i = 0; i < m; ++i) {
            const Src s = ss[i];
            const double xv = sx[i];
#pragma unroll
            for (int u = 0; u < kTPT; ++u) {
                if (ACC32)
                    acc32[u] += (float)entry<MODE>(N, t[u], s, corr != 0, band, hrow) * (float)xv;
                else
                    acc[u] += entry<MODE>(N, t[u], s, corr != 0, band, hrow) * xv;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kTPT; ++u) {
        const int r = blockIdx.x * 256 * kTPT + u * 256 + threadIdx.x;
        if (live[u]) part[(long)blockIdx.y * nr + r] = ACC32 ? (double)acc32[u] : acc[u];
    }
}

template <int MODE, bool ACC32>
__global__ __launch_bounds__(256) void k_otf_cols(Nodes N, const double *hrow, int r0, int nr,
                                                  int c0, int nc,
                                                  int chunk, int corr, int band,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ part,
                                                  const int *active) {
    if (active && *active == 0) return;
    __shared__ Tgt ts[kStage];
    __shared__ double sx[kStage];
    const int q = blockIdx.x * 256 + threadIdx.x;
    const bool live = q < nc;
    Src s;
    if (live) s = load_src(N, c0 + q);
    const int pb = blockIdx.y * chunk;
    const int pe = min(nr, pb + chunk);
    double acc = 0.0;
    float acc32 = 0.0f;
    for (int pp = pb; pp < pe; pp += kStage) {
        const int p = pp + threadIdx.x;
        if (p < pe) {
            ts[threadIdx.x] = load_tgt(N, r0 + p);
            sx[threadIdx.x] = x[p];
        }
        __syncthreads();
        const int m = min(kStage, pe - pp);
        if (live) {
            for (int i = 0; i < m; ++i) {
                if (ACC32)
                    acc32 += (float)entry<MODE>(N, ts[i], s, corr != 0, band, hrow) * (float)sx[i];
                else
                    acc += entry<MODE>(N, ts[i], s, corr != 0, band, hrow) * sx[i];
            }
        }
        __syncthreads();
    }
    if (live) part[(long)blockIdx.y * nc + q] = ACC32 ? (double)acc32 : acc;
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

int otf_chunk(int n) {
    int c = cdiv(n, 64);
    c = cdiv(c, kStage) * kStage;
    return c < kStage ? kStage : c;
}
int otf_nsplit(int n) { return cdiv(n, otf_chunk(n)); }

void launch_assemble64(const Layout &L, const Nodes &N, int flags, double *A, long ld,
                       hipStream_t st) {
    const double *hrow = nullptr;
    const int n = L.n;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsmBlock));
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    hipLaunchKernelGGL((k_assemble<false, false>), grid, dim3(256), 0, st, N, hrow, 0, n, 0, n, corr, 0,
                       (void *)A, ld);
}

void launch_assemble32(const Layout &L, const Nodes &N, int flags, int band, float *A, long ld,
                       hipStream_t st) {
    const double *hrow = nullptr;
    const int n = L.n;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsmBlock));
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    hipLaunchKernelGGL((k_assemble<true, false>), grid, dim3(256), 0, st, N, hrow, 0, n, 0, n, corr,
                       band, (void *)A, ld);
}

void launch_assemble_wall64(const Layout &L, const Nodes &N, const double *hrow, double *W, long ld,
                            hipStream_t st) {
    const int c0 = L.off[1], nw = L.n - L.off[1];
    dim3 grid(cdiv(ld, 256), cdiv(nw, kRowsPerAsmBlock));
    hipLaunchKernelGGL((k_assemble<false, true>), grid, dim3(256), 0, st, N, hrow, c0, nw, c0, nw, 1, 0,
                       (void *)W, ld);
}

static int gemv_blocks(int n, int R) { return cdiv(cdiv(n, R), 4); }

constexpr int kGemvR = 2;   // rows per wave
constexpr int kGemvU = 4;   // 16-byte steps in flight per row

void launch_gemv64(const double *A, long ld, int n, const double *x, const double *c, double *y,
                   const int *active, hipStream_t st) {
    hipLaunchKernelGGL((k_gemv<double, double, double, kGemvR, kGemvU>),
                       dim3(gemv_blocks(n, kGemvR)), dim3(256), 0, st, A, ld, n, x, c, y, active);
}

void launch_gemv32(const float *A, long ld, int n, const float *x, const double *c, double *y,
                   const int *active, hipStream_t st) {
    hipLaunchKernelGGL((k_gemv<float, float, float, kGemvR, kGemvU>),
                       dim3(gemv_blocks(n, kGemvR)), dim3(256), 0, st, A, ld, n, x, c, y, active);
}

void launch_gemv32_x64(const float *A, long ld, int n, const double *x, const double *c,
                       double *y, const int *active, hipStream_t st) {
    hipLaunchKernelGGL((k_gemv<float, double, float, kGemvR, kGemvU>),
                       dim3(gemv_blocks(n, kGemvR)), dim3(256), 0, st, A, ld, n, x, c, y, active);
}

void launch_reduce_partials(int n, const double *part, int nsplit, const double *c, double scale,
                            double *y, const int *active, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(cdiv(n, 256)), dim3(256), 0, st, n, part, nsplit, c,
                       scale, y, active);
}

int gemvT_nsplit(int n) { return cdiv(n, 160) > 64 ? 64 : cdiv(n, 160); }

void launch_gemvT64(const double *A, long ld, int n, const double *x, const double *c, double *y,
                    double *part, const int *active, hipStream_t st) {
    const int ns = gemvT_nsplit(n);
    const int rows_per = cdiv(n, ns);
    dim3 grid(cdiv(n, 256 * 2), ns);
    hipLaunchKernelGGL((k_gemvT<double, double>), grid, dim3(256), 0, st, A, ld, n, x, part,
                       rows_per, active);
    launch_reduce_partials(n, part, ns, c, 1.0, y, active, st);
}

void launch_gemvT32(const float *A, long ld, int n, const double *x, const double *c, double *y,
                    double *part, const int *active, hipStream_t st) {
    const int ns = gemvT_nsplit(n);
    const int rows_per = cdiv(n, ns);
    dim3 grid(cdiv(n, 256 * 4), ns);
    hipLaunchKernelGGL((k_gemvT<float, float>), grid, dim3(256), 0, st, A, ld, n, x, part,
                       rows_per, active);
    launch_reduce_partials(n, part, ns, c, 1.0, y, active, st);
}

void launch_otf_matvec(const Layout &L, const Nodes &N, int flags, int fp32, int band,
                       int transpose, const double *x, const double *c, double *y, double *part,
                       const int *active, hipStream_t st) {
    const double *hrow = nullptr;
    const int n = L.n;
    const int chunk = otf_chunk(n);
    const int ns = cdiv(n, chunk);
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    dim3 grid(cdiv(n, 256), ns);
    dim3 gridr(cdiv(n, 256 * kTPT), ns);
    if (!transpose) {
        if (fp32)
            hipLaunchKernelGGL((k_otf_rows<1, true>), gridr, dim3(256), 0, st, N, hrow, 0, n, 0, n,
                               chunk, corr, band, x, part, active);
        else
            hipLaunchKernelGGL((k_otf_rows<0, false>), gridr, dim3(256), 0, st, N, hrow, 0, n, 0, n,
                               chunk, corr, band, x, part, active);
    } else {
        if (fp32)
            hipLaunchKernelGGL((k_otf_cols<1, true>), grid, dim3(256), 0, st, N, hrow, 0, n, 0, n, chunk,
                               corr, band, x, part, active);
        else
            hipLaunchKernelGGL((k_otf_cols<0, false>), grid, dim3(256), 0, st, N, hrow, 0, n, 0, n,
                               chunk, corr, band, x, part, active);
    }
    launch_reduce_partials(n, part, ns, c, 1.0, y, active, st);
}

int rflavour_nsplit(int nc) { return cdiv(nc, otf_chunk(nc)); }

void launch_rflavour(const Layout &L, const Nodes &N, const double *hrow, int mode, int transpose,
                     int r0, int nr, int c0, int nc, const double *x, double *part,
                     const int *active, hipStream_t st) {
    (void)L;
    if (!transpose) {
        const int chunk = otf_chunk(nc);
        dim3 grid(cdiv(nr, 256 * kTPT), cdiv(nc, chunk));
        if (mode == 3)
            hipLaunchKernelGGL((k_otf_rows<3, false>), grid, dim3(256), 0, st, N, hrow, r0, nr, c0, nc,
                               chunk, 1, 0, x, part, active);
        else
            hipLaunchKernelGGL((k_otf_rows<2, false>), grid, dim3(256), 0, st, N, hrow, r0, nr, c0, nc,
                               chunk, 1, 0, x, part, active);
    } else {
        const int chunk = otf_chunk(nr);
        dim3 grid(cdiv(nc, 256), cdiv(nr, chunk));
        if (mode == 3)
            hipLaunchKernelGGL((k_otf_cols<3, false>), grid, dim3(256), 0, st, N, hrow, r0, nr, c0, nc,
                               chunk, 1, 0, x, part, active);
        else
            hipLaunchKernelGGL((k_otf_cols<2, false>), grid, dim3(256), 0, st, N, hrow, r0, nr, c0, nc,
                               chunk, 1, 0, x, part, active);
    }
}

}  // namespace wwbi
