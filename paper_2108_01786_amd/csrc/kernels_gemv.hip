// Product with a stored matrix, y = c - A x (one wave per row pair), for
// FP64 and FP32 matrices: the dominant kernel of every solve.
//
// Stored matrices are row-major with a leading dimension padded to a multiple
// of 64 elements; padding columns hold zeros.  Every product that can be
// skipped after GMRES convergence takes `active` (device flag, may be null).
#include "internal.h"

namespace wwbi {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

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

}  // namespace

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


}  // namespace wwbi
