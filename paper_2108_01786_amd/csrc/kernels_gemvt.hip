// Transpose product with a stored matrix (the adjoint's A^T x), split over
// row chunks, and the fixed-order reduction of split partial sums.
//
// Stored matrices are row-major with a leading dimension padded to a multiple
// of 64 elements; padding columns hold zeros.  Every product that can be
// skipped after GMRES convergence takes `active` (device flag, may be null).
#include "internal.h"

namespace wwbi {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// 16-byte vectors of the matrix element type, read with a non-temporal hint.
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

constexpr int kRowsInFlight = 8;

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
    // kRowsInFlight rows' loads are issued before their products; the sum
    // still runs over p in increasing order
    int p = p0;
    for (; p + kRowsInFlight <= p1; p += kRowsInFlight) {
        V a[kRowsInFlight];
        TACC xs[kRowsInFlight];
#pragma unroll
        for (int u = 0; u < kRowsInFlight; ++u) {
            a[u] = stream_load(A + (long)(p + u) * ld + col);
            xs[u] = (TACC)x[p + u];
        }
#pragma unroll
        for (int u = 0; u < kRowsInFlight; ++u)
#pragma unroll
            for (int v = 0; v < VW; ++v) acc[v] += (TACC)a[u][v] * xs[u];
    }
    for (; p < p1; ++p) {
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
    double s = sum_slices(part, nsplit, n, i);
    s *= scale;
    y[i] = c ? c[i] - s : s;
}

}  // namespace

void launch_reduce_partials(int n, const double *part, int nsplit, const double *c, double scale,
                            double *y, const int *active, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(cdiv(n, 64)), dim3(64), 0, st, n, part, nsplit, c,
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

}  // namespace wwbi
