// Fixed-order reduction of the partial slices that the split products
// (on-the-fly chunks, near band) write: y = c - scale * sum_k part[k], or
// y = scale * sum_k part[k] when c is null.  Skipped when `active` (device
// flag, may be null) points to 0.
#include "internal.h"

namespace wwbi {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// 64 outputs per block, kSliceWaves waves sharing their slices.
__global__ __launch_bounds__(64 * kSliceWaves) void k_reduce_partials(
    int n, const double *__restrict__ part, int nsplit, const double *__restrict__ c,
    double scale, double *__restrict__ y, const int *active) {
    if (active && *active == 0) return;
    __shared__ double red[kSliceWaves][64];
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    double s = sum_slices_waves<kSliceWaves>(part, nsplit, n, i, i < n, red);
    if (threadIdx.x >= 64 || i >= n) return;
    s *= scale;
    y[i] = c ? c[i] - s : s;
}

}  // namespace

void launch_reduce_partials(int n, const double *part, int nsplit, const double *c, double scale,
                            double *y, const int *active, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(cdiv(n, 64)), dim3(64 * kSliceWaves), 0, st, n, part,
                       nsplit, c, scale, y, active);
}

}  // namespace wwbi
