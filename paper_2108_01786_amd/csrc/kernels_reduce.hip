// Fixed-order reduction of the partial slices that the split products
// (on-the-fly chunks, near band) write: y = c - scale * sum_k part[k], or
// y = scale * sum_k part[k] when c is null.  Skipped when `active` (device
// flag, may be null) points to 0.
#include "internal.h"

namespace wwbi {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

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

}  // namespace wwbi
