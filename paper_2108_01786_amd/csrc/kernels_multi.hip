// One pass over the stored matrix for several right-hand sides:
//   Y_s = A X_s,  s < nr,
// on the matrix cores (v_mfma_f64_16x16x4_f64 for an FP64 matrix,
// v_mfma_f32_16x16x4_f32 for FP32).  A wave owns 16 rows and up to 32
// systems (two 16x16 accumulators); K is split over grid.y and the partial
// products are reduced in a fixed order.
//
// Operand mapping of one 16x16x4 step: lane l supplies A(i, k) with
// i = l % 16, k = l / 16 and B(k, j) with j = l % 16, k = l / 16.  The result
// D(i, j) sits in lane l with j = l % 16 and element r, where the row is
// i = 4 (l / 16) + r for the FP32 instruction and i = l / 16 + 4 r for the
// FP64 one (checked on the device).  The four k indices of a step are
// relabelled so that every lane reads four consecutive columns: step t of a
// 16-column tile uses columns k0 + 4 (l / 16) + t.
#include "internal.h"

namespace wwbi {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    using acc = v4d;
    static __device__ __forceinline__ int row(int q, int r) { return q + 4 * r; }
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<float> {
    using acc = v4f;
    static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// four consecutive elements p[0..3] of a row, zero past `end`; the matrix is
// streamed with a non-temporal hint
template <typename T>
__device__ __forceinline__ void load4(const T *p, int k, int end, T (&v)[4], bool stream) {
    if (k + 3 < end) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
            v[t] = stream ? __builtin_nontemporal_load(p + k + t) : p[k + t];
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = (k + t < end) ? p[k + t] : (T)0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mfma_multi(const T *__restrict__ A, long ld, int n,
                                                    const T *__restrict__ X, long xs, int nr,
                                                    int kchunk, double *__restrict__ part) {
    using M = Mfma<T>;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row0 = (blockIdx.x * 4 + wv) * 16;
    if (row0 >= n) return;
    const int kb = blockIdx.y * kchunk;
    const int ke = min(n, kb + kchunk);
    const int i = lane & 15, q = lane >> 4;
    const int row = row0 + i;
    const bool rok = row < n;
    const T *arow = A + (long)(rok ? row : 0) * ld;
    const bool two = nr > 16;
    const int s0 = i, s1 = 16 + i;
    const T *x0 = X + (long)(s0 < nr ? s0 : 0) * xs;
    const T *x1 = X + (long)(s1 < nr ? s1 : 0) * xs;
    typename M::acc c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        const int kk = k0 + 4 * q;
        T a[4], b[4];
        load4(arow, kk, rok ? ke : kk, a, true);
        load4(x0, kk, s0 < nr ? ke : kk, b, false);
#pragma unroll
        for (int t = 0; t < 4; ++t) c0 = M::step(a[t], b[t], c0);
        if (two) {
            load4(x1, kk, s1 < nr ? ke : kk, b, false);
#pragma unroll
            for (int t = 0; t < 4; ++t) c1 = M::step(a[t], b[t], c1);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rr = row0 + M::row(q, r);
        if (rr < n) {
            if (s0 < nr) part[((long)blockIdx.y * nr + s0) * n + rr] = (double)c0[r];
            if (two && s1 < nr) part[((long)blockIdx.y * nr + s1) * n + rr] = (double)c1[r];
        }
    }
}

// y_s = c_s - sum_k part[k][s] (or the plain sum when c is null)
__global__ void k_reduce_multi(int n, int nr, const double *__restrict__ part, int ks,
                               const double *__restrict__ c, long cs, double *__restrict__ y,
                               long ys) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (m >= n || s >= nr) return;
    double acc = 0.0;
    for (int k = 0; k < ks; ++k) acc += part[((long)k * nr + s) * n + m];
    y[(long)s * ys + m] = c ? c[(long)s * cs + m] - acc : acc;
}

__global__ void k_copy_strided(const double *src, long ss, double *dst, long ds, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const long s = blockIdx.y;
    if (m < n) dst[s * ds + m] = src[s * ss + m];
}

__global__ void k_to_f32_batched(const double *src, long ss, float *dst, long ds, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const long s = blockIdx.y;
    if (m < n) dst[s * ds + m] = (float)src[s * ss + m];
}

}  // namespace

int multi_ksplit(int n) {
    // about 16 waves of K per row tile; K chunks a multiple of 16 columns
    int ks = cdiv(n, 16) >= 16 * 64 ? 16 : 8;
    return ks;
}

void launch_mfma_multi64(const double *A, long ld, int n, const double *X, long xs, int nr,
                         const double *c, long cs, double *y, long ys, double *part,
                         hipStream_t st) {
    const int ks = multi_ksplit(n);
    const int kchunk = cdiv(cdiv(n, ks), 16) * 16;
    const int ksn = cdiv(n, kchunk);
    hipLaunchKernelGGL((k_mfma_multi<double>), dim3(cdiv(n, 64), ksn), dim3(256), 0, st, A, ld, n,
                       X, xs, nr, kchunk, part);
    hipLaunchKernelGGL(k_reduce_multi, dim3(cdiv(n, 256), nr), dim3(256), 0, st, n, nr, part, ksn,
                       c, cs, y, ys);
}

void launch_mfma_multi32(const float *A, long ld, int n, const float *X, long xs, int nr,
                         const double *c, long cs, double *y, long ys, double *part,
                         hipStream_t st) {
    const int ks = multi_ksplit(n);
    const int kchunk = cdiv(cdiv(n, ks), 16) * 16;
    const int ksn = cdiv(n, kchunk);
    hipLaunchKernelGGL((k_mfma_multi<float>), dim3(cdiv(n, 64), ksn), dim3(256), 0, st, A, ld, n,
                       X, xs, nr, kchunk, part);
    hipLaunchKernelGGL(k_reduce_multi, dim3(cdiv(n, 256), nr), dim3(256), 0, st, n, nr, part, ksn,
                       c, cs, y, ys);
}

void launch_to_f32_batched(const double *src, long ss, float *dst, long ds, int n, int nr,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_to_f32_batched, dim3(cdiv(n, 256), nr), dim3(256), 0, st, src, ss, dst,
                       ds, n);
}

void launch_copy_strided(const double *src, long ss, double *dst, long ds, int n, int nr,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_copy_strided, dim3(cdiv(n, 256), nr), dim3(256), 0, st, src, ss, dst, ds,
                       n);
}

int multi_part_size(int n, int nr) {
    const int ks = multi_ksplit(n);
    const int kchunk = cdiv(cdiv(n, ks), 16) * 16;
    return cdiv(n, kchunk) * nr * n;
}

}  // namespace wwbi
