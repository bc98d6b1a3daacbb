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

// Optional epilogue of the Arnoldi step: the first Gram-Schmidt dots
// P[i * gridDim.x + block] = sum over the block's rows of V_i * y, i <= j < 64,
// and the block's squared norm of y in P3[block], for the next kernel to sum
// in a fixed order.  Lane i loads V_i at the wave's rows before the matrix
// stream starts, so the epilogue waits on nothing new.
struct GemvDots {
    const double *V;    // basis, row i at V + i * ldv
    long ldv;
    int j;              // last basis vector (j < 64)
    double *P, *P3;
};

// y = c - A x (or A x): each wave owns R rows and walks them in steps of
// 64 lanes x 16 bytes, U steps in flight, every product accumulated in TACC.
// An FP32 matrix (and FP32 x) accumulates in FP64: the accumulation then adds
// no error that grows with the row length, and a product's error is set by
// the FP32 entries and vector alone.
template <typename TA, typename TX, typename TACC, int R, int U, bool DOTS = false, int WPB = 4>
__global__ __launch_bounds__(64 * WPB) void k_gemv(const TA *__restrict__ A, long ld, int n,
                                              const TX *__restrict__ x,
                                              const double *__restrict__ c,
                                              double *__restrict__ y, const int *active,
                                              GemvDots d = GemvDots{}) {
    if (active && *active == 0) return;     // uniform over the grid
    using V = typename Vec16<TA>::type;
    constexpr int VW = Vec16<TA>::n;
    constexpr int STEP = 64 * VW;
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * WPB + (threadIdx.x >> 6);
    const long r0 = wave * R;
    double vr[R];
    if (DOTS) {
        // waves past the last row still reach the block barrier below
#pragma unroll
        for (int r = 0; r < R; ++r)
            vr[r] = (lane <= d.j && r0 + r < n) ? d.V[(long)lane * d.ldv + r0 + r] : 0.0;
    } else if (r0 >= n) {
        return;
    }
    const TA *rowp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rowp[r] = A + (r0 + r < n ? r0 + r : n - 1) * ld;
    TACC acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = (TACC)0;
    const int nbig = r0 < n ? (n / (STEP * U)) * (STEP * U) : 0;
    for (int c0 = 0; c0 < nbig; c0 += STEP * U) {
        // every load of the U steps is issued before any value is converted
        // or used, so that all of them are in flight together
        V a[U][R];
        TX xv[U][VW];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int col = c0 + u * STEP + lane * VW;
#pragma unroll
            for (int r = 0; r < R; ++r) a[u][r] = stream_load(rowp[r] + col);
            load_x<TX, TX, VW>(x, col, xv[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int v = 0; v < VW; ++v) acc[r] += (TACC)a[u][r][v] * (TACC)xv[u][v];
    }
    const int nstep = r0 < n ? (n / STEP) * STEP : 0;
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
    for (int col = nstep + lane; r0 < n && col < n; col += 64) {
        const TACC xv = (TACC)x[col];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += (TACC)rowp[r][col] * xv;
    }
    double pd = 0.0, nn = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const TACC s = wave_sum(acc[r]);
        const double v = (double)s;
        if (!DOTS) {
            if (lane == 0 && r0 + r < n) y[r0 + r] = c ? c[r0 + r] - v : v;
        } else if (r0 + r < n) {
            // the fused step is an Arnoldi product: y = A x (no c)
            if (lane == 0) y[r0 + r] = v;
            pd += vr[r] * v;
            nn += v * v;
        }
    }
    if (DOTS) {
        __shared__ double sp[WPB][64];
        __shared__ double sn[WPB];
        const int wv = threadIdx.x >> 6;
        sp[wv][lane] = pd;
        if (lane == 0) sn[wv] = nn;
        __syncthreads();
        if (wv == 0) {
            double t = 0.0, u = 0.0;
#pragma unroll
            for (int k = 0; k < WPB; ++k) {
                t += sp[k][lane];
                u += sn[k];
            }
            if (lane <= d.j) d.P[(long)lane * gridDim.x + blockIdx.x] = t;
            if (lane == 0) d.P3[blockIdx.x] = u;
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

// waves per block of the fused product (8, with half the partials, streamed
// slower: 70.9 against 65 us per launch at n = 10240)
constexpr int kDotsWaves = 4;

int gemv_partials(int n) { return cdiv(cdiv(n, kGemvR), kDotsWaves); }

void launch_gemv32_dots(const float *A, long ld, int n, const float *x, double *y,
                        const int *active, const double *V, long ldv, int j, double *P,
                        double *P3, hipStream_t st) {
    hipLaunchKernelGGL((k_gemv<float, float, double, kGemvR, kGemvU, true, kDotsWaves>),
                       dim3(gemv_partials(n)), dim3(64 * kDotsWaves), 0, st, A, ld, n, x, nullptr,
                       y, active, GemvDots{V, ldv, j, P, P3});
}

void launch_gemv64_dots(const double *A, long ld, int n, const double *x, double *y,
                        const int *active, const double *V, long ldv, int j, double *P,
                        double *P3, hipStream_t st) {
    hipLaunchKernelGGL((k_gemv<double, double, double, kGemvR, kGemvU, true, kDotsWaves>),
                       dim3(gemv_partials(n)), dim3(64 * kDotsWaves), 0, st, A, ld, n, x,
                       nullptr, y, active, GemvDots{V, ldv, j, P, P3});
}

void launch_gemv32(const float *A, long ld, int n, const float *x, const double *c, double *y,
                   const int *active, hipStream_t st) {
    hipLaunchKernelGGL((k_gemv<float, float, double, kGemvR, kGemvU>),
                       dim3(gemv_blocks(n, kGemvR)), dim3(256), 0, st, A, ld, n, x, c, y, active);
}


}  // namespace wwbi
