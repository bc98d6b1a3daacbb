// One pass over a stored m x n matrix for several vectors:
//   Y_s = A X_s,  s < nr,
// on the matrix cores (v_mfma_f64_16x16x4_f64 for an FP64 matrix,
// v_mfma_f32_16x16x4_f32 for FP32).  A wave owns RT tiles of 16 rows and ST
// tiles of 16 systems and shares each B fragment across its row tiles; K is
// split over grid.y and the partial products are reduced in a fixed order.
// The launcher runs k_mfma_multi for up to 16 systems and
// k_mfma_multi_shared, which shares the B tile across the block, for more.
//
// Operand mapping of one 16x16x4 step: lane l supplies A(i, k) with
// i = l % 16, k = l / 16 and B(k, j) with j = l % 16, k = l / 16.  The result
// D(i, j) sits in lane l with j = l % 16 and element r, where the row is
// i = 4 (l / 16) + r for the FP32 instruction and i = l / 16 + 4 r for the
// FP64 one (checked on the device).  The contraction does not care which
// column a k slot stands for: with E elements per 16 bytes, group u of a step
// gives lane (i, q) the E consecutive columns 4E u + E q .. of row i, and
// element e of them feeds the MFMA in slot q.
//
// The matrix is read in 256-byte row pieces, 4 rows per load instruction, so
// that every instruction reads whole contiguous runs; each wave writes its
// tile into its own LDS region and reads it back in the MFMA layout (16-byte
// reads, rows padded by 16 bytes so that 16 lanes hit 16 different bank
// groups).  The next step's matrix and B loads are issued right after the
// LDS write, behind the current step's B loads, so the only wait per step is
// for data requested one step earlier.
//
// Reads run to the end of the step that holds column n - 1, at most
// round_up(n, 64) columns: the matrix rows (ld) and the system rows (xs, and
// the allocation behind the last one) must extend that far.  Columns at or
// past n are zeroed in registers, so padding of any value is harmless.
#include "internal.h"

namespace wwbi {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    using acc = v4d;
    using vec = v2d;                 // 16 bytes
    static constexpr int E = 2;
    static __device__ __forceinline__ int row(int q, int r) { return q + 4 * r; }
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<float> {
    using acc = v4f;
    using vec = v4f;
    static constexpr int E = 4;
    static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// rows per wave (in tiles of 16) and the wave count the K split aims at,
// measured at n = 4608 and 10240: for up to 16 systems, 32 rows (FP32) or 64
// rows (FP64) per wave; for more, the B tile shared by the block
// (k_mfma_multi_shared) and 16 rows (FP32; its LDS then admits four blocks
// per CU) or 32 rows (FP64) per wave, on a grid that runs in one round
template <typename T, int ST> struct MultiShape {
    static constexpr int RT = ST == 2 ? (sizeof(T) == 4 ? 1 : 2) : (sizeof(T) == 4 ? 2 : 4);
    static constexpr int waves = ST == 2 ? 2304 : (RT == 2 ? 4096 : 1920);
};

template <typename T, int ST>
__global__ __launch_bounds__(256) void k_mfma_multi(const T *__restrict__ A, long ld, int m,
                                                    int n, const T *__restrict__ X, long xs,
                                                    int nr, int kchunk,
                                                    double *__restrict__ part) {
    using M = Mfma<T>;
    using V = typename M::vec;
    constexpr int RT = MultiShape<T, ST>::RT;
    constexpr int E = M::E;
    constexpr int KS = 16 * E;           // columns per step: 256 bytes of a row
    constexpr int R = 16 * RT;           // rows per wave
    constexpr int P = R / 4;             // load instructions per step, 4 rows each
    constexpr int U = 4;                 // MFMA groups per step (KS / (4 E))
    constexpr int SW = 64 + 4;           // LDS row stride in 4-byte words
    __shared__ float lds[4][R * SW];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row0 = (blockIdx.x * 4 + wv) * R;
    if (row0 >= m) return;
    const int kb = blockIdx.y * kchunk;
    const int ke = min(n, kb + kchunk);
    const int i = lane & 15, q = lane >> 4;
    // load p: lane l reads 16 bytes at column (l % 16) E of row 4 p + l / 16
    const int lr = lane >> 4, lc = (lane & 15) * E;
    const V *ap[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = min(row0 + 4 * p + lr, m - 1);
        ap[p] = reinterpret_cast<const V *>(A + (long)r * ld + kb + lc);
    }
    const V *xp[ST];
#pragma unroll
    for (int st = 0; st < ST; ++st) {
        const int s = 16 * st + i;
        xp[st] = reinterpret_cast<const V *>(X + (long)(s < nr ? s : 0) * xs + kb + E * q);
    }
    float *L = lds[wv];
    typename M::acc c[RT][ST];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int st = 0; st < ST; ++st) c[rt][st] = typename M::acc{0, 0, 0, 0};
    V ga[P];
    V bb[U][ST];
#pragma unroll
    for (int p = 0; p < P; ++p) ga[p] = __builtin_nontemporal_load(ap[p]);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int st = 0; st < ST; ++st) bb[u][st] = xp[st][4 * u];
    // one step at column k0; pf: fetch the next step, tail: zero columns >= ke
    auto body = [&](const int k0, const bool pf, const bool tail) __attribute__((always_inline)) {
        const int off = (k0 - kb) / E;
        if (tail) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const bool in = k0 + lc + e < ke;
#pragma unroll
                for (int p = 0; p < P; ++p) ga[p][e] = in ? ga[p][e] : (T)0;
            }
        }
        // the compiler keeps LDS and global accesses in this order; one
        // wave's LDS operations complete in issue order, so the writes land
        // after the previous step's fragment reads
        asm volatile("" ::: "memory");
#pragma unroll
        for (int p = 0; p < P; ++p)
            *reinterpret_cast<V *>(L + (4 * p + lr) * SW + lc * (int)sizeof(T) / 4) = ga[p];
        asm volatile("" ::: "memory");
        V bn[U][ST];
        if (pf) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int st = 0; st < ST; ++st) bn[u][st] = xp[st][off + KS / E + 4 * u];
#pragma unroll
            for (int p = 0; p < P; ++p)
                ga[p] = __builtin_nontemporal_load(ap[p] + off + KS / E);
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < U; ++u) {
            V b[ST];
#pragma unroll
            for (int st = 0; st < ST; ++st) b[st] = bb[u][st];
            if (tail) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const bool in = k0 + 4 * E * u + E * q + e < ke;
#pragma unroll
                    for (int st = 0; st < ST; ++st) b[st][e] = in ? b[st][e] : (T)0;
                }
            }
            V a[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                a[rt] = *reinterpret_cast<const V *>(L + (16 * rt + i) * SW +
                                                     (4 * E * u + E * q) * (int)sizeof(T) / 4);
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int st = 0; st < ST; ++st)
                        c[rt][st] = M::step(a[rt][e], b[st][e], c[rt][st]);
        }
        if (pf) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int st = 0; st < ST; ++st) bb[u][st] = bn[u][st];
        }
    };
    // every step but the last fetches its successor unconditionally, so the
    // waits of the loop count only the loads they need
    int k0 = kb;
    for (; k0 + KS < ke; k0 += KS) body(k0, true, false);
    body(k0, false, k0 + KS > ke);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int st = 0; st < ST; ++st) {
            const int s = 16 * st + i;
            if (s >= nr) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = row0 + 16 * rt + M::row(q, r);
                if (rr < m) part[((long)blockIdx.y * nr + s) * m + rr] = (double)c[rt][st][r];
            }
        }
}

// The same product for 17..32 systems with the B tile shared by the block:
// the 4 waves of a block cover consecutive row tiles over one K chunk, so the
// block loads the 32 x 256-byte B tile of a step once, into one of two LDS
// buffers, and synchronises once per step.  The buffer written at step t was
// last read at step t - 2, and every wave has passed the barrier of step t - 1
// (which follows its reads of step t - 2) before any wave writes it again.
// Each wave keeps its own matrix tile in LDS as in k_mfma_multi.  Waves past
// the last row load row m - 1, join every barrier and store nothing.
template <typename T>
__global__ __launch_bounds__(256) void k_mfma_multi_shared(const T *__restrict__ A, long ld, int m,
                                                           int n, const T *__restrict__ X,
                                                           long xs, int nr, int kchunk,
                                                           double *__restrict__ part) {
    using M = Mfma<T>;
    using V = typename M::vec;
    constexpr int RT = MultiShape<T, 2>::RT;
    constexpr int E = M::E;
    constexpr int KS = 16 * E;           // columns per step: 256 bytes of a row
    constexpr int R = 16 * RT;           // rows per wave
    constexpr int P = R / 4;             // matrix load instructions per step
    constexpr int U = 4;                 // MFMA groups per step
    constexpr int SW = 64 + 4;           // LDS row stride in 4-byte words
    constexpr int NS = 32;               // systems in the B tile
    constexpr int XB = NS * 16 / 256;    // B pieces of 16 bytes per thread per step
    __shared__ float lds[4][R * SW];
    __shared__ float ldx[2][NS * SW];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
    const int row0 = (blockIdx.x * 4 + wv) * R;
    const int kb = blockIdx.y * kchunk;
    const int ke = min(n, kb + kchunk);
    const int i = lane & 15, q = lane >> 4;
    const int lr = lane >> 4, lc = (lane & 15) * E;
    const V *ap[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = min(row0 + 4 * p + lr, m - 1);
        ap[p] = reinterpret_cast<const V *>(A + (long)r * ld + kb + lc);
    }
    // B piece f = tid + 256 j: system f / 16, columns (f % 16) E ..
    const V *xq[XB];
    int xrow[XB], xcol[XB];
#pragma unroll
    for (int j = 0; j < XB; ++j) {
        const int f = tid + 256 * j;
        xrow[j] = f / 16;
        xcol[j] = (f % 16) * E;
        xq[j] = reinterpret_cast<const V *>(X + (long)(xrow[j] < nr ? xrow[j] : 0) * xs + kb +
                                            xcol[j]);
    }
    float *L = lds[wv];
    typename M::acc c[RT][2];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) c[rt][0] = c[rt][1] = typename M::acc{0, 0, 0, 0};
    V ga[P], gx[XB];
#pragma unroll
    for (int p = 0; p < P; ++p) ga[p] = __builtin_nontemporal_load(ap[p]);
#pragma unroll
    for (int j = 0; j < XB; ++j) gx[j] = xq[j][0];
    int buf = 0;
    auto body = [&](const int k0, const bool pf, const bool tail) __attribute__((always_inline)) {
        const int off = (k0 - kb) / E;
        if (tail) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
#pragma unroll
                for (int p = 0; p < P; ++p) ga[p][e] = (k0 + lc + e < ke) ? ga[p][e] : (T)0;
#pragma unroll
                for (int j = 0; j < XB; ++j) gx[j][e] = (k0 + xcol[j] + e < ke) ? gx[j][e] : (T)0;
            }
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int p = 0; p < P; ++p)
            *reinterpret_cast<V *>(L + (4 * p + lr) * SW + lc * (int)sizeof(T) / 4) = ga[p];
        float *LX = ldx[buf];
#pragma unroll
        for (int j = 0; j < XB; ++j)
            *reinterpret_cast<V *>(LX + xrow[j] * SW + xcol[j] * (int)sizeof(T) / 4) = gx[j];
        asm volatile("" ::: "memory");
        if (pf) {
#pragma unroll
            for (int j = 0; j < XB; ++j) gx[j] = xq[j][off + KS / E];
#pragma unroll
            for (int p = 0; p < P; ++p)
                ga[p] = __builtin_nontemporal_load(ap[p] + off + KS / E);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            V a[RT], b[2];
#pragma unroll
            for (int st = 0; st < 2; ++st)
                b[st] = *reinterpret_cast<const V *>(LX + (16 * st + i) * SW +
                                                     (4 * E * u + E * q) * (int)sizeof(T) / 4);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                a[rt] = *reinterpret_cast<const V *>(L + (16 * rt + i) * SW +
                                                     (4 * E * u + E * q) * (int)sizeof(T) / 4);
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int st = 0; st < 2; ++st)
                        c[rt][st] = M::step(a[rt][e], b[st][e], c[rt][st]);
        }
        buf ^= 1;
    };
    int k0 = kb;
    for (; k0 + KS < ke; k0 += KS) body(k0, true, false);
    body(k0, false, k0 + KS > ke);
    if (row0 >= m) return;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const int s = 16 * st + i;
            if (s >= nr) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = row0 + 16 * rt + M::row(q, r);
                if (rr < m) part[((long)blockIdx.y * nr + s) * m + rr] = (double)c[rt][st][r];
            }
        }
}

// y_s = c_s - sum_k part[k][s] (or the plain sum when c is null), m rows
__global__ void k_reduce_multi(int m, int nr, const double *__restrict__ part, int ks,
                               const double *__restrict__ c, long cs, double *__restrict__ y,
                               long ys) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (r >= m || s >= nr) return;
    double acc = 0.0;
    for (int k = 0; k < ks; ++k) acc += part[((long)k * nr + s) * m + r];
    y[(long)s * ys + r] = c ? c[(long)s * cs + r] - acc : acc;
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

// K split: chunks a multiple of 64 columns (every step then starts on a
// 64-column boundary), as many as bring the grid near the shape's wave count
struct MultiGrid {
    int kchunk, ksn;
};

MultiGrid multi_grid(int m, int n, int rt, int waves) {
    const int tiles = cdiv(m, 16 * rt);
    const int ks = std::max(1, std::min(16, cdiv(waves, tiles)));
    const int kchunk = cdiv(cdiv(n, ks), 64) * 64;
    return {kchunk, cdiv(n, kchunk)};
}

template <typename T, int ST> MultiGrid multi_grid_for(int m, int n) {
    return multi_grid(m, n, MultiShape<T, ST>::RT, MultiShape<T, ST>::waves);
}

// the product into K-split partial slices, then (y non-null) their sum;
// returns the slice count
template <typename T, int ST>
int launch_mfma_st(const T *A, long ld, int m, int n, const T *X, long xs, int nr,
                   const double *c, long cs, double *y, long ys, double *part, hipStream_t st) {
    const MultiGrid g = multi_grid_for<T, ST>(m, n);
    const dim3 grid(cdiv(m, 4 * 16 * MultiShape<T, ST>::RT), g.ksn);
    if (ST == 2)
        hipLaunchKernelGGL((k_mfma_multi_shared<T>), grid, dim3(256), 0, st, A, ld, m, n, X, xs,
                           nr, g.kchunk, part);
    else
        hipLaunchKernelGGL((k_mfma_multi<T, 1>), grid, dim3(256), 0, st, A, ld, m, n, X, xs, nr,
                           g.kchunk, part);
    if (y)
        hipLaunchKernelGGL(k_reduce_multi, dim3(cdiv(m, 256), nr), dim3(256), 0, st, m, nr, part,
                           g.ksn, c, cs, y, ys);
    return g.ksn;
}

template <typename T>
int launch_mfma_multi(const T *A, long ld, int m, int n, const T *X, long xs, int nr,
                      const double *c, long cs, double *y, long ys, double *part,
                      hipStream_t st) {
    if (nr > 16) return launch_mfma_st<T, 2>(A, ld, m, n, X, xs, nr, c, cs, y, ys, part, st);
    return launch_mfma_st<T, 1>(A, ld, m, n, X, xs, nr, c, cs, y, ys, part, st);
}

}  // namespace

void launch_mfma_multi64(const double *A, long ld, int n, const double *X, long xs, int nr,
                         const double *c, long cs, double *y, long ys, double *part,
                         hipStream_t st) {
    launch_mfma_multi<double>(A, ld, n, n, X, xs, nr, c, cs, y, ys, part, st);
}

void launch_mfma_multi32(const float *A, long ld, int n, const float *X, long xs, int nr,
                         const double *c, long cs, double *y, long ys, double *part,
                         hipStream_t st) {
    launch_mfma_multi<float>(A, ld, n, n, X, xs, nr, c, cs, y, ys, part, st);
}

int launch_mfma_parts64(const double *A, long ld, int n, const double *X, long xs, int nr,
                        double *part, hipStream_t st) {
    return launch_mfma_multi<double>(A, ld, n, n, X, xs, nr, nullptr, 0, nullptr, 0, part, st);
}

int launch_mfma_parts32(const float *A, long ld, int n, const float *X, long xs, int nr,
                        double *part, hipStream_t st) {
    return launch_mfma_multi<float>(A, ld, n, n, X, xs, nr, nullptr, 0, nullptr, 0, part, st);
}

void launch_mfma_rect64(const double *A, long ld, int m, int n, const double *X, long xs, int nr,
                        double *y, long ys, double *part, hipStream_t st) {
    launch_mfma_multi<double>(A, ld, m, n, X, xs, nr, nullptr, 0, y, ys, part, st);
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

// the largest partial-sum buffer any shape and precision needs for nr systems
int multi_part_size(int n, int nr) {
    int ks = 0;
    for (const MultiGrid g : {multi_grid_for<float, 1>(n, n), multi_grid_for<float, 2>(n, n),
                              multi_grid_for<double, 1>(n, n), multi_grid_for<double, 2>(n, n)})
        ks = std::max(ks, g.ksn);
    return ks * nr * n;
}

// the same for the FP64 product of an m x n matrix
int multi_part_size_rect64(int m, int n, int nr) {
    int ks = 0;
    for (const MultiGrid g : {multi_grid_for<double, 1>(m, n), multi_grid_for<double, 2>(m, n)})
        ks = std::max(ks, g.ksn);
    return ks * nr * m;
}

}  // namespace wwbi
