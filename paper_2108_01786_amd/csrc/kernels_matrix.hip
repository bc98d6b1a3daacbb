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

// Kinds of a far entry of A when the target and source boundaries are
// uniform: the real part of the source-flavour term (surface row and wall
// column), its negative (wall row and surface column), or the imaginary part.
enum { kFastReNeg = 0, kFastRePos = 1, kFastIm = 2 };

// ---------------------------------------------------------------------------
// assembly: one thread per column (coalesced row writes), a tile of rows per
// block with the target data staged in LDS (read as broadcasts).
// ---------------------------------------------------------------------------
// FP64 assembly of A (WALL = 0), of the wall operator T - I/2 on the walls
// (WALL = 1), of the gamma_t operator (WALL = 2) or of the normal-velocity
// map T on the surface rows (WALL = 3): one column per thread.
template <int WALL, typename OutT = double>
__global__ __launch_bounds__(256) void k_assemble(Nodes N, const double *hrow, int r0, int nr,
                                                  int c0, int nc, int corr, OutT *out,
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
        double v = 0.0;
        if (live) {
            if (WALL == 2) {
                v = gt_val64(N, tg[i], s);
            } else if (WALL == 3) {
                v = t_val64(N, tg[i], s, hrow);
            } else if (WALL == 1) {
                v = t_val64(N, tg[i], s, hrow);
                if (tg[i].k == s.k && tg[i].loc == s.loc) v -= 0.5;
            } else {
                v = a_val64(N, tg[i], s, corr != 0);
            }
        }
        __builtin_nontemporal_store((OutT)v, out + (long)(rbase + i) * ld + col);
    }
}

// FP64 assembly of the transpose A^T (row q = source q, column p = target p):
// the staged rows hold sources, each thread one target.
__global__ __launch_bounds__(256) void k_assemble64T(Nodes N, int n, int corr, double *out,
                                                     long ld) {
    __shared__ Src ss[kRowsPerAsmBlock];
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int rbase = blockIdx.y * kRowsPerAsmBlock;
    if (threadIdx.x < kRowsPerAsmBlock) {
        const int r = rbase + threadIdx.x;
        if (r < n) ss[threadIdx.x] = load_src(N, r);
    }
    __syncthreads();
    if (col >= ld) return;
    const bool live = col < n;
    const Tgt t = load_tgt(N, live ? col : 0);
    const int rend = min(kRowsPerAsmBlock, n - rbase);
    for (int i = 0; i < rend; ++i)
        __builtin_nontemporal_store(live ? a_val64(N, t, ss[i], corr != 0) : 0.0,
                                    out + (long)(rbase + i) * ld + col);
}

// FP32 entry of A for a pair outside the FP64 band, when the wave's columns
// lie on one boundary (the kind of entry is then wave-uniform): the same
// quotient as kappa32 with the hardware reciprocal, and the source data
// pre-scaled as a = w dx / 2, b = w dy / 2 (see rows_tile_a64 for the parts).
template <int KIND>
__device__ __forceinline__ float a_far32_fast(const Tgt &t, double sex, double sey, float a,
                                              float b, float ec) {
    const float nr = (float)(sex + t.ex), ni = (float)(sey + t.ey);
    const float dr = (float)(sex - t.ex), di = (float)(sey - t.ey);
    const float inv = __builtin_amdgcn_rcpf(dr * dr + di * di);
    const float pr = nr * dr + ni * di;
    const float pi = ni * dr - nr * di;
    if (KIND == kFastReNeg) return -(a * pi + b * pr) * inv;
    if (KIND == kFastRePos) return (a * pi + b * pr) * inv;
    return (a * pr - b * pi) * inv - ec;
}

// FP32 assembly of A in two passes.  The far pass writes every entry outside
// the FP64 band (same-boundary pairs within `band` steps, diagonal included),
// one column per thread and kRowsPerAsm32 rows per block: a wave whose live
// columns lie on one boundary and whose row is clear of their band takes the
// wave-uniform fast entry, any other wave a_far32 (zero inside the band).
// The band pass then overwrites the band entries with FP64 values rounded
// once, as a_val32 gives them.
// Keeping the FP64 near-field code out of the far pass keeps its register
// count, and so its occupancy, low: the far pass is bound by its stores.
constexpr int kRowsPerAsm32 = 16;

__global__ __launch_bounds__(256) void k_assemble32_far(Nodes N, int n, int corr, int band,
                                                        float *out, long ld) {
    __shared__ Tgt tg[kRowsPerAsm32];
    const int wb = wave_base();
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int rbase = blockIdx.y * kRowsPerAsm32;
    if (threadIdx.x < kRowsPerAsm32) {
        const int r = rbase + threadIdx.x;
        if (r < n) tg[threadIdx.x] = load_tgt(N, r);
    }
    __syncthreads();
    if (col >= ld) return;
    const bool live = col < n;
    const Src s = load_src(N, live ? col : 0);
    const float fa = (float)(0.5 * s.w * s.dx), fb = (float)(0.5 * s.w * s.dy);
    const float fw = (float)s.w;
    // the wave's live columns [ca, cb]: on one boundary kq (local indices
    // [lqa, lqb] of mq nodes), or kq = -1
    const int ca = blockIdx.x * 256 + wb, cb = min(ca + 63, n - 1);
    int kq = -1, lqa = 0, lqb = 0, mq = 0;
    if (ca < n) {
        kq = range_boundary(N, ca, cb);
        lqa = N.loc[ca];
        lqb = N.loc[cb];
        mq = N.Mk[ca];
    }
    const int rend = min(kRowsPerAsm32, n - rbase);
    float *o = out + (long)rbase * ld + col;
    // the usual case: all rows of the tile on one boundary kp and clear of the
    // band of all the wave's columns, one kind of entry for the whole tile
    const int kr = kq >= 0 ? range_boundary(N, rbase, rbase + rend - 1) : -1;
    if (kr >= 0 && ranges_apart(N, rbase, rbase + rend - 1, ca, cb, band)) {
        if ((kr == 0) == (kq == 0)) {
            const float ec = (corr && kr == kq && kr >= 2) ? fw : 0.0f;
            for (int i = 0; i < rend; ++i)
                __builtin_nontemporal_store(
                    live ? a_far32_fast<kFastIm>(tg[i], s.ex, s.ey, fa, fb, ec) : 0.0f, o + i * ld);
        } else if (kr == 0) {
            for (int i = 0; i < rend; ++i)
                __builtin_nontemporal_store(
                    live ? a_far32_fast<kFastReNeg>(tg[i], s.ex, s.ey, fa, fb, 0.0f) : 0.0f,
                    o + i * ld);
        } else {
            for (int i = 0; i < rend; ++i)
                __builtin_nontemporal_store(
                    live ? a_far32_fast<kFastRePos>(tg[i], s.ex, s.ey, fa, fb, 0.0f) : 0.0f,
                    o + i * ld);
        }
        return;
    }
    for (int i = 0; i < rend; ++i) {
        bool apart = false;
        int kp = -1;
        if (kq >= 0) {
            kp = __builtin_amdgcn_readfirstlane(tg[i].k);
            apart = kp != kq;
            if (!apart) {
                const int lp = __builtin_amdgcn_readfirstlane(tg[i].loc);
                const int gap = max(0, max(lqa - lp, lp - lqb));
                const int span = max(lp - lqa, lqb - lp);
                apart = gap > band && mq - span > band;
            }
        }
        float v;
        if (apart) {
            if ((kp == 0) == (kq == 0))
                v = a_far32_fast<kFastIm>(tg[i], s.ex, s.ey, fa, fb,
                                          (corr && kp == kq && kp >= 2) ? fw : 0.0f);
            else if (kp == 0)
                v = a_far32_fast<kFastReNeg>(tg[i], s.ex, s.ey, fa, fb, 0.0f);
            else
                v = a_far32_fast<kFastRePos>(tg[i], s.ex, s.ey, fa, fb, 0.0f);
        } else {
            v = a_far32(tg[i], s, corr != 0, band);
        }
        __builtin_nontemporal_store(live ? v : 0.0f, o + i * ld);
    }
}

// The same far pass for the transpose: row q of the output is source q and
// column p target p, so out = A^T with the same row-major layout (the adjoint
// then streams it with the forward product).  The staged rows hold sources,
// each thread one target.
struct SrcRow {
    Src s;
    float fa, fb, fw;   // w dx / 2, w dy / 2, w in FP32
};

__global__ __launch_bounds__(256) void k_assemble32T_far(Nodes N, int n, int corr, int band,
                                                         float *out, long ld) {
    __shared__ SrcRow sr[kRowsPerAsm32];
    const int wb = wave_base();
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int rbase = blockIdx.y * kRowsPerAsm32;
    if (threadIdx.x < kRowsPerAsm32) {
        const int r = rbase + threadIdx.x;
        if (r < n) {
            const Src v = load_src(N, r);
            sr[threadIdx.x] = SrcRow{v, (float)(0.5 * v.w * v.dx), (float)(0.5 * v.w * v.dy),
                                     (float)v.w};
        }
    }
    __syncthreads();
    if (col >= ld) return;
    const bool live = col < n;
    const Tgt t = load_tgt(N, live ? col : 0);
    // the wave's live columns (targets) [ca, cb]: on one boundary kp (local
    // indices [lpa, lpb] of mp nodes), or kp = -1
    const int ca = blockIdx.x * 256 + wb, cb = min(ca + 63, n - 1);
    int kp = -1, lpa = 0, lpb = 0, mp = 0;
    if (ca < n) {
        kp = range_boundary(N, ca, cb);
        lpa = N.loc[ca];
        lpb = N.loc[cb];
        mp = N.Mk[ca];
    }
    const int rend = min(kRowsPerAsm32, n - rbase);
    float *o = out + (long)rbase * ld + col;
    const int kr = kp >= 0 ? range_boundary(N, rbase, rbase + rend - 1) : -1;   // sources
    if (kr >= 0 && ranges_apart(N, ca, cb, rbase, rbase + rend - 1, band)) {
        if ((kp == 0) == (kr == 0)) {
            const bool ec = corr && kp == kr && kp >= 2;
            for (int i = 0; i < rend; ++i) {
                const SrcRow &q = sr[i];
                __builtin_nontemporal_store(
                    live ? a_far32_fast<kFastIm>(t, q.s.ex, q.s.ey, q.fa, q.fb, ec ? q.fw : 0.0f)
                         : 0.0f,
                    o + i * ld);
            }
        } else if (kp == 0) {
            for (int i = 0; i < rend; ++i) {
                const SrcRow &q = sr[i];
                __builtin_nontemporal_store(
                    live ? a_far32_fast<kFastReNeg>(t, q.s.ex, q.s.ey, q.fa, q.fb, 0.0f) : 0.0f,
                    o + i * ld);
            }
        } else {
            for (int i = 0; i < rend; ++i) {
                const SrcRow &q = sr[i];
                __builtin_nontemporal_store(
                    live ? a_far32_fast<kFastRePos>(t, q.s.ex, q.s.ey, q.fa, q.fb, 0.0f) : 0.0f,
                    o + i * ld);
            }
        }
        return;
    }
    for (int i = 0; i < rend; ++i) {
        const SrcRow &q = sr[i];
        bool apart = false;
        int kq = -1;
        if (kp >= 0) {
            kq = __builtin_amdgcn_readfirstlane(q.s.k);
            apart = kp != kq;
            if (!apart) {
                const int lq = __builtin_amdgcn_readfirstlane(q.s.loc);
                const int gap = max(0, max(lpa - lq, lq - lpb));
                const int span = max(lq - lpa, lpb - lq);
                apart = gap > band && mp - span > band;
            }
        }
        float v;
        if (apart) {
            if ((kp == 0) == (kq == 0))
                v = a_far32_fast<kFastIm>(t, q.s.ex, q.s.ey, q.fa, q.fb,
                                          (corr && kp == kq && kp >= 2) ? q.fw : 0.0f);
            else if (kp == 0)
                v = a_far32_fast<kFastReNeg>(t, q.s.ex, q.s.ey, q.fa, q.fb, 0.0f);
            else
                v = a_far32_fast<kFastRePos>(t, q.s.ex, q.s.ey, q.fa, q.fb, 0.0f);
        } else {
            v = a_far32(t, q.s, corr != 0, band);
        }
        __builtin_nontemporal_store(live ? v : 0.0f, o + i * ld);
    }
}

// Band pass: thread (row p, offset j) writes A(p, q) for the same-boundary
// node q at cyclic offset j - band (every node of a boundary with at most
// 2 band + 1 nodes, each once), evaluated in FP64 and rounded once; at
// (q, p) for the transpose.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_assemble32_band(Nodes N, int n, int corr, int band,
                                                         float *out, long ld) {
    const int w = 2 * band + 1;
    const long id = (long)blockIdx.x * 256 + threadIdx.x;
    if (id >= (long)n * w) return;
    const int p = (int)(id / w), j = (int)(id % w);
    const int loc = N.loc[p], M = N.Mk[p];
    const bool whole = w >= M;
    if (whole && j >= M) return;
    int l = whole ? j : loc + j - band;
    if (l < 0) l += M;
    if (l >= M) l -= M;
    const int q = p - loc + l;
    const float v = (float)a_val64(N, load_tgt(N, p), load_src(N, q), corr != 0);
    if (TRANS)
        out[(long)q * ld + p] = v;
    else
        out[(long)p * ld + q] = v;
}

// ---------------------------------------------------------------------------
// on-the-fly products: entries recomputed in registers, never stored.
// Forward: one thread per target row, a chunk of sources per grid.y staged in
// LDS.  Transpose: one thread per source column, a chunk of targets staged.
// Mode selects the entry: 0 = A in FP64, 1 = A in FP32 (with FP64 band),
// 2 = target-flavour T, 3 = target-flavour wall operator (T - I/2),
// 4 = stream-function map P on the surface, 5 = tangential map Q,
// 6 / 7 = source-flavour maps KS / GS of the F operators, 8 = gamma_t operator.
// ---------------------------------------------------------------------------
constexpr int kStage = 256;          // chunk granularity of otf_chunk (adjoint contractions)
// Sources (targets) staged per pass of the forward (transpose) product: 128
// keeps a block's LDS near 13 KB, so that LDS does not limit the resident
// blocks below the wave limit.
constexpr int kOtfStage = 128;
constexpr int kOtfBlocks = 8192;     // target grid size of an on-the-fly product
constexpr int kOtfMaxSlices = 256;   // at most this many partial slices (+ the near band)

// Far part of an entry (zero inside the near band of width nb).
template <int MODE>
__device__ __forceinline__ double entry(const Nodes &N, const Tgt &t, const Src &s, bool corr,
                                        int nb, const double *hrow) {
    (void)N;
    if (MODE == 0) return a_far64(t, s, corr, nb);
    if (MODE == 1) return (double)a_far32(t, s, corr, nb);
    if (MODE == 4) return psi_far64(t, s, hrow, nb);
    if (MODE == 5) return tan_far64(t, s, hrow, nb);
    if (MODE == 6) return ks_far64(t, s, nb);
    if (MODE == 7) return gs_far64(t, s, hrow, nb);
    if (MODE == 8) return gt_far64(t, s, nb);
    return t_far64(t, s, hrow, nb);
}

// Full entry (near band pairs), with the FP32 band rule of the stored matrix.
template <int MODE>
__device__ __forceinline__ double entry_full(const Nodes &N, const Tgt &t, const Src &s, bool corr,
                                             int band, const double *hrow) {
    if (MODE == 0) return a_val64(N, t, s, corr);
    if (MODE == 1) return (double)a_val32(N, t, s, corr, band);
    if (MODE == 4) return psi_val64(N, t, s, hrow);
    if (MODE == 5) return tan_val64(N, t, s, hrow);
    if (MODE == 6) return ks_val64(N, t, s);
    if (MODE == 7) return gs_val64(N, t, s, hrow);
    if (MODE == 8) return gt_val64(N, t, s);
    double v = t_val64(N, t, s, hrow);
    if (MODE == 3 && t.k == s.k && t.loc == s.loc) v -= 0.5;
    return v;
}

// Near part: for each output node, the same-boundary partners within nb
// grid steps, with the exact entry (written as one more partial slice).
//   rows: out[r] = sum over q near r0+r (q in [c0, c0+nc)) of E(r0+r, q) x[q-c0]
//   cols: out[c] = sum over p near c0+c (p in [r0, r0+nr)) of E(p, c0+c) x[p-r0]
// A group of kNearLanes lanes shares one output: lane g takes the partners
// d0 + g, d0 + g + kNearLanes, ... and the group adds its lanes in a fixed
// butterfly order.
constexpr int kNearLanes = 8;
constexpr int kNearPerBlock = 256 / kNearLanes;

template <int MODE, bool COLS>
__global__ __launch_bounds__(256) void k_near_band(Nodes N, const double *hrow, int r0, int nr,
                                                   int c0, int nc, int corr, int band, int nb,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ out, const int *active) {
    if (active && *active == 0) return;
    const int g = threadIdx.x % kNearLanes;
    const int i = blockIdx.x * kNearPerBlock + threadIdx.x / kNearLanes;
    const int nout = COLS ? nc : nr;
    double acc = 0.0;
    if (i < nout) {
        const int me = (COLS ? c0 : r0) + i;
        const int loc = N.loc[me], M = N.Mk[me];
        const int base = me - loc;
        // partners: every node with cyclic distance <= nb, each exactly once
        // (the whole boundary when it has at most 2 nb + 1 nodes)
        const bool whole = 2 * nb + 1 >= M;
        const int d0 = whole ? -loc : -nb, d1 = whole ? M - 1 - loc : nb;
        if (!COLS) {
            const Tgt t = load_tgt(N, me);
            for (int d = d0 + g; d <= d1; d += kNearLanes) {
                int l = loc + d;
                if (l < 0) l += M;
                if (l >= M) l -= M;
                const int q = base + l;
                if (q < c0 || q >= c0 + nc) continue;
                acc += entry_full<MODE>(N, t, load_src(N, q), corr != 0, band, hrow) * x[q - c0];
            }
        } else {
            const Src s = load_src(N, me);
            for (int d = d0 + g; d <= d1; d += kNearLanes) {
                int l = loc + d;
                if (l < 0) l += M;
                if (l >= M) l -= M;
                const int p = base + l;
                if (p < r0 || p >= r0 + nr) continue;
                acc += entry_full<MODE>(N, load_tgt(N, p), s, corr != 0, band, hrow) * x[p - r0];
            }
        }
    }
#pragma unroll
    for (int o = kNearLanes / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (i < nout && g == 0) out[i] = acc;
}

// Forward product: each thread owns kTPT target rows (rows t, t + 256, ... of
// the block's 256 * kTPT).  One row per thread and many short blocks measured
// fastest: the FP64 entry is a long dependent chain, and more resident blocks
// hide it better than more rows per thread (2 rows: +3%, 4 rows: +18%).
constexpr int kTPT = 1;

// One staged tile of the forward product; CHECK = false when the tile is
// known to hold no near-band pair (the entries are then the same as with
// the test, which always fails).
template <int MODE, bool ACC32, bool CHECK>
__device__ __forceinline__ void rows_tile(const Nodes &N, const Tgt (&t)[kTPT], const Src *ss,
                                          const double *sx, int m, bool corr, int nb,
                                          const double *hrow, double (&acc)[kTPT],
                                          float (&acc32)[kTPT]) {
    for (int i = 0; i < m; ++i) {
        const Src s = ss[i];
        const double xv = sx[i];
#pragma unroll
        for (int u = 0; u < kTPT; ++u) {
            const double e = entry<MODE>(N, t[u], s, corr, CHECK ? nb : -1, hrow);
            if (ACC32)
                acc32[u] += (float)e * (float)xv;
            else
                acc[u] += e * xv;
        }
    }
}

// Far entries of the FP64 matrix A for a tile whose targets all lie on one
// boundary and whose sources all lie on one boundary, with no near-band pair.
// With kappa = i (PR + i PI) / |D|^2 (D = E_q - E_p, PR + i PI = (E_q + E_p)
// conj(D)) and the source data pre-scaled as a = w x dx / 2, b = w x dy / 2,
// the entry times x_q is
//   Re part (surface row, wall column): -(a PI + b PR) / |D|^2,
//   the same negated (wall row, surface column),
//   Im part (rows and columns of one kind): (a PR - b PI) / |D|^2,
// less w x_q for the rank-one correction of a pair on one obstacle.
struct SrcA {
    double ex, ey, a, b;
};

template <int KIND, bool ECORR>
__device__ __forceinline__ void rows_tile_a64(const Tgt (&t)[kTPT], const SrcA *sa,
                                              const double *swx, int m, double (&acc)[kTPT]) {
    for (int i = 0; i < m; ++i) {
        const SrcA q = sa[i];
#pragma unroll
        for (int u = 0; u < kTPT; ++u) {
            const double dr = q.ex - t[u].ex, di = q.ey - t[u].ey;
            const double nr = q.ex + t[u].ex, ni = q.ey + t[u].ey;
            const double inv = recip64_from32(dr * dr + di * di);
            const double pr = nr * dr + ni * di;
            const double pi = ni * dr - nr * di;
            if (KIND == kFastReNeg) acc[u] -= (q.a * pi + q.b * pr) * inv;
            if (KIND == kFastRePos) acc[u] += (q.a * pi + q.b * pr) * inv;
            if (KIND == kFastIm) acc[u] += (q.a * pr - q.b * pi) * inv;
            if (ECORR) acc[u] -= swx[i];
        }
    }
}

template <int MODE, bool ACC32>
__global__ __launch_bounds__(256) void k_otf_rows(Nodes N, const double *hrow, int r0, int nr,
                                                  int c0, int nc,
                                                  int chunk, int corr, int nb,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ part,
                                                  const int *active) {
    if (active && *active == 0) return;
    constexpr bool FAST = MODE == 0 && !ACC32;        // specialised far tiles of A
    constexpr int kFastStage = FAST ? kOtfStage : 1;
    __shared__ Src ss[kOtfStage];
    __shared__ double sx[kOtfStage];
    __shared__ SrcA sa[kFastStage];
    __shared__ double swx[kFastStage];
    const int wb = wave_base();
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
    for (int cc = cb; cc < ce; cc += kOtfStage) {
        const int q = cc + threadIdx.x;
        if (threadIdx.x < kOtfStage && q < ce) {
            const Src sv = load_src(N, c0 + q);
            const double xv = x[q];
            ss[threadIdx.x] = sv;
            sx[threadIdx.x] = xv;
            if (FAST) {
                const double hw = 0.5 * sv.w * xv;
                sa[threadIdx.x] = SrcA{sv.ex, sv.ey, hw * sv.dx, hw * sv.dy};
                swx[threadIdx.x] = sv.w * xv;
            }
        }
        __syncthreads();
        const int m = min(kOtfStage, ce - cc);
        bool apart = true;
        int kp = -2;               // the wave's target boundary (-1: not one boundary)
#pragma unroll
        for (int u = 0; u < kTPT; ++u) {
            const int o0 = blockIdx.x * 256 * kTPT + u * 256 + wb;
            apart = apart && wave_apart<false>(N, r0, o0, nr, c0 + cc, m, nb);
            if (FAST && o0 < nr) {
                const int k = range_boundary(N, r0 + o0, r0 + min(o0 + 63, nr - 1));
                kp = (kp == -2 || kp == k) ? k : -1;
            }
        }
        const int kq = FAST ? range_boundary(N, c0 + cc, c0 + cc + m - 1) : -1;
        if (FAST && apart && kp >= 0 && kq >= 0) {
            const bool ec = corr != 0 && kp == kq && kp >= 2;
            if ((kp == 0) == (kq == 0)) {
                if (ec) rows_tile_a64<kFastIm, true>(t, sa, swx, m, acc);
                else rows_tile_a64<kFastIm, false>(t, sa, swx, m, acc);
            } else if (kp == 0) {
                rows_tile_a64<kFastReNeg, false>(t, sa, swx, m, acc);
            } else {
                rows_tile_a64<kFastRePos, false>(t, sa, swx, m, acc);
            }
        } else if (apart) {
            rows_tile<MODE, ACC32, false>(N, t, ss, sx, m, corr != 0, nb, hrow, acc, acc32);
        } else {
            rows_tile<MODE, ACC32, true>(N, t, ss, sx, m, corr != 0, nb, hrow, acc, acc32);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kTPT; ++u) {
        const int r = blockIdx.x * 256 * kTPT + u * 256 + threadIdx.x;
        if (live[u]) part[(long)blockIdx.y * nr + r] = ACC32 ? (double)acc32[u] : acc[u];
    }
}

// Transposed counterpart of rows_tile_a64: the thread's source q is fixed
// (a = w dx / 2, b = w dy / 2, E_q = (sex, sey)) and the staged targets carry
// (E_p, x_p); acc gains A(p, q) x_p for every target of the tile.
struct TgtA {
    double ex, ey, x;
};

template <int KIND, bool ECORR>
__device__ __forceinline__ void cols_tile_a64(double sex, double sey, double a, double b,
                                              double w, const TgtA *ta, int m, double &acc) {
    for (int i = 0; i < m; ++i) {
        const TgtA p = ta[i];
        const double dr = sex - p.ex, di = sey - p.ey;
        const double nr = sex + p.ex, ni = sey + p.ey;
        const double ix = recip64_from32(dr * dr + di * di) * p.x;
        const double pr = nr * dr + ni * di;
        const double pi = ni * dr - nr * di;
        if (KIND == kFastReNeg) acc -= (a * pi + b * pr) * ix;
        if (KIND == kFastRePos) acc += (a * pi + b * pr) * ix;
        if (KIND == kFastIm) acc += (a * pr - b * pi) * ix;
        if (ECORR) acc -= w * p.x;
    }
}

template <int MODE, bool ACC32, bool CHECK>
__device__ __forceinline__ void cols_tile(const Nodes &N, const Src &s, const Tgt *ts,
                                          const double *sx, int m, bool corr, int nb,
                                          const double *hrow, double &acc, float &acc32) {
    for (int i = 0; i < m; ++i) {
        const double e = entry<MODE>(N, ts[i], s, corr, CHECK ? nb : -1, hrow);
        if (ACC32)
            acc32 += (float)e * (float)sx[i];
        else
            acc += e * sx[i];
    }
}

template <int MODE, bool ACC32>
__global__ __launch_bounds__(256) void k_otf_cols(Nodes N, const double *hrow, int r0, int nr,
                                                  int c0, int nc,
                                                  int chunk, int corr, int nb,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ part,
                                                  const int *active) {
    if (active && *active == 0) return;
    constexpr bool FAST = MODE == 0 && !ACC32;        // specialised far tiles of A
    constexpr int kFastStage = FAST ? kOtfStage : 1;
    __shared__ Tgt ts[kOtfStage];
    __shared__ double sx[kOtfStage];
    __shared__ TgtA ta[kFastStage];
    const int wb = wave_base();
    const int q = blockIdx.x * 256 + threadIdx.x;
    const bool live = q < nc;
    Src s;
    if (live) s = load_src(N, c0 + q);
    const double fa = live ? 0.5 * s.w * s.dx : 0.0, fb = live ? 0.5 * s.w * s.dy : 0.0;
    // the wave's source boundary (-1: the wave's columns cross a boundary end)
    const int o0 = blockIdx.x * 256 + wb;
    const int kq = (FAST && o0 < nc) ? range_boundary(N, c0 + o0, c0 + min(o0 + 63, nc - 1)) : -1;
    const int pb = blockIdx.y * chunk;
    const int pe = min(nr, pb + chunk);
    double acc = 0.0;
    float acc32 = 0.0f;
    for (int pp = pb; pp < pe; pp += kOtfStage) {
        const int p = pp + threadIdx.x;
        if (threadIdx.x < kOtfStage && p < pe) {
            const Tgt tv = load_tgt(N, r0 + p);
            const double xv = x[p];
            ts[threadIdx.x] = tv;
            sx[threadIdx.x] = xv;
            if (FAST) ta[threadIdx.x] = TgtA{tv.ex, tv.ey, xv};
        }
        __syncthreads();
        const int m = min(kOtfStage, pe - pp);
        const bool apart = wave_apart<true>(N, c0, o0, nc, r0 + pp, m, nb);
        const int kp = (FAST && kq >= 0) ? range_boundary(N, r0 + pp, r0 + pp + m - 1) : -1;
        if (live) {
            if (FAST && apart && kp >= 0 && kq >= 0) {
                const double w = s.w;
                if ((kp == 0) == (kq == 0)) {
                    if (corr != 0 && kp == kq && kp >= 2)
                        cols_tile_a64<kFastIm, true>(s.ex, s.ey, fa, fb, w, ta, m, acc);
                    else
                        cols_tile_a64<kFastIm, false>(s.ex, s.ey, fa, fb, w, ta, m, acc);
                } else if (kp == 0) {
                    cols_tile_a64<kFastReNeg, false>(s.ex, s.ey, fa, fb, w, ta, m, acc);
                } else {
                    cols_tile_a64<kFastRePos, false>(s.ex, s.ey, fa, fb, w, ta, m, acc);
                }
            } else if (apart) {
                cols_tile<MODE, ACC32, false>(N, s, ts, sx, m, corr != 0, nb, hrow, acc, acc32);
            } else {
                cols_tile<MODE, ACC32, true>(N, s, ts, sx, m, corr != 0, nb, hrow, acc, acc32);
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

// Chunk of the summed index for an on-the-fly product with `nout` outputs
// (`per_block` of them per block) and `nsum` summed indices: enough chunks
// for about kOtfBlocks blocks, a multiple of 32 indices, at most
// kOtfMaxSlices chunks.
static int split_chunk(int nout, int nsum, int per_block) {
    const int ob = cdiv(nout, per_block);
    int ns = cdiv(kOtfBlocks, ob);
    ns = ns < 1 ? 1 : (ns > kOtfMaxSlices ? kOtfMaxSlices : ns);
    int c = cdiv(nsum, ns);
    c = cdiv(c, 32) * 32;
    return c < 32 ? 32 : c;
}
static int rows_chunk(int nr, int nc) { return split_chunk(nr, nc, 256 * kTPT); }
static int cols_chunk(int nr, int nc) { return split_chunk(nc, nr, 256); }

int rflavour_nsplit(int nr, int nc, int transpose) {
    return transpose ? cdiv(nr, cols_chunk(nr, nc)) + 1 : cdiv(nc, rows_chunk(nr, nc)) + 1;
}

void launch_assemble64(const Layout &L, const Nodes &N, int flags, double *A, long ld,
                       hipStream_t st) {
    const int n = L.n;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsmBlock));
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    hipLaunchKernelGGL(k_assemble<0>, grid, dim3(256), 0, st, N, nullptr, 0, n, 0, n, corr, A, ld);
}

void launch_assemble32(const Layout &L, const Nodes &N, int flags, int band, float *A, long ld,
                       hipStream_t st) {
    const int n = L.n;
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsm32));
    hipLaunchKernelGGL(k_assemble32_far, grid, dim3(256), 0, st, N, n, corr, band, A, ld);
    const long nbw = (long)n * (2 * band + 1);
    hipLaunchKernelGGL(k_assemble32_band<false>, dim3(cdiv(nbw, 256)), dim3(256), 0, st, N, n,
                       corr, band, A, ld);
}

void launch_assemble32_T(const Layout &L, const Nodes &N, int flags, int band, float *AT,
                         long ld, hipStream_t st) {
    const int n = L.n;
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsm32));
    hipLaunchKernelGGL(k_assemble32T_far, grid, dim3(256), 0, st, N, n, corr, band, AT, ld);
    const long nbw = (long)n * (2 * band + 1);
    hipLaunchKernelGGL(k_assemble32_band<true>, dim3(cdiv(nbw, 256)), dim3(256), 0, st, N, n,
                       corr, band, AT, ld);
}

void launch_assemble64_T(const Layout &L, const Nodes &N, int flags, double *AT, long ld,
                         hipStream_t st) {
    const int n = L.n;
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsmBlock));
    hipLaunchKernelGGL(k_assemble64T, grid, dim3(256), 0, st, N, n, corr, AT, ld);
}

void launch_assemble_gt64(const Layout &L, const Nodes &N, double *B, long ld, hipStream_t st) {
    const int n = L.n;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsmBlock));
    hipLaunchKernelGGL(k_assemble<2>, grid, dim3(256), 0, st, N, nullptr, 0, n, 0, n, 1, B, ld);
}

void launch_assemble_gt32(const Layout &L, const Nodes &N, float *B, long ld, hipStream_t st) {
    const int n = L.n;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsmBlock));
    hipLaunchKernelGGL((k_assemble<2, float>), grid, dim3(256), 0, st, N, nullptr, 0, n, 0, n, 1,
                       B, ld);
}

void launch_assemble_T64(const Layout &L, const Nodes &N, const double *hrow, double *T, long ld,
                         hipStream_t st) {
    const int n = L.n, n0 = L.off[1];
    dim3 grid(cdiv(ld, 256), cdiv(n0, kRowsPerAsmBlock));
    hipLaunchKernelGGL(k_assemble<3>, grid, dim3(256), 0, st, N, hrow, 0, n0, 0, n, 1, T, ld);
}

void launch_assemble_wall64(const Layout &L, const Nodes &N, const double *hrow, double *W, long ld,
                            hipStream_t st) {
    const int c0 = L.off[1], nw = L.n - L.off[1];
    dim3 grid(cdiv(ld, 256), cdiv(nw, kRowsPerAsmBlock));
    hipLaunchKernelGGL(k_assemble<1>, grid, dim3(256), 0, st, N, hrow, c0, nw, c0, nw, 1, W, ld);
}

void launch_assemble_wall32(const Layout &L, const Nodes &N, const double *hrow, float *W, long ld,
                            hipStream_t st) {
    const int c0 = L.off[1], nw = L.n - L.off[1];
    dim3 grid(cdiv(ld, 256), cdiv(nw, kRowsPerAsmBlock));
    hipLaunchKernelGGL((k_assemble<1, float>), grid, dim3(256), 0, st, N, hrow, c0, nw, c0, nw, 1,
                       W, ld);
}

static int near_width(int band) { return band > kNearBand ? band : kNearBand; }

void launch_otf_matvec(const Layout &L, const Nodes &N, int flags, int fp32, int band,
                       int transpose, const double *x, const double *c, double *y, double *part,
                       const int *active, hipStream_t st) {
    const double *hrow = nullptr;
    const int n = L.n;
    const int chunk = transpose ? cols_chunk(n, n) : rows_chunk(n, n);
    const int ns = cdiv(n, chunk);
    const int nb = near_width(band);
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    dim3 grid(cdiv(n, 256), ns);
    dim3 gridr(cdiv(n, 256 * kTPT), ns);
    const dim3 gnear(cdiv(n, kNearPerBlock));
    double *near = part + (long)ns * n;
    if (!transpose) {
        if (fp32) {
            hipLaunchKernelGGL((k_otf_rows<1, true>), gridr, dim3(256), 0, st, N, hrow, 0, n, 0, n,
                               chunk, corr, nb, x, part, active);
            hipLaunchKernelGGL((k_near_band<1, false>), gnear, dim3(256), 0, st, N,
                               hrow, 0, n, 0, n, corr, band, nb, x, near, active);
        } else {
            hipLaunchKernelGGL((k_otf_rows<0, false>), gridr, dim3(256), 0, st, N, hrow, 0, n, 0, n,
                               chunk, corr, nb, x, part, active);
            hipLaunchKernelGGL((k_near_band<0, false>), gnear, dim3(256), 0, st, N,
                               hrow, 0, n, 0, n, corr, band, nb, x, near, active);
        }
    } else {
        if (fp32) {
            hipLaunchKernelGGL((k_otf_cols<1, true>), grid, dim3(256), 0, st, N, hrow, 0, n, 0, n,
                               chunk, corr, nb, x, part, active);
            hipLaunchKernelGGL((k_near_band<1, true>), gnear, dim3(256), 0, st, N,
                               hrow, 0, n, 0, n, corr, band, nb, x, near, active);
        } else {
            hipLaunchKernelGGL((k_otf_cols<0, false>), grid, dim3(256), 0, st, N, hrow, 0, n, 0, n,
                               chunk, corr, nb, x, part, active);
            hipLaunchKernelGGL((k_near_band<0, true>), gnear, dim3(256), 0, st, N,
                               hrow, 0, n, 0, n, corr, band, nb, x, near, active);
        }
    }
    launch_reduce_partials(n, part, ns + 1, c, 1.0, y, active, st);
}


template <int MODE>
static void rflavour_mode(const Nodes &N, const double *hrow, int transpose, int r0, int nr,
                          int c0, int nc, const double *x, double *part, const int *active,
                          hipStream_t st) {
    const int nb = kNearBand;
    if (!transpose) {
        const int chunk = rows_chunk(nr, nc);
        const int ns = cdiv(nc, chunk);
        dim3 grid(cdiv(nr, 256 * kTPT), ns);
        hipLaunchKernelGGL((k_otf_rows<MODE, false>), grid, dim3(256), 0, st, N, hrow, r0, nr, c0,
                           nc, chunk, 1, nb, x, part, active);
        hipLaunchKernelGGL((k_near_band<MODE, false>), dim3(cdiv(nr, kNearPerBlock)), dim3(256), 0,
                           st, N, hrow, r0, nr, c0, nc, 1, 0, nb, x, part + (long)ns * nr,
                           active);
    } else {
        const int chunk = cols_chunk(nr, nc);
        const int ns = cdiv(nr, chunk);
        dim3 grid(cdiv(nc, 256), ns);
        hipLaunchKernelGGL((k_otf_cols<MODE, false>), grid, dim3(256), 0, st, N, hrow, r0, nr, c0,
                           nc, chunk, 1, nb, x, part, active);
        hipLaunchKernelGGL((k_near_band<MODE, true>), dim3(cdiv(nc, kNearPerBlock)), dim3(256), 0,
                           st, N, hrow, r0, nr, c0, nc, 1, 0, nb, x, part + (long)ns * nc,
                           active);
    }
}

void launch_rflavour(const Layout &L, const Nodes &N, const double *hrow, int mode, int transpose,
                     int r0, int nr, int c0, int nc, const double *x, double *part,
                     const int *active, hipStream_t st) {
    (void)L;
    switch (mode) {
    case 3: rflavour_mode<3>(N, hrow, transpose, r0, nr, c0, nc, x, part, active, st); break;
    case 4: rflavour_mode<4>(N, hrow, transpose, r0, nr, c0, nc, x, part, active, st); break;
    case 5: rflavour_mode<5>(N, hrow, transpose, r0, nr, c0, nc, x, part, active, st); break;
    case 6: rflavour_mode<6>(N, hrow, transpose, r0, nr, c0, nc, x, part, active, st); break;
    case 7: rflavour_mode<7>(N, hrow, transpose, r0, nr, c0, nc, x, part, active, st); break;
    case 8: rflavour_mode<8>(N, hrow, transpose, r0, nr, c0, nc, x, part, active, st); break;
    default: rflavour_mode<2>(N, hrow, transpose, r0, nr, c0, nc, x, part, active, st); break;
    }
}

}  // namespace wwbi
