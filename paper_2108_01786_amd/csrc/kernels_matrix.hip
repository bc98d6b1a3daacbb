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
constexpr int kOtfMaxSlices = 256;   // at most this many far slices (+ near band and near fix)

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

// Smallest distance between two discs of E values (centre, radius) against
// the cut |E| / f of the larger |E| (a relative margin covers the rounding of
// the discs): false when no pair of the two cells is closer than the cut.
__device__ __forceinline__ bool discs_within(const double *a, const double *b, double f) {
    const double gx = a[0] - b[0], gy = a[1] - b[1];
    return (sqrt(gx * gx + gy * gy) - a[2] - b[2]) * f < 1.001 * max(a[3], b[3]);
}
__device__ __forceinline__ bool discs_may_be_near(const double *a, const double *b) {
    return discs_within(a, b, kNearCut);
}

// True when every pair of target nodes [pa, pb] and source nodes [qa, qb] is
// at least |E_p| / 4 apart in E (tested on the 64-node cells' discs).  The far
// tiles of A then form E_q - E_p from the leading parts of E alone: its
// relative error stays below about 8 units of rounding, against 2 with the
// trailing parts, which nearer pairs need.
__device__ __forceinline__ bool cells_far(const Nodes &N, int pa, int pb, int qa, int qb) {
    for (int a = pa / kCellNodes; a <= pb / kCellNodes; ++a)
        for (int b = qa / kCellNodes; b <= qb / kCellNodes; ++b)
            if (discs_within(N.cell + 4 * a, N.cell + 4 * b, 4.0)) return false;
    return true;
}

// FP64 assembly of A.  One column per thread and kRowsPerAsm64 rows per
// block, as in the FP32 far pass.  A wave whose live columns lie on one
// boundary, in a block whose rows lie on one boundary, clear of the
// same-boundary band and, by the 64-node cells' E discs, of every near pair,
// takes the E quotient with one entry formula for the whole tile: the source
// data pre-scaled (a = w dx / 2, b = w dy / 2), the reciprocal of |D|^2 from
// the FP32 estimate refined twice, and E's trailing parts only where the
// discs come within |E| / 4 (cells_far).  Every other wave takes a_val64,
// the full entry (band, near pairs, diagonal limits).
constexpr int kRowsPerAsm64 = 32;

template <int KIND, bool LO>
__device__ __forceinline__ double a_fast64(const Tgt &t, const Src &s, double fa, double fb,
                                           double ec) {
    const double dr = LO ? (s.ex - t.ex) + (s.exl - t.exl) : s.ex - t.ex;
    const double di = LO ? (s.ey - t.ey) + (s.eyl - t.eyl) : s.ey - t.ey;
    const double nr = s.ex + t.ex, ni = s.ey + t.ey;
    const double inv = recip64_from32(dr * dr + di * di);
    const double pr = nr * dr + ni * di;
    const double pi = ni * dr - nr * di;
    if (KIND == kFastReNeg) return -(fa * pi + fb * pr) * inv;
    if (KIND == kFastRePos) return (fa * pi + fb * pr) * inv;
    return (fa * pr - fb * pi) * inv - ec;
}

template <int KIND, bool LO>
__device__ __forceinline__ void asm64_tile(const Tgt *tg, int rend, const Src &s, double fa,
                                           double fb, double ec, bool live, double *o, long ld) {
    for (int i = 0; i < rend; ++i)
        __builtin_nontemporal_store(live ? a_fast64<KIND, LO>(tg[i], s, fa, fb, ec) : 0.0,
                                    o + i * ld);
}

__global__ __launch_bounds__(256) void k_assemble64(Nodes N, int n, int corr, double *out,
                                                    long ld) {
    __shared__ Tgt tg[kRowsPerAsm64];
    const int wb = wave_base();
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int rbase = blockIdx.y * kRowsPerAsm64;
    if (threadIdx.x < kRowsPerAsm64) {
        const int r = rbase + threadIdx.x;
        if (r < n) tg[threadIdx.x] = load_tgt(N, r);
    }
    __syncthreads();
    if (col >= ld) return;
    const bool live = col < n;
    const Src s = load_src(N, live ? col : 0);
    const int rend = min(kRowsPerAsm64, n - rbase);
    double *o = out + (long)rbase * ld + col;
    // the wave's live columns [ca, cb] and the block's rows, each on one
    // boundary, clear of the band and of near pairs (wave-uniform tests)
    const int ca = blockIdx.x * 256 + wb, cb = min(ca + 63, n - 1);
    const int re = rbase + rend - 1;
    int kq = -1, kr = -1;
    if (ca < n) {
        kq = range_boundary(N, ca, cb);
        kr = range_boundary(N, rbase, re);
    }
    bool fast = kq >= 0 && kr >= 0 && ranges_apart(N, rbase, re, ca, cb, kNearBand);
    for (int a = rbase / kCellNodes; fast && a <= re / kCellNodes; ++a)
        for (int b = ca / kCellNodes; fast && b <= cb / kCellNodes; ++b)
            fast = !discs_may_be_near(N.cell + 4 * a, N.cell + 4 * b);
    if (fast) {
        const double fa = 0.5 * s.w * s.dx, fb = 0.5 * s.w * s.dy;
        const double ec = (corr && kr == kq && kr >= 2) ? s.w : 0.0;
        const bool lo = !cells_far(N, rbase, re, ca, cb);
        if ((kr == 0) == (kq == 0)) {
            if (lo) asm64_tile<kFastIm, true>(tg, rend, s, fa, fb, ec, live, o, ld);
            else asm64_tile<kFastIm, false>(tg, rend, s, fa, fb, ec, live, o, ld);
        } else if (kr == 0) {
            if (lo) asm64_tile<kFastReNeg, true>(tg, rend, s, fa, fb, 0.0, live, o, ld);
            else asm64_tile<kFastReNeg, false>(tg, rend, s, fa, fb, 0.0, live, o, ld);
        } else {
            if (lo) asm64_tile<kFastRePos, true>(tg, rend, s, fa, fb, 0.0, live, o, ld);
            else asm64_tile<kFastRePos, false>(tg, rend, s, fa, fb, 0.0, live, o, ld);
        }
        return;
    }
    for (int i = 0; i < rend; ++i)
        __builtin_nontemporal_store(live ? a_val64(N, tg[i], s, corr != 0) : 0.0, o + i * ld);
}

// Near pairs outside the band.  The far loops of the on-the-fly products
// take kappa from the E quotient for every pair outside the same-boundary
// band; a pair closer than |E_q - E_p| < max(|E_p|, |E_q|) / 64 (kappa64's
// near test: two boundaries that come close, or one boundary folding back
// towards itself) needs the half-angle formula instead.  E is periodic, so
// distances between E values cover every period image.
//
// Once per geometry, k_near_cells lists for every 64-node cell a the cells b
// holding a node q that forms a near pair outside the band with a node of a
// (at most kNearList of them, in increasing order; more, and the list is
// marked full).  The relation is symmetric.  Each product then adds, as one
// more partial slice, (full entry - far entry) x for exactly those pairs
// (k_near_fix), visiting only the listed cells.
constexpr int kMaxScanCells = 1024;        // cells tested per pass of the full scan

// The pair test shared by the list build and the fix: outside the band of
// `nb` steps (by index: me's boundary starts at mbase, has mM nodes, me is
// node mloc of it) and inside the near cut.
__device__ __forceinline__ bool near_pair(int q, int mbase, int mloc, int mM, int nb, double ex,
                                          double ey, double exl, double eyl, double qx, double qy,
                                          double qxl, double qyl) {
    const int l = q - mbase;
    if (l >= 0 && l < mM && cyc_dist(l, mloc, mM) <= nb) return false;
    const double dr = (qx - ex) + (qxl - exl);
    const double di = (qy - ey) + (qyl - eyl);
    return (dr * dr + di * di) * (kNearCut * kNearCut) < max(ex * ex + ey * ey, qx * qx + qy * qy);
}

// Ordered list, in LDS, of the cells of [c0, c0 + cn) whose discs come within
// the near cut of disc `d` (cn <= kMaxScanCells); returns its length.  Every
// thread of the block calls it.
__device__ int list_disc_cells(const Nodes &N, const double *d, int c0, int cn, int *list,
                               int *wcnt) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int nl = 0;
    for (int j0 = 0; j0 < cn; j0 += 256) {
        const int j = j0 + (int)threadIdx.x;
        const bool f = j < cn && discs_may_be_near(N.cell + 4 * (long)(c0 + j), d);
        const unsigned long long bal = __ballot(f);
        if (lane == 0) wcnt[wv] = __popcll(bal);
        __syncthreads();
        int before = nl;
        for (int w = 0; w < wv; ++w) before += wcnt[w];
        if (f) list[before + __popcll(bal & ((1ull << lane) - 1ull))] = c0 + j;
        nl += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
    return nl;
}

// Stage the E values of cell b's nodes in LDS (threads 0..63; clamped to the
// last node).  Every thread of the block calls it.
__device__ __forceinline__ void stage_cell(const Nodes &N, int b, double (*se)[kCellNodes]) {
    __syncthreads();
    if (threadIdx.x < kCellNodes) {
        const int q = min(b * kCellNodes + (int)threadIdx.x, N.n - 1);
        se[0][threadIdx.x] = N.ex[q];
        se[1][threadIdx.x] = N.ey[q];
        se[2][threadIdx.x] = N.exl[q];
        se[3][threadIdx.x] = N.eyl[q];
    }
    __syncthreads();
}

// One block per cell a: its list, and the number of near pairs (p in a, any
// q) added into *count.
__global__ __launch_bounds__(256) void k_near_cells(Nodes N, int nb, int *lists, double *count) {
    __shared__ int list[kMaxScanCells];
    __shared__ int wcnt[4];
    __shared__ int hit;
    __shared__ double se[4][kCellNodes];
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int a = blockIdx.x;
    const int p = a * kCellNodes + lane;
    const bool live = p < N.n;
    const int me = live ? p : a * kCellNodes;
    const double ex = N.ex[me], ey = N.ey[me], exl = N.exl[me], eyl = N.eyl[me];
    const int mloc = N.loc[me], mM = N.Mk[me], mbase = me - mloc;
    const double *da = N.cell + 4 * a;
    const int ncell = (N.n + kCellNodes - 1) / kCellNodes;
    int nfound = 0;
    bool full = false;
    double pairs = 0.0;
    for (int c0 = 0; c0 < ncell; c0 += kMaxScanCells) {
        __syncthreads();
        const int nl = list_disc_cells(N, da, c0, min(kMaxScanCells, ncell - c0), list, wcnt);
        for (int li = 0; li < nl; ++li) {
            const int b = list[li];
            if (threadIdx.x == 0) hit = 0;
            stage_cell(N, b, se);
            int mine = 0;
            if (live) {
                for (int jj = 16 * wv; jj < 16 * wv + 16; ++jj) {
                    const int q = b * kCellNodes + jj;
                    if (q >= N.n) break;
                    mine += near_pair(q, mbase, mloc, mM, nb, ex, ey, exl, eyl, se[0][jj],
                                      se[1][jj], se[2][jj], se[3][jj]) ? 1 : 0;
                }
            }
            if (mine) atomicOr(&hit, 1);
            pairs += (double)mine;
            __syncthreads();
            const bool h = hit != 0;
            __syncthreads();                // every thread has read hit before it is reset
            if (h) {
                if (nfound < kNearList) {
                    if (threadIdx.x == 0) lists[(long)a * kNearStride + 1 + nfound] = b;
                    ++nfound;
                } else {
                    full = true;
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) pairs += __shfl_xor(pairs, o, 64);
    if (lane == 0) red[wv] = pairs;
    __syncthreads();
    if (threadIdx.x == 0) {
        lists[(long)a * kNearStride] = full ? -1 : nfound;
        const double tot = ((red[0] + red[1]) + red[2]) + red[3];
        if (tot > 0.0) atomicAdd(count, tot);       // integer counts: exact in any order
    }
}

// Everything the entries need of one node, staged in LDS by the fix kernel.
struct NodeRec {
    double ex, ey, exl, eyl, dx, dy, w, lre, lim, x, y;
    int k, loc, M;
};
__device__ __forceinline__ NodeRec load_rec(const Nodes &N, int q) {
    return NodeRec{N.ex[q], N.ey[q], N.exl[q], N.eyl[q], N.dx[q], N.dy[q], N.w[q], N.lre[q],
                   N.lim[q], N.x[q], N.y[q], N.bid[q], N.loc[q], N.Mk[q]};
}
__device__ __forceinline__ Src rec_src(const NodeRec &r, int q) {
    Src s;
    s.ex = r.ex; s.ey = r.ey; s.exl = r.exl; s.eyl = r.eyl; s.dx = r.dx; s.dy = r.dy;
    s.w = r.w; s.x = r.x; s.y = r.y; s.k = r.k; s.loc = r.loc; s.M = r.M; s.idx = q;
    return s;
}
__device__ __forceinline__ Tgt rec_tgt(const NodeRec &r, int p) {
    Tgt t;
    t.ex = r.ex; t.ey = r.ey; t.exl = r.exl; t.eyl = r.eyl; t.dx = r.dx; t.dy = r.dy;
    t.lre = r.lre; t.lim = r.lim; t.x = r.x; t.y = r.y; t.k = r.k; t.loc = r.loc; t.M = r.M;
    t.idx = p;
    return t;
}

// The fix slice: one block per 64-node cell a overlapping the outputs, one
// output (node 64 a + lane) per lane; wave w takes nodes 16 w .. 16 w + 15 of
// every visited cell for every output, and the waves' sums are added in a
// fixed order.  A full list falls back to scanning every cell whose disc
// comes within the cut.
template <int MODE, bool COLS>
__global__ __launch_bounds__(256) void k_near_fix(Nodes N, const int *lists, const double *hrow,
                                                  int r0, int nr, int c0, int nc, int corr,
                                                  int band, int nb,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ out, const int *active) {
    if (active && *active == 0) return;
    __shared__ int list[kMaxScanCells];
    __shared__ int wcnt[4];
    __shared__ NodeRec rec[kCellNodes];
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int obase = COLS ? c0 : r0, nout = COLS ? nc : nr;
    const int sbase = COLS ? r0 : c0, nsum = COLS ? nr : nc;
    const int a = obase / kCellNodes + blockIdx.x;
    const int p = a * kCellNodes + lane;
    const bool live = p >= obase && p < obase + nout;
    const int me = live ? p : max(obase, a * kCellNodes);
    const NodeRec mr = load_rec(N, me);
    const Tgt mt = rec_tgt(mr, me);
    const Src ms = rec_src(mr, me);
    const int mbase = me - mr.loc;
    const int *la = lists + (long)a * kNearStride;
    const int cnt = la[0];
    double acc = 0.0;
    const int cfirst = sbase / kCellNodes, clast = (sbase + nsum - 1) / kCellNodes;
    for (int cs = cnt < 0 ? cfirst : 0; cs <= (cnt < 0 ? clast : 0); cs += kMaxScanCells) {
        int nl;
        const int *cells;
        if (cnt < 0) {
            __syncthreads();
            nl = list_disc_cells(N, N.cell + 4 * a, cs, min(kMaxScanCells, clast - cs + 1), list,
                                 wcnt);
            cells = list;
        } else {
            nl = cnt;
            cells = la + 1;
        }
        for (int li = 0; li < nl; ++li) {
            const int b = cells[li];
            if (b < cfirst || b > clast) continue;        // block-uniform
            __syncthreads();
            if (threadIdx.x < kCellNodes)
                rec[threadIdx.x] = load_rec(N, min(b * kCellNodes + (int)threadIdx.x, N.n - 1));
            __syncthreads();
            if (!live) continue;
            for (int jj = 16 * wv; jj < 16 * wv + 16; ++jj) {
                const int q = b * kCellNodes + jj;
                if (q < sbase || q >= sbase + nsum) continue;
                const NodeRec &r = rec[jj];
                if (!near_pair(q, mbase, mr.loc, mr.M, nb, mr.ex, mr.ey, mr.exl, mr.eyl, r.ex,
                               r.ey, r.exl, r.eyl))
                    continue;
                const Tgt t = COLS ? rec_tgt(r, q) : mt;
                const Src s = COLS ? ms : rec_src(r, q);
                const double e = entry_full<MODE>(N, t, s, corr != 0, band, hrow) -
                                 entry<MODE>(N, t, s, corr != 0, -1, hrow);
                acc += e * x[q - sbase];
            }
        }
    }
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && live)
        out[p - obase] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
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
    double ex, ey, exl, eyl, a, b;
};

template <int KIND, bool ECORR, bool LO>
__device__ __forceinline__ void rows_tile_a64(const Tgt (&t)[kTPT], const SrcA *sa,
                                              const double *swx, int m, double (&acc)[kTPT]) {
    for (int i = 0; i < m; ++i) {
        const SrcA q = sa[i];
#pragma unroll
        for (int u = 0; u < kTPT; ++u) {
            const double dr = LO ? (q.ex - t[u].ex) + (q.exl - t[u].exl) : q.ex - t[u].ex;
            const double di = LO ? (q.ey - t[u].ey) + (q.eyl - t[u].eyl) : q.ey - t[u].ey;
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

// Far entries of the normal-velocity map T (targets on the surface) for a
// tile whose sources all lie on one boundary, with no near-band pair.  With
// the same quotient and the target data halved (a = dx_p / 2, b = dy_p / 2),
// the entry times x_q is w_q x_q times
//   surface source: (a PI + b PR) / |D|^2 + h((alpha_q - alpha_p)),
//   wall source:   -(a PR - b PI) / |D|^2,
// h read from the surface's table (for one source, the wave's consecutive
// targets read consecutive entries).
struct SrcT {
    double ex, ey, exl, eyl, wx;
    int loc;
};

template <bool SURF, bool LO>
__device__ __forceinline__ void rows_tile_t64(const Tgt (&t)[kTPT], const SrcT *sv, int m,
                                              const double *hrow, double (&acc)[kTPT]) {
    double ta[kTPT], tb[kTPT];
#pragma unroll
    for (int u = 0; u < kTPT; ++u) { ta[u] = 0.5 * t[u].dx; tb[u] = 0.5 * t[u].dy; }
    for (int i = 0; i < m; ++i) {
        const SrcT q = sv[i];
#pragma unroll
        for (int u = 0; u < kTPT; ++u) {
            const double dr = LO ? (q.ex - t[u].ex) + (q.exl - t[u].exl) : q.ex - t[u].ex;
            const double di = LO ? (q.ey - t[u].ey) + (q.eyl - t[u].eyl) : q.ey - t[u].ey;
            const double nr = q.ex + t[u].ex, ni = q.ey + t[u].ey;
            const double inv = recip64_from32(dr * dr + di * di);
            const double pr = nr * dr + ni * di;
            const double pi = ni * dr - nr * di;
            if (SURF) {
                int d = q.loc - t[u].loc;
                if (d < 0) d += t[u].M;
                acc[u] += q.wx * ((ta[u] * pi + tb[u] * pr) * inv + hrow[d]);
            } else {
                acc[u] -= q.wx * ((ta[u] * pr - tb[u] * pi) * inv);
            }
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
    // specialised far tiles of A and of T
    constexpr bool FAST = (MODE == 0 || MODE == 2) && !ACC32;
    constexpr int kStageA = FAST && MODE == 0 ? kOtfStage : 1;
    constexpr int kStageT = FAST && MODE == 2 ? kOtfStage : 1;
    __shared__ Src ss[kOtfStage];
    __shared__ double sx[kOtfStage];
    __shared__ SrcA sa[kStageA];
    __shared__ double swx[kStageA];
    __shared__ SrcT stt[kStageT];
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
            if constexpr (FAST && MODE == 0) {
                const double hw = 0.5 * sv.w * xv;
                sa[threadIdx.x] = SrcA{sv.ex, sv.ey, sv.exl, sv.eyl, hw * sv.dx, hw * sv.dy};
                swx[threadIdx.x] = sv.w * xv;
            }
            if constexpr (FAST && MODE == 2)
                stt[threadIdx.x] = SrcT{sv.ex, sv.ey, sv.exl, sv.eyl, sv.w * xv, sv.loc};
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
        if (FAST && apart && kp >= 0 && kq >= 0 && (MODE == 0 || kp == 0)) {
            const bool ec = corr != 0 && kp == kq && kp >= 2;
            const int o0 = blockIdx.x * 256 * kTPT + wb;
            const bool lo = o0 >= nr || !cells_far(N, r0 + o0, r0 + min(o0 + 256 * (kTPT - 1) + 63,
                                                                         nr - 1),
                                                   c0 + cc, c0 + cc + m - 1);
            if constexpr (MODE == 2) {
                if (kq == 0) {
                    if (lo) rows_tile_t64<true, true>(t, stt, m, hrow, acc);
                    else rows_tile_t64<true, false>(t, stt, m, hrow, acc);
                } else {
                    if (lo) rows_tile_t64<false, true>(t, stt, m, hrow, acc);
                    else rows_tile_t64<false, false>(t, stt, m, hrow, acc);
                }
            } else if (lo) {
                if ((kp == 0) == (kq == 0)) {
                    if (ec) rows_tile_a64<kFastIm, true, true>(t, sa, swx, m, acc);
                    else rows_tile_a64<kFastIm, false, true>(t, sa, swx, m, acc);
                } else if (kp == 0) {
                    rows_tile_a64<kFastReNeg, false, true>(t, sa, swx, m, acc);
                } else {
                    rows_tile_a64<kFastRePos, false, true>(t, sa, swx, m, acc);
                }
            } else {
                if ((kp == 0) == (kq == 0)) {
                    if (ec) rows_tile_a64<kFastIm, true, false>(t, sa, swx, m, acc);
                    else rows_tile_a64<kFastIm, false, false>(t, sa, swx, m, acc);
                } else if (kp == 0) {
                    rows_tile_a64<kFastReNeg, false, false>(t, sa, swx, m, acc);
                } else {
                    rows_tile_a64<kFastRePos, false, false>(t, sa, swx, m, acc);
                }
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
    double ex, ey, exl, eyl, x;
};

template <int KIND, bool ECORR, bool LO>
__device__ __forceinline__ void cols_tile_a64(double sex, double sey, double sexl, double seyl,
                                              double a, double b, double w, const TgtA *ta, int m,
                                              double &acc) {
    for (int i = 0; i < m; ++i) {
        const TgtA p = ta[i];
        const double dr = LO ? (sex - p.ex) + (sexl - p.exl) : sex - p.ex;
        const double di = LO ? (sey - p.ey) + (seyl - p.eyl) : sey - p.ey;
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
            if (FAST) ta[threadIdx.x] = TgtA{tv.ex, tv.ey, tv.exl, tv.eyl, xv};
        }
        __syncthreads();
        const int m = min(kOtfStage, pe - pp);
        const bool apart = wave_apart<true>(N, c0, o0, nc, r0 + pp, m, nb);
        const int kp = (FAST && kq >= 0) ? range_boundary(N, r0 + pp, r0 + pp + m - 1) : -1;
        const bool lo = FAST && kp >= 0 && kq >= 0 &&
                        (o0 >= nc || !cells_far(N, r0 + pp, r0 + pp + m - 1, c0 + o0,
                                                 c0 + min(o0 + 63, nc - 1)));
        if (live) {
            if (FAST && apart && kp >= 0 && kq >= 0) {
                const double w = s.w;
                const bool ec = corr != 0 && kp == kq && kp >= 2;
                if (lo) {
                    if ((kp == 0) == (kq == 0)) {
                        if (ec)
                            cols_tile_a64<kFastIm, true, true>(s.ex, s.ey, s.exl, s.eyl, fa, fb,
                                                               w, ta, m, acc);
                        else
                            cols_tile_a64<kFastIm, false, true>(s.ex, s.ey, s.exl, s.eyl, fa, fb,
                                                                w, ta, m, acc);
                    } else if (kp == 0) {
                        cols_tile_a64<kFastReNeg, false, true>(s.ex, s.ey, s.exl, s.eyl, fa, fb,
                                                               w, ta, m, acc);
                    } else {
                        cols_tile_a64<kFastRePos, false, true>(s.ex, s.ey, s.exl, s.eyl, fa, fb,
                                                               w, ta, m, acc);
                    }
                } else {
                    if ((kp == 0) == (kq == 0)) {
                        if (ec)
                            cols_tile_a64<kFastIm, true, false>(s.ex, s.ey, s.exl, s.eyl, fa, fb,
                                                                w, ta, m, acc);
                        else
                            cols_tile_a64<kFastIm, false, false>(s.ex, s.ey, s.exl, s.eyl, fa,
                                                                 fb, w, ta, m, acc);
                    } else if (kp == 0) {
                        cols_tile_a64<kFastReNeg, false, false>(s.ex, s.ey, s.exl, s.eyl, fa, fb,
                                                                w, ta, m, acc);
                    } else {
                        cols_tile_a64<kFastRePos, false, false>(s.ex, s.ey, s.exl, s.eyl, fa, fb,
                                                                w, ta, m, acc);
                    }
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

// Disc of the E values of every cell of kCellNodes consecutive nodes: the
// centre and half-diagonal of their bounding box, and the largest |E|; one
// wave per cell.
__global__ __launch_bounds__(256) void k_cells(Nodes N, double *cell) {
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int a = c * kCellNodes;
    if (a >= N.n) return;
    const int q = min(a + (int)(threadIdx.x & 63), N.n - 1);
    const double ex = N.ex[q], ey = N.ey[q];
    double xlo = ex, xhi = ex, ylo = ey, yhi = ey, amax = ex * ex + ey * ey;
    for (int o = 32; o > 0; o >>= 1) {
        xlo = min(xlo, __shfl_xor(xlo, o, 64));
        xhi = max(xhi, __shfl_xor(xhi, o, 64));
        ylo = min(ylo, __shfl_xor(ylo, o, 64));
        yhi = max(yhi, __shfl_xor(yhi, o, 64));
        amax = max(amax, __shfl_xor(amax, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        cell[4 * c] = 0.5 * (xlo + xhi);
        cell[4 * c + 1] = 0.5 * (ylo + yhi);
        cell[4 * c + 2] = 0.5 * sqrt((xhi - xlo) * (xhi - xlo) + (yhi - ylo) * (yhi - ylo));
        cell[4 * c + 3] = sqrt(amax);
    }
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

// Partial slices of an on-the-fly product of modes 2..8: the far chunks, the
// near band and, when the geometry has near pairs, the near-pair fix.
int rflavour_nsplit(const Nodes &N, int nr, int nc, int transpose) {
    const int fix = N.near ? 2 : 1;
    return transpose ? cdiv(nr, cols_chunk(nr, nc)) + fix : cdiv(nc, rows_chunk(nr, nc)) + fix;
}

void launch_cells(const Nodes &N, double *cell, hipStream_t st) {
    hipLaunchKernelGGL(k_cells, dim3(cdiv(cdiv(N.n, kCellNodes), 4)), dim3(256), 0, st, N, cell);
}

// Lists of the cells holding near pairs outside the kNearBand band, and their
// pair count added into *count (the products launch their fix kernels only
// when there are any).
void launch_near_cells(const Nodes &N, int *lists, double *count, hipStream_t st) {
    hipLaunchKernelGGL(k_near_cells, dim3(cdiv(N.n, kCellNodes)), dim3(256), 0, st, N, kNearBand,
                       lists, count);
}

// Blocks of the fix kernel: the 64-node cells overlapping [o, o + n).
static int fix_blocks(int o, int n) { return (o + n - 1) / kCellNodes - o / kCellNodes + 1; }

void launch_assemble64(const Layout &L, const Nodes &N, int flags, double *A, long ld,
                       hipStream_t st) {
    const int n = L.n;
    dim3 grid(cdiv(ld, 256), cdiv(n, kRowsPerAsm64));
    const int corr = (flags & WWBI_FLAG_NO_CORRECTION) ? 0 : 1;
    hipLaunchKernelGGL(k_assemble64, grid, dim3(256), 0, st, N, n, corr, A, ld);
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
    const dim3 gfix(fix_blocks(0, n));
    double *near = part + (long)ns * n;
    double *fix = near + n;
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
            if (N.near)
                hipLaunchKernelGGL((k_near_fix<0, false>), gfix, dim3(256), 0, st, N, N.nlist,
                                   hrow, 0, n, 0, n, corr, band, nb, x, fix, active);
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
            if (N.near)
                hipLaunchKernelGGL((k_near_fix<0, true>), gfix, dim3(256), 0, st, N, N.nlist,
                                   hrow, 0, n, 0, n, corr, band, nb, x, fix, active);
        }
    }
    // FP64: far chunks, near band and the near-pair fix when there are near
    // pairs; FP32 takes no fix (the quotient's error is far below FP32 rounding)
    launch_reduce_partials(n, part, (fp32 || !N.near) ? ns + 1 : ns + 2, c, 1.0, y, active, st);
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
        if (N.near)
            hipLaunchKernelGGL((k_near_fix<MODE, false>), dim3(fix_blocks(r0, nr)), dim3(256), 0,
                               st, N, N.nlist, hrow, r0, nr, c0, nc, 1, 0, nb, x,
                               part + (long)(ns + 1) * nr, active);
    } else {
        const int chunk = cols_chunk(nr, nc);
        const int ns = cdiv(nr, chunk);
        dim3 grid(cdiv(nc, 256), ns);
        hipLaunchKernelGGL((k_otf_cols<MODE, false>), grid, dim3(256), 0, st, N, hrow, r0, nr, c0,
                           nc, chunk, 1, nb, x, part, active);
        hipLaunchKernelGGL((k_near_band<MODE, true>), dim3(cdiv(nc, kNearPerBlock)), dim3(256), 0,
                           st, N, hrow, r0, nr, c0, nc, 1, 0, nb, x, part + (long)ns * nc,
                           active);
        if (N.near)
            hipLaunchKernelGGL((k_near_fix<MODE, true>), dim3(fix_blocks(c0, nc)), dim3(256), 0,
                               st, N, N.nlist, hrow, r0, nr, c0, nc, 1, 0, nb, x,
                               part + (long)(ns + 1) * nc, active);
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
