// Kernel entries of the collocated boundary-integral operators (device code).
//
// With zeta_p the target node and zeta_q the source node, write
//   kappa = cot((zeta_q - zeta_p)/2),
//   S_pq  = (1/2) zeta_q' kappa        (source flavour, Sec. 3.2 table),
//   R_pq  = -(1/2) zeta_p' kappa       (target flavour: the integration
//                                       variable sits in the first kernel slot,
//                                       Sec. 3.4 and Sec. 4.1).
// The velocity-potential matrix A (Sec. 3.3) takes Im S or Re S block by block,
// the normal-velocity map and the vortex-sheet wall system take Im R or
// Re(R + h), h = (1/2) cot((alpha_q - alpha_p)/2) on the surface's own block.
// On the diagonal every regularised kernel tends to zeta''/(2 zeta').
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace wwbi {

struct Src {               // source node q
    double ex, ey, exl, eyl, dx, dy, w;   // E = e^{i zeta} (leading + trailing), zeta', 1/M_k
    double x, y;                          // zeta (the near pairs' exact differences)
    int k, loc, M, idx;
};
struct Tgt {               // target node p
    double ex, ey, exl, eyl, dx, dy, lre, lim;
    double x, y;
    int k, loc, M, idx;
};

// Same-boundary pairs within this many grid steps take kappa from the exact
// difference of the positions (see kappa64); the on-the-fly products leave
// them (and the diagonal) to their near-band kernels.
constexpr int kNearBand = 16;

__device__ __forceinline__ Src load_src(const Nodes &N, int q) {
    Src s;
    s.ex = N.ex[q]; s.ey = N.ey[q]; s.exl = N.exl[q]; s.eyl = N.eyl[q];
    s.dx = N.dx[q]; s.dy = N.dy[q]; s.w = N.w[q]; s.x = N.x[q]; s.y = N.y[q];
    s.k = N.bid[q]; s.loc = N.loc[q]; s.M = N.Mk[q]; s.idx = q;
    return s;
}
__device__ __forceinline__ Tgt load_tgt(const Nodes &N, int p) {
    Tgt t;
    t.ex = N.ex[p]; t.ey = N.ey[p]; t.exl = N.exl[p]; t.eyl = N.eyl[p];
    t.dx = N.dx[p]; t.dy = N.dy[p]; t.x = N.x[p]; t.y = N.y[p];
    t.lre = N.lre[p]; t.lim = N.lim[p];
    t.k = N.bid[p]; t.loc = N.loc[p]; t.M = N.Mk[p]; t.idx = p;
    return t;
}

// cot((u + i v)/2) = (sin u - i sinh v) / (2 (sin^2(u/2) + sinh^2(v/2))), with
// half angles so that nearby points lose no digits (cosh v - cos u is never
// formed).  Used for the multi-valued terms and for near pairs.
__device__ __forceinline__ void cot_half64(double u, double v, double &cr, double &ci) {
    double su, cu;
    sincos(0.5 * u, &su, &cu);
    const double em = expm1(0.5 * v);        // e^{v/2} - 1, accurate for small v
    const double ep = em + 1.0;
    const double ie = 1.0 / ep;
    const double sh = 0.5 * em * (1.0 + ie); // sinh(v/2)
    const double ch = 0.5 * (ep + ie);       // cosh(v/2)
    const double r = 1.0 / (su * su + sh * sh);
    cr = su * cu * r;
    ci = -sh * ch * r;
}

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (each step doubles the correct bits; the result is within an ulp of 1/x).
__device__ __forceinline__ double recip64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// The same from the FP32 reciprocal estimate (1 ulp of FP32, about 2^-23):
// two Newton steps reach 2^-46 and then the FP64 rounding.  For x within the
// FP32 normal range (every |E_q - E_p|^2 of a far pair).
__device__ __forceinline__ double recip64_from32(double x) {
    double r = (double)__builtin_amdgcn_rcpf((float)x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ int cyc_dist(int a, int b, int M) {
    int d = a - b;
    if (d < 0) d = -d;
    return d < M - d ? d : M - d;
}

// kappa = cot((zeta_q - zeta_p)/2) from E = e^{i zeta} stored per node:
// cot(w/2) = i (e^{iw} + 1) / (e^{iw} - 1) with e^{i(zeta_q - zeta_p)} =
// E_q / E_p, i.e. kappa = i (E_q + E_p) / (E_q - E_p) -- one complex quotient
// and no transcendental function.  E is stored as a double-double, and the
// difference D = E_q - E_p is formed from both parts: the leading parts
// subtract exactly for nearby nodes, so D carries a relative error of a few
// units of rounding however close the pair (a single rounded E would leave
// an error of about 1e-16 / |zeta_q - zeta_p| relative).  The sum in the
// numerator needs no such care.
//
// Near pairs -- on one boundary within kNearBand grid steps, or closer than
// |E_q - E_p| < max(|E_p|, |E_q|) / 64 (|zeta_q - zeta_p| below about 1/64,
// any boundaries) -- take the half-angle formula on the exact difference of the
// positions instead: its real and imaginary parts are each accurate to their
// own size, while the quotient's error is a few units of |kappa| in both.
// Near a nearly flat stretch of boundary the entries Im(zeta' kappa)/2
// cancel a term 1/|slope| times their size, where that difference shows.
__device__ __forceinline__ void kappa64(const Nodes &N, const Tgt &t, const Src &s, double &cr,
                                        double &ci) {
    const double dr = (s.ex - t.ex) + (s.exl - t.exl);
    const double di = (s.ey - t.ey) + (s.eyl - t.eyl);
    const double den = dr * dr + di * di;
    const double ee = max(t.ex * t.ex + t.ey * t.ey, s.ex * s.ex + s.ey * s.ey);
    if ((t.k == s.k && cyc_dist(t.loc, s.loc, t.M) <= kNearBand) ||
        den * (kNearCut * kNearCut) < ee) {
        cot_half64(s.x - t.x, s.y - t.y, cr, ci);
        return;
    }
    const double nr = s.ex + t.ex, ni = s.ey + t.ey;
    const double inv = recip64(den);
    // N conj(D) / |D|^2 = p; kappa = i p
    const double pr = (nr * dr + ni * di) * inv;
    const double pi = (ni * dr - nr * di) * inv;
    cr = -pi;
    ci = pr;
}

// The quotient alone, for pairs outside the band (the loops of the on-the-fly
// products).
__device__ __forceinline__ void kappa64_far(const Tgt &t, const Src &s, double &cr, double &ci) {
    const double dr = (s.ex - t.ex) + (s.exl - t.exl);
    const double di = (s.ey - t.ey) + (s.eyl - t.eyl);
    const double nr = s.ex + t.ex, ni = s.ey + t.ey;
    const double inv = recip64(dr * dr + di * di);
    const double pr = (nr * dr + ni * di) * inv;
    const double pi = (ni * dr - nr * di) * inv;
    cr = -pi;
    ci = pr;
}

// FP32 quotient for far pairs; the sums and differences of E are formed in
// FP64 first, so the FP32 rounding is not amplified for nearby points.
__device__ __forceinline__ void kappa32(const Tgt &t, const Src &s, float &cr, float &ci) {
    const float nr = (float)(s.ex + t.ex), ni = (float)(s.ey + t.ey);
    const float dr = (float)(s.ex - t.ex), di = (float)(s.ey - t.ey);
    const float inv = 1.0f / (dr * dr + di * di);
    const float pr = (nr * dr + ni * di) * inv;
    const float pi = (ni * dr - nr * di) * inv;
    cr = -pi;
    ci = pr;
}

// h = (1/2) cot(pi n / M), n = (l - m) mod M, from a table of one boundary's grid.
__device__ __forceinline__ double hrow_lookup(const double *hrow, int l, int m, int M) {
    int n = l - m;
    if (n < 0) n += M;
    return hrow[n];
}

// h_pq = (1/2) cot((alpha_q - alpha_p)/2) for a same-boundary pair, from the
// table of every boundary (laid out like the nodes: boundary k's row starts at
// the node index of its first node).
__device__ __forceinline__ double h_pair(const double *hall, const Tgt &t, const Src &s) {
    return hrow_lookup(hall + (t.idx - t.loc), s.loc, t.loc, t.M);
}

// A(p, q) in FP64 (Sec. 3.3):
//   k=0,j=0: -delta/2 + w Im S     k=0,j>=1: w Re S
//   k>=1,j=0: -w Re S              k>=1,j>=1: delta/2 + w Im S - [k=j>=2] w
// the diagonal of a same-boundary block is the limit Im{zeta''/(2 zeta')}.
__device__ __forceinline__ double a_val64(const Nodes &N, const Tgt &t, const Src &s, bool corr) {
    const bool same = (t.k == s.k);
    const double ecorr = (same && t.k >= 2 && corr) ? s.w : 0.0;
    if (same && t.loc == s.loc)
        return (t.k == 0 ? -0.5 : 0.5) + s.w * t.lim - ecorr;
    double cr, ci;
    kappa64(N, t, s, cr, ci);
    const double sr = 0.5 * (s.dx * cr - s.dy * ci);
    const double si = 0.5 * (s.dx * ci + s.dy * cr);
    double v = ((t.k == 0) != (s.k == 0)) ? sr : si;
    if (t.k != 0 && s.k == 0) v = -v;
    return v * s.w - ecorr;
}

// A(p, q) stored in FP32.  Differences of positions are always formed in FP64;
// same-boundary pairs within `band` nodes (cyclically) and the diagonal limits
// are evaluated entirely in FP64 and rounded once.
__device__ __forceinline__ float a_val32(const Nodes &N, const Tgt &t, const Src &s, bool corr,
                                        int band) {
    const bool same = (t.k == s.k);
    if (same && cyc_dist(t.loc, s.loc, t.M) <= band) return (float)a_val64(N, t, s, corr);
    const float ecorr = (same && t.k >= 2 && corr) ? (float)s.w : 0.0f;
    float cr, ci;
    kappa32(t, s, cr, ci);
    const float dx = (float)s.dx, dy = (float)s.dy;
    const float sr = 0.5f * (dx * cr - dy * ci);
    const float si = 0.5f * (dx * ci + dy * cr);
    float v = ((t.k == 0) != (s.k == 0)) ? sr : si;
    if (t.k != 0 && s.k == 0) v = -v;
    return v * (float)s.w - ecorr;
}

// Target-flavour entry T(p, q) = w_q sel(R_pq + [k=j=0] h_pq), sel = Re for a
// surface source and Im for a wall source; diagonal: w Re L (surface) or
// w Im L (walls).  Rows on the surface give the normal-velocity map
// (Sec. 3.4 / Sec. 4.1 formula for U); rows and columns on the walls give
// the wall operator K^dagger; wall rows with surface sources give G_0k^dagger.
__device__ __forceinline__ double t_val64(const Nodes &N, const Tgt &t, const Src &s,
                                         const double *hrow) {
    if (t.k == s.k && t.loc == s.loc) return s.w * (t.k == 0 ? t.lre : t.lim);
    double cr, ci;
    kappa64(N, t, s, cr, ci);
    const double rr = -0.5 * (t.dx * cr - t.dy * ci);
    const double ri = -0.5 * (t.dx * ci + t.dy * cr);
    double v;
    if (s.k == 0) {
        v = rr;
        if (t.k == 0) v += hrow_lookup(hrow, s.loc, t.loc, t.M);
    } else {
        v = ri;
    }
    return s.w * v;
}

// Stream function on the fluid side of the free surface from the dipole
// densities (Sec. 5.2 energy; Plemelj limits of the Table 1 integrals):
//   psi = psi_mv + (1/2) H omega_0 + sum_q P(p, q) omega_q,
//   P = -w Re(S - h) for a surface source (diagonal -w Re L), w Im S for a
//   wall source.  Targets are surface nodes only.
__device__ __forceinline__ double psi_s(const Tgt &t, const Src &s, double cr, double ci,
                                        const double *hall) {
    const double sr = 0.5 * (s.dx * cr - s.dy * ci);
    const double si = 0.5 * (s.dx * ci + s.dy * cr);
    if (s.k == 0) return -s.w * (sr - h_pair(hall, t, s));
    return s.w * si;
}
__device__ __forceinline__ double psi_val64(const Nodes &N, const Tgt &t, const Src &s,
                                           const double *hall) {
    if (t.k == s.k && t.loc == s.loc) return -s.w * t.lre;
    double cr, ci;
    kappa64(N, t, s, cr, ci);
    return psi_s(t, s, cr, ci, hall);
}

// Tangential derivative on every boundary from gamma (Sec. 5.1, the formula
// for s dphi/ds_k): the integral terms are sum_q Q(p, q) gamma_q with
//   Q = w Im R for a surface source (diagonal w Im L),
//   Q = -w Re(R + [same boundary] h) for a wall source (diagonal -w Re L);
// the local terms (+gamma_0/2 on the surface, -H gamma_k / 2 on wall k) and
// the multi-valued part are added separately.
__device__ __forceinline__ double tan_r(const Tgt &t, const Src &s, double cr, double ci,
                                        const double *hall) {
    const double rr = -0.5 * (t.dx * cr - t.dy * ci);
    const double ri = -0.5 * (t.dx * ci + t.dy * cr);
    if (s.k == 0) return s.w * ri;
    const double h = (t.k == s.k) ? h_pair(hall, t, s) : 0.0;
    return -s.w * (rr + h);
}
__device__ __forceinline__ double tan_val64(const Nodes &N, const Tgt &t, const Src &s,
                                           const double *hall) {
    if (t.k == s.k && t.loc == s.loc) return s.k == 0 ? s.w * t.lim : -s.w * t.lre;
    double cr, ci;
    kappa64(N, t, s, cr, ci);
    return tan_r(t, s, cr, ci, hall);
}

// Source-flavour maps of the F operators (Sec. 4.2), sources on the surface:
//   KS(p, q) = w Im S (diagonal w Im L),  GS(p, q) = w Re(S - [same] h)
//   (diagonal w Re L); targets anywhere.
__device__ __forceinline__ double ks_s(const Src &s, double cr, double ci) {
    return s.w * 0.5 * (s.dx * ci + s.dy * cr);
}
__device__ __forceinline__ double gs_s(const Tgt &t, const Src &s, double cr, double ci,
                                       const double *hall) {
    const double sr = 0.5 * (s.dx * cr - s.dy * ci);
    return s.w * (t.k == s.k ? sr - h_pair(hall, t, s) : sr);
}
__device__ __forceinline__ double ks_val64(const Nodes &N, const Tgt &t, const Src &s) {
    if (t.k == s.k && t.loc == s.loc) return s.w * t.lim;
    double cr, ci;
    kappa64(N, t, s, cr, ci);
    return ks_s(s, cr, ci);
}
__device__ __forceinline__ double gs_val64(const Nodes &N, const Tgt &t, const Src &s,
                                          const double *hall) {
    if (t.k == s.k && t.loc == s.loc) return s.w * t.lre;
    double cr, ci;
    kappa64(N, t, s, cr, ci);
    return gs_s(t, s, cr, ci, hall);
}

// Operator of the gamma_t system (Sec. 4.2), all blocks in the dagger form:
//   surface row: I/2 + w Im R (surface source), -w Re R (wall source);
//   wall row:    w Re R (surface source), -I/2 + w Im R (wall source);
// diagonals +-1/2 + w Im L.
__device__ __forceinline__ double gt_r(const Tgt &t, const Src &s, double cr, double ci) {
    const double rr = -0.5 * (t.dx * cr - t.dy * ci);
    const double ri = -0.5 * (t.dx * ci + t.dy * cr);
    if ((t.k == 0) == (s.k == 0)) return s.w * ri;
    return t.k == 0 ? -s.w * rr : s.w * rr;
}
__device__ __forceinline__ double gt_val64(const Nodes &N, const Tgt &t, const Src &s) {
    if (t.k == s.k && t.loc == s.loc) return (t.k == 0 ? 0.5 : -0.5) + s.w * t.lim;
    double cr, ci;
    kappa64(N, t, s, cr, ci);
    return gt_r(t, s, cr, ci);
}

// ---------------------------------------------------------------------------
// split evaluation for the on-the-fly products: the far part skips every
// same-boundary pair within `nb` grid steps (diagonal included); the near
// part evaluates exactly those pairs with the full entry functions above.
// ---------------------------------------------------------------------------
// nb < 0 means no pair is in the band (a stage that ranges_apart has cleared).
__device__ __forceinline__ bool in_band(const Tgt &t, const Src &s, int nb) {
    return nb >= 0 && t.k == s.k && cyc_dist(t.loc, s.loc, t.M) <= nb;
}

// True when no target node in [pa, pb] and source node in [qa, qb] form a
// same-boundary pair within nb grid steps, so that a tile of the far part can
// skip the per-pair band test.  A range that crosses from one boundary to the
// next returns false (the caller keeps the per-pair test).  The pairs of two
// ranges on one boundary of M nodes have index distances d between their gap
// and their span, and a pair is in the band when min(d, M - d) <= nb.
__device__ __forceinline__ bool ranges_apart(const Nodes &N, int pa, int pb, int qa, int qb,
                                             int nb) {
    const int kp = N.bid[pa], kq = N.bid[qa];
    if (N.bid[pb] != kp || N.bid[qb] != kq) return false;
    if (kp != kq) return true;
    const int lpa = N.loc[pa], lpb = N.loc[pb], lqa = N.loc[qa], lqb = N.loc[qb];
    const int gap = max(0, max(lqa - lpb, lpa - lqb));
    const int span = max(lpb - lqa, lqb - lpa);
    return gap > nb && N.Mk[pa] - span > nb;
}

// Boundary of the nodes [a, b], or -1 when the range crosses a boundary end.
__device__ __forceinline__ int range_boundary(const Nodes &N, int a, int b) {
    const int k = N.bid[a];
    return N.bid[b] == k ? k : -1;
}

// First thread of the calling wave (wave-uniform; call where every lane is active).
__device__ __forceinline__ int wave_base() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x) & ~63;
}

// Whether a wave's outputs [o0, o0 + 64) (clipped to [0, nout)) are clear of
// the near band of the summed nodes [q0, q0 + m); output node = obase +
// output, and COLS says the outputs are sources.  Vacuously true for a wave
// without live outputs.
template <bool COLS>
__device__ __forceinline__ bool wave_apart(const Nodes &N, int obase, int o0, int nout, int q0,
                                           int m, int nb) {
    if (o0 >= nout) return true;
    const int a = obase + o0, b = obase + min(o0 + 63, nout - 1);
    return COLS ? ranges_apart(N, q0, q0 + m - 1, a, b, nb)
                : ranges_apart(N, a, b, q0, q0 + m - 1, nb);
}

__device__ __forceinline__ double a_far64(const Tgt &t, const Src &s, bool corr, int nb) {
    if (in_band(t, s, nb)) return 0.0;
    const double ecorr = (t.k == s.k && t.k >= 2 && corr) ? s.w : 0.0;
    double cr, ci;
    kappa64_far(t, s, cr, ci);
    const double sr = 0.5 * (s.dx * cr - s.dy * ci);
    const double si = 0.5 * (s.dx * ci + s.dy * cr);
    double v = ((t.k == 0) != (s.k == 0)) ? sr : si;
    if (t.k != 0 && s.k == 0) v = -v;
    return v * s.w - ecorr;
}

__device__ __forceinline__ float a_far32(const Tgt &t, const Src &s, bool corr, int nb) {
    if (in_band(t, s, nb)) return 0.0f;
    const float ecorr = (t.k == s.k && t.k >= 2 && corr) ? (float)s.w : 0.0f;
    float cr, ci;
    kappa32(t, s, cr, ci);
    const float dx = (float)s.dx, dy = (float)s.dy;
    const float sr = 0.5f * (dx * cr - dy * ci);
    const float si = 0.5f * (dx * ci + dy * cr);
    float v = ((t.k == 0) != (s.k == 0)) ? sr : si;
    if (t.k != 0 && s.k == 0) v = -v;
    return v * (float)s.w - ecorr;
}

__device__ __forceinline__ double psi_far64(const Tgt &t, const Src &s, const double *hall,
                                            int nb) {
    if (in_band(t, s, nb)) return 0.0;
    double cr, ci;
    kappa64_far(t, s, cr, ci);
    return psi_s(t, s, cr, ci, hall);
}

__device__ __forceinline__ double tan_far64(const Tgt &t, const Src &s, const double *hall,
                                            int nb) {
    if (in_band(t, s, nb)) return 0.0;
    double cr, ci;
    kappa64_far(t, s, cr, ci);
    return tan_r(t, s, cr, ci, hall);
}

__device__ __forceinline__ double ks_far64(const Tgt &t, const Src &s, int nb) {
    if (in_band(t, s, nb)) return 0.0;
    double cr, ci;
    kappa64_far(t, s, cr, ci);
    return ks_s(s, cr, ci);
}
__device__ __forceinline__ double gs_far64(const Tgt &t, const Src &s, const double *hall, int nb) {
    if (in_band(t, s, nb)) return 0.0;
    double cr, ci;
    kappa64_far(t, s, cr, ci);
    return gs_s(t, s, cr, ci, hall);
}
__device__ __forceinline__ double gt_far64(const Tgt &t, const Src &s, int nb) {
    if (in_band(t, s, nb)) return 0.0;
    double cr, ci;
    kappa64_far(t, s, cr, ci);
    return gt_r(t, s, cr, ci);
}

__device__ __forceinline__ double t_far64(const Tgt &t, const Src &s, const double *hrow, int nb) {
    if (in_band(t, s, nb)) return 0.0;
    double cr, ci;
    kappa64_far(t, s, cr, ci);
    const double rr = -0.5 * (t.dx * cr - t.dy * ci);
    const double ri = -0.5 * (t.dx * ci + t.dy * cr);
    double v;
    if (s.k == 0) {
        v = rr;
        if (t.k == 0) v += hrow_lookup(hrow, s.loc, t.loc, t.M);
    } else {
        v = ri;
    }
    return s.w * v;
}

}  // namespace wwbi
