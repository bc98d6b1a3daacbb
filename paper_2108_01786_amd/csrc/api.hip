// Host side of libwwbi: context and workspace, input validation, the GMRES
// and iterative-refinement drivers, and the C entry points of wwbi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "api_internal.h"

using namespace wwbi;

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------

namespace wwbi {

static int hip_ok(hipError_t e) { return e == hipSuccess ? WWBI_OK : WWBI_EHIP; }

template <typename T>
static int grow(T *&p, size_t &cap, size_t want) {
    if (want <= cap && p) return WWBI_OK;
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc((void **)&p, want * sizeof(T)) != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return WWBI_ECAPACITY;
    }
    hipMemset(p, 0, want * sizeof(T));
    cap = want;
    return WWBI_OK;
}

// The per-solve workspace of n unknowns and restart length `restart`: every
// buffer with its element count.  ensure() grows each to that count; the
// allocation-free entry point carves the same list out of its static array.
int Ctx::ws_plan(int n, int restart, WsItem *it, bool recycle) {
    const size_t nn = (size_t)round_up(n, 64);
    const size_t rr = (size_t)std::max(restart, 8);
    const size_t pre = recycle ? kRecycleMax : 0;
    int k = 0;
    auto D = [&](double *&p, size_t &c, size_t w) { it[k++] = WsItem{(void **)&p, &c, w, 8}; };
    auto I = [&](int *&p, size_t &c, size_t w) { it[k++] = WsItem{(void **)&p, &c, w, 4}; };
    D(V, capV, (pre + rr + 1) * nn);
    it[k++] = WsItem{(void **)&v32, &capv32, nn, 4};   // FP32 copy of the newest basis vector
    for (int i = 0; i < kNumVec; ++i) D(vec[i], capvec[i], nn);
    D(H, capH, (rr + 1) * (rr + 1));
    D(cs, capcs, rr + 1);
    D(sn, capsn, rr + 1);
    D(gv, capg, rr + 1);
    D(yv, capy, rr + 1);
    D(P, capP, 3 * 64 * (pre + rr + 1) + 128);
    if (recycle) {
        D(Urec, capUrec, pre * nn);
        D(Brec, capBrec, pre * (rr + 2));
    }
    D(part, cappart, 258 * nn + 64);   // up to 256 far slices + the near-band and near-fix slices
    D(pw, cappw, 65 * (size_t)gemv_partials(nn) + 64);   // 64 dot rows + the norms
    D(hsum, caphsum, 128);
    I(bid, capbid, nn);
    I(loc, caploc, nn);
    I(Mk, capMk, nn);
    D(wq, capwq, nn);
    D(s, caps, nn);
    D(lre, caplre, nn);
    D(lim, caplim, nn);
    D(rowD, caprowD, nn);
    D(rowH, caprowH, nn);
    D(hrow, caphrow, nn);
    D(eR, capeR, nn);
    D(eI, capeI, nn);
    D(eRl, capeRl, nn);
    D(eIl, capeIl, nn);
    D(cell, capcell, 4 * (nn / kCellNodes) + 4);
    I(nlist, capnlist, (size_t)kNearStride * (nn / kCellNodes));
    D(val, capval, 4 * kMaxB + 8 + kValidateBlocks);
    return k;
}

int Ctx::ensure(int n, int restart) {
    trace = std::getenv("WWBI_TRACE") != nullptr;
    WsItem it[kMaxWsItems];
    // a carved workspace (the allocation-free entry point) has no room for a
    // recycled space
    const int k = ws_plan(n, restart, it, !fixed_ws);
    if (fixed_ws) {
        // workspace carved for this call: it cannot grow
        for (int i = 0; i < k; ++i)
            if (it[i].count > *it[i].cap) return WWBI_ESCRATCH;
        return WWBI_OK;
    }
    for (int i = 0; i < k; ++i) {
        unsigned char *p = static_cast<unsigned char *>(*it[i].p);
        size_t cap = *it[i].cap * it[i].esize;
        const int rc = grow(p, cap, it[i].count * it[i].esize);
        *it[i].p = p;
        *it[i].cap = cap / it[i].esize;
        if (rc) return rc;
    }
    vpre = kRecycleMax;
    return WWBI_OK;
}

namespace {
int grow_bytes(void *&p, size_t &cap, size_t bytes) {
    if (bytes <= cap && p) return WWBI_OK;
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return WWBI_ECAPACITY;
    }
    cap = bytes;
    return WWBI_OK;
}
}  // namespace

int Ctx::ensure_matrix(size_t bytes) { return grow_bytes(A, capA, bytes); }

int Ctx::ensure_matrix64(size_t bytes) {
    void *p = A64;
    const int rc = grow_bytes(p, capA64, bytes);
    A64 = static_cast<double *>(p);
    return rc;
}

void Ctx::release() {
    auto F = [](auto *&p) { if (p) hipFree((void *)p); p = nullptr; };
    F(A);
    F(A64);
    capA64 = 0;
    F(pw);
    cappw = 0;
    F(hsum);
    F(V);
    F(v32);
    F(Urec);
    F(Brec);
    vpre = 0;
    for (int i = 0; i < kNumVec; ++i) F(vec[i]);
    F(H); F(cs); F(sn); F(gv); F(yv); F(P); F(part);
    F(bid); F(loc); F(Mk); F(wq); F(s); F(lre); F(lim); F(rowD); F(rowH); F(val); F(apart);
    F(evrow); F(ew); F(ek); F(hop); F(hoi);
    F(hrow); F(eR); F(eI); F(eRl); F(eIl); F(cell); F(nlist);
    if (gs) hipFree(gs);
    gs = nullptr;
    if (hst) hipHostFree(hst);
    hst = nullptr;
    if (hmir) hipHostFree(hmir);
    hmir = dmir = nullptr;
    for (auto &e : ev) if (e) hipEventDestroy(e);
    for (auto &e : prof) if (e) hipEventDestroy(e);
    for (auto &e : pollev) if (e) hipEventDestroy(e);
    for (auto &e : stepev) if (e) hipEventDestroy(e);
    {
        MultiWS &m = mw;
        F(m.V); F(m.v32); F(m.x32); F(m.w); F(m.r); F(m.x); F(m.b); F(m.d); F(m.rr); F(m.P); F(m.H);
        F(m.cs); F(m.sn); F(m.g); F(m.y); F(m.part); F(m.nrm); F(m.gs);
    }
}

// ---------------------------------------------------------------------------
// geometry set-up and validation
// ---------------------------------------------------------------------------

int Ctx::setup(const wwbi_geom *g, const double *phi, int nphi, bool check) {
    if (!g || !g->M || !g->x || !g->y || !g->dx || !g->dy || !g->ddx || !g->ddy)
        return WWBI_EINVAL_NULL;
    if (g->nb < 2 || g->nb > kMaxB) return WWBI_EINVAL_SIZE;
    if (g->nb > 2 && (!g->zc || !g->a)) return WWBI_EINVAL_NULL;
    L.nb = g->nb;
    L.off[0] = 0;
    for (int k = 0; k < g->nb; ++k) {
        const int m = g->M[k];
        if (m < 8 || (m & 1)) return WWBI_EINVAL_SIZE;
        if ((long)L.off[k] + m > (1L << 28)) return WWBI_EINVAL_SIZE;
        L.off[k + 1] = L.off[k] + m;
    }
    L.n = L.off[g->nb];
    F.V1 = g->V1;
    F.nobs = g->nb - 2;
    if (!std::isfinite(g->V1)) return WWBI_EINVAL_NONFINITE;
    for (int j = 0; j < F.nobs; ++j) {
        F.a[j] = g->a[j];
        F.zx[j] = g->zc[2 * j];
        F.zy[j] = g->zc[2 * j + 1];
        if (!std::isfinite(F.a[j]) || !std::isfinite(F.zx[j]) || !std::isfinite(F.zy[j]))
            return WWBI_EINVAL_NONFINITE;
    }
    int rc = ensure(L.n, restart_cap);
    if (rc) return rc;
    N.x = g->x; N.y = g->y; N.dx = g->dx; N.dy = g->dy; N.ddx = g->ddx; N.ddy = g->ddy;
    N.bid = bid; N.loc = loc; N.Mk = Mk; N.w = wq; N.s = s; N.lre = lre; N.lim = lim;
    N.ex = eR; N.ey = eI; N.exl = eRl; N.eyl = eIl; N.cell = cell; N.nlist = nlist;
    N.n = L.n;
    psi_wall = g->psi_wall;
    launch_prep_nodes(L, g->x, g->y, g->dx, g->dy, g->ddx, g->ddy, bid, loc, Mk, wq, s, lre, lim,
                      eR, eI, eRl, eIl, stream);
    launch_cells(N, cell, stream);
    launch_circulant_rows(L, kOpHalfCot, hrow, stream);
    N.near = 0;
    val_blocks = validate_data_blocks(phi ? nphi : 0);
    launch_validate(L, N, phi, phi ? nphi : 0, val, stream);   // also zeroes val[4 nb + 1]
    launch_near_cells(N, nlist, val + 4 * L.nb + 1, stream);
    if (hipMemcpyAsync(hst, val, sizeof(double) * (4 * L.nb + 2 + val_blocks),
                       hipMemcpyDeviceToHost, stream) != hipSuccess)
        return WWBI_EHIP;
    if (hipEventRecord(pollev[2], stream) != hipSuccess) return WWBI_EHIP;
    return check ? setup_check() : WWBI_OK;
}

// The device-side checks of setup(): finite samples and data, even counts in
// range, the orientation of every boundary, and the near-pair count.
int Ctx::setup_check() {
    // wait for the copy of the checks only: work queued after it keeps running
    if (hipEventSynchronize(pollev[2]) != hipSuccess) return WWBI_EHIP;
    const double *h = (const double *)hst;
    for (int k = 0; k < L.nb; ++k)
        if (h[4 * k] != 0.0) return WWBI_EINVAL_NONFINITE;
    for (int b = 0; b < val_blocks; ++b)
        if (h[4 * L.nb + 2 + b] != 0.0) return WWBI_EINVAL_NONFINITE;
    for (int k = 0; k < L.nb; ++k)
        if (h[4 * k + 3] != 0.0) return WWBI_EINVAL_RANGE;
    N.near = h[4 * L.nb + 1] > 0.0 ? 1 : 0;
    near_pairs = (long)h[4 * L.nb + 1];
    for (int k = 0; k < L.nb; ++k) {
        if (k <= 1 && !(h[4 * k + 2] > 0.0)) return WWBI_EINVAL_ORIENTATION;
        if (k >= 2 && !(h[4 * k + 1] < 0.0)) return WWBI_EINVAL_ORIENTATION;
    }
    return WWBI_OK;
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------

void Ctx::apply(const Op &op, const double *x, const float *x32, const double *c, double *y,
                const int *active) {
    const long ld = op.ld;
    switch (op.kind) {
    case OP_A_S64:
        launch_gemv64((const double *)A, ld, op.n, x, c, y, active, stream);
        break;
    case OP_A_S32:
    case OP_GT_S32:
    case OP_W_S32:
        // FP32 products read x in FP32 (the caller's copy, or one made here)
        if (!x32) {
            launch_to_f32(x, v32, op.n, stream);
            x32 = v32;
        }
        launch_gemv32((const float *)A, ld, op.n, x32, c, y, active, stream);
        break;
    case OP_A_O64:
        launch_otf_matvec(L, N, op.flags, 0, op.band, 0, x, c, y, part, active, stream);
        break;
    case OP_A_O32:
        launch_otf_matvec(L, N, op.flags, 1, op.band, 0, x, c, y, part, active, stream);
        break;
    case OP_AT_O64:
        launch_otf_matvec(L, N, op.flags, 0, op.band, 1, x, c, y, part, active, stream);
        break;
    case OP_AT_O32:
        launch_otf_matvec(L, N, op.flags, 1, op.band, 1, x, c, y, part, active, stream);
        break;
    case OP_W_S64:
        launch_gemv64((const double *)A, ld, op.n, x, c, y, active, stream);
        break;
    case OP_W_O64: {
        const int o1 = L.off[1], nw = L.n - o1;
        launch_rflavour(L, N, hrow, 3, 0, o1, nw, o1, nw, x, part, active, stream);
        launch_reduce_partials(nw, part, rflavour_nsplit(N, nw, nw, 0), c, 1.0, y, active,
                               stream);
        break;
    }
    case OP_GT_S64:
        launch_gemv64((const double *)A, ld, op.n, x, c, y, active, stream);
        break;
    case OP_GT_O64:
        launch_rflavour(L, N, hrow, 8, 0, 0, L.n, 0, L.n, x, part, active, stream);
        launch_reduce_partials(L.n, part, rflavour_nsplit(N, L.n, L.n, 0), c, 1.0, y, active,
                               stream);
        break;
    }
}

double Ctx::op_bytes(const Op &op) const {
    const double n = op.n;
    switch (op.kind) {
    case OP_A_S64: case OP_W_S64: case OP_GT_S64:
        return n * n * 8.0 + 2.0 * n * 8.0;
    case OP_A_S32: case OP_GT_S32: case OP_W_S32: return n * n * 4.0 + n * 4.0 + n * 8.0;
    default: return 0.0;
    }
}

int Ctx::read_state(GState &out) {
    if (hipMemcpyAsync(hst, gs, sizeof(GState), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return WWBI_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return WWBI_EHIP;
    std::memcpy(&out, hst, sizeof(GState));
    return WWBI_OK;
}

int Ctx::final_state(GState &out) {
    const volatile GState *m = hmir;
    if (m->cyc != cyc_id) return read_state(out);
    out.active = m->active;
    out.jdone = m->jdone;
    out.breakdown = m->breakdown;
    out.its = m->its;
    out.bnorm = m->bnorm;
    out.tol_abs = m->tol_abs;
    out.beta = m->beta;
    out.resid = m->resid;
    out.cyc = m->cyc;
    return WWBI_OK;
}

void Ctx::prof_begin() {
    if (profiling && nprof < kProfPairs) {
        hipEventRecord(prof[2 * nprof], stream);
        prof_cycle[nprof] = cur_cycle;
        prof_step[nprof] = cur_step;
    }
}
void Ctx::prof_end() {
    if (profiling && nprof < kProfPairs) {
        hipEventRecord(prof[2 * nprof + 1], stream);
        ++nprof;
    }
}

// Restarted GMRES on op: x <- solution of op x = b.  x must hold the initial
// guess unless x_zero.  With verify, every cycle starts from the true residual
// b - op x and convergence is declared only on it.  Without verify a single
// cycle runs and the call returns as soon as the update of x is enqueued; the
// final cycle state is copied asynchronously to host slot 2, which the caller
// reads after its next synchronisation (inner solves of the refinement).
//
// The host enqueues `poll` Arnoldi steps at a time.  After each batch it
// records an event (one without the system-scope fence, 1% of a refined solve
// on the 10240-unknown cell), enqueues the next batch and only then waits for
// the previous event, so the device never idles on the host.  The kernel that
// ends a cycle publishes the cycle's state, with its id, into host-mapped
// memory: the host sees the end without a queued copy, and steps enqueued
// after it return at once on the device flag.
int Ctx::gmres(const Op &op, const double *b, double *x, bool x_zero, double tol, int restart,
               int max_iter, int poll, bool verify, SolveStats &st, int kc) {
    const int n = op.n;
    const int G = gmres_nblocks(n);
    const int ldp = restart + 1 + vpre;    // rows of Gram-Schmidt partials (recycled ones too)
    const long ldv = round_up(n, 64);
    double *r = vec[VR], *w = vec[VW];
    double *P1 = P, *P2 = P + 64 * ldp, *P3 = P + 2 * 64 * ldp;   // P[i*G + b] layout
    const int NB = gemv_partials(n);
    // the Arnoldi basis, and in front of it the kc recycled vectors C
    double *Vb = V + (long)vpre * ldv;
    double *Cb = Vb - (long)kc * ldv;
    double *Bm = Brec, *zc = Brec + (long)kRecycleMax * (restart + 1);
    // stored FP32 products read the newest basis vector's FP32 copy, written
    // by the kernel that forms the vector
    float *x32 = stored_fp32(op.kind) ? v32 : nullptr;
    // the inner solves of the refinement (the only callers without the
    // true-residual check) orthogonalise once; every other solve twice
    const bool single_pass = !verify;
    if (kc > 0) {
        // deflated solve: r0 = b - C C^T b starts the (only) cycle; the
        // tolerance is relative to ||b||
        if (verify || !x_zero || kc > vpre) return WWBI_EINVAL_OPTS;
        restart = std::min(restart, WWBI_MAX_RESTART - kc);
        launch_recycle_dots(Cb, ldv, b, n, kc, P1, P3, G, stream);
        launch_set_tol(P3, G, tol, gs, stream);
        launch_recycle_project(Cb, ldv, b, n, kc, P1, P3, G, r, zc, stream);
    } else {
        launch_norm_partial(b, n, P3, G, stream);
        launch_set_tol(P3, G, tol, gs, stream);
    }
    bool first = true;
    bool x_set = !x_zero;      // a cold start writes x with its first update
    double prev_beta = HUGE_VAL;
    int status = WWBI_NOT_CONVERGED;
    const int its0 = st.iters;
    int its_seen = 0;          // device step count at the previous cycle start
    GState h{};
    for (;;) {
        cur_cycle = -1;        // the residual product is not an Arnoldi step
        const double *r0 = r;
        if (kc > 0) {
            // r holds b - C C^T b and P3 its norm partials
        } else if (!x_set) {
            r0 = b;            // r = b - A 0, whose norm partials are already in P3
        } else {
            apply(op, x, nullptr, b, r, nullptr);
            launch_norm_partial(r, n, P3, G, stream);
        }
        cyc_id = cyc_id == INT_MAX ? 1 : cyc_id + 1;   // never 0, the mirror's initial id
        const int cid = cyc_id;
        launch_cycle_start(r0, n, P3, G, Vb, x32, gv, restart + 1, gs, cid, dmir, stream);
        int jmax = std::min(restart, max_iter - st.iters);
        if (verify) {
            int rc = read_state(h);
            if (rc) return rc;
            if (!cyc_done.empty() && cyc_done.back() < 0) cyc_done.back() = h.its - its_seen;
            its_seen = h.its;
            st.iters = its0 + h.its;
            st.rel_resid = h.bnorm > 0 ? h.beta / h.bnorm : 0.0;
            note_resid(st.rel_resid);
            if (trace)
                std::fprintf(stderr, "wwbi: op %d n %d cycle %d its %d beta/bnorm %.3e\n",
                             op.kind, n, st.cycles, st.iters, st.rel_resid);
            if (!h.active) { status = WWBI_OK; break; }
            if (!std::isfinite(h.beta)) { status = WWBI_STAGNATED; break; }
            if (st.iters >= max_iter) { status = WWBI_NOT_CONVERGED; break; }
            if (!first && h.beta > 0.99 * prev_beta) { status = WWBI_STAGNATED; break; }
            prev_beta = h.beta;
            jmax = std::min(restart, max_iter - st.iters);
        }
        jmax = std::max(jmax, 1);
        cyc_done.push_back(-1);
        cur_cycle = (int)cyc_done.size() - 1;
        last_cycle = cur_cycle;
        int pending = -1;          // slot of the flag copy not yet waited for
        bool ended = false;
        for (int j0 = 0; j0 < jmax && !ended; j0 += poll) {
            const int j1 = std::min(jmax, j0 + poll);
            for (int j = j0; j < j1; ++j) {
                const double *vj = Vb + (long)j * ldv;
                cur_step = j;
                // steps on a stored matrix take the first Gram-Schmidt dots in the
                // product's epilogue (one partial per product block), for up to
                // 64 rows (the recycled ones included)
                const bool fuse32 = single_pass && stored_fp32(op.kind) && kc + j < 64;
                const bool fuse64 = !single_pass && stored_fp64(op.kind) && j < 64;
                prof_begin();
                if (fuse32)
                    launch_gemv32_dots((const float *)A, op.ld, n, x32, w, &gs->active, Cb, ldv,
                                       kc + j, pw, pw + 64L * NB, stream);
                else if (fuse64)
                    launch_gemv64_dots((const double *)A, op.ld, n, vj, w, &gs->active, Vb, ldv,
                                       j, pw, pw + 64L * NB, stream);
                else
                    apply(op, vj, x32, nullptr, w, &gs->active);
                prof_end();
                if (fuse32) {
                    // the product's partials summed once (kc + j + 1 dots and the norm)
                    launch_reduce_rows(pw, NB, pw + 64L * NB, kc + j + 2, hsum, gs, stream);
                    launch_cgs_final(Cb, ldv, w, n, j, pw, pw + 64L * NB, G, x32, H, restart + 1,
                                     false, cs, sn, gv, jmax, gs, cid, dmir, stream, kSingle, NB,
                                     kc, Bm, kRecycleMax, hsum);
                    continue;
                }
                if (fuse64) {
                    launch_reduce_rows(pw, NB, nullptr, j + 1, hsum, gs, stream);
                    launch_cgs_first(Vb, ldv, w, n, j, pw, P2, P3, G, H, restart + 1, gs, stream,
                                     kSingle, NB, hsum);
                    launch_cgs_final(Vb, ldv, w, n, j, P2, P3, G, x32, H, restart + 1, true, cs,
                                     sn, gv, jmax, gs, cid, dmir, stream);
                    continue;
                }
                launch_cgs_dot(Cb, ldv, w, n, kc + j, P1, P3, G, gs, stream);
                if (single_pass) {
                    launch_cgs_final(Cb, ldv, w, n, j, P1, P3, G, x32, H, restart + 1, false, cs,
                                     sn, gv, jmax, gs, cid, dmir, stream, kSingle, 0, kc, Bm,
                                     kRecycleMax);
                } else {
                    launch_cgs_first(Vb, ldv, w, n, j, P1, P2, P3, G, H, restart + 1, gs, stream);
                    launch_cgs_final(Vb, ldv, w, n, j, P2, P3, G, x32, H, restart + 1, true, cs,
                                     sn, gv, jmax, gs, cid, dmir, stream);
                }
            }
            const int cur = (j0 / poll) & 1;
            if (hipEventRecord(stepev[cur], stream) != hipSuccess) return WWBI_EHIP;
            if (pending >= 0) {
                if (hipEventSynchronize(stepev[pending]) != hipSuccess) return WWBI_EHIP;
                // a mirror that still lags only delays the end by a batch of
                // no-op steps: the id is new for every cycle
                if (static_cast<const volatile GState *>(hmir)->cyc == cid) ended = true;
            }
            pending = cur;
        }
        launch_hsolve(H, restart + 1, gv, yv, gs, stream);
        if (kc > 0) {
            launch_recycle_coef(zc, Bm, kRecycleMax, yv, kc, gs, stream);
            launch_xupdate_recycled(x, Vb, ldv, n, yv, Urec, zc, kc, gs, stream);
        } else {
            launch_xupdate(x, Vb, ldv, n, yv, !x_set, gs, stream);
        }
        x_set = true;
        st.cycles += 1;
        first = false;
        if (!verify) {
            status = WWBI_OK;      // the caller reads the final state (final_state)
            break;
        }
    }
    if (!x_set) launch_fill(x, 0.0, n, stream);   // stopped before the first update
    return status;
}

// Tolerance of an inner FP32 solve: o.inner_tol (the contraction the FP32
// operator supports: FP32 entries and vector, FP64 accumulation), loosened
// when the residual is already close to the target -- a correction only needs
// to gain the remaining factor (with a 3x margin), which keeps the last
// refinement step short.
constexpr double kMulti32Floor = 3e-7;

double inner_tolerance(const wwbi_opts &o, double bnorm, double rnorm) {
    const double need = rnorm > 0 ? 0.3 * o.tol * bnorm / rnorm : 1.0;
    return std::min(0.1, std::max(o.inner_tol, need));
}

double Ctx::device_norm(const double *v, int n) {
    const int G = gmres_nblocks(n);
    double *P3 = norm_partials();
    launch_norm_partial(v, n, P3, G, stream);
    if (hipMemcpyAsync(hst, P3, sizeof(double) * G, hipMemcpyDeviceToHost, stream) != hipSuccess)
        return NAN;
    if (hipStreamSynchronize(stream) != hipSuccess) return NAN;
    const double *h = (const double *)hst;
    double s2 = 0.0;
    for (int b = 0; b < G; ++b) s2 += h[b];
    return std::sqrt(s2);
}

// FP64 iterative refinement around an FP32 inner solve:
//   r = b - A64 x (FP64 operator); stop at ||r|| <= tol ||b||;
//   solve A32 d = r by GMRES to the inner tolerance; x += d.
// One host synchronisation per step: the norm of the new residual and the
// final state of the inner solve are read together.
//
// Unless WWBI_FLAG_NO_RECYCLE, the first inner solve's Krylov space is kept
// (C orthonormal, A32 U = C; up to kRecycleMax vectors) and every later inner
// solve deflates it: the residuals of the later steps are dominated by the
// same slowly converging directions, which the first solve has already found.
int Ctx::refine(const Op &op32, const Op &op64, const double *b, double *x, bool x_zero,
                const wwbi_opts &o, SolveStats &st) {
    const int n = op64.n;
    const int G = gmres_nblocks(n);
    const long ldv = round_up(n, 64);
    double *r = vec[VRR], *d = vec[VD];
    const bool recycle = !(o.flags & WWBI_FLAG_NO_RECYCLE) && vpre > 0 && op32.n == n &&
                         stored_fp32(op32.kind);
    int kc = 0;                // recycled vectors the later inner solves deflate
    bool first_inner = true;   // the pending inner solve is the first one
    double *Pn = norm_partials() + 64;   // norm partials (64 doubles)
    // From a cold start the first inner solve takes b itself and writes x;
    // ||b|| then comes back in that solve's final state, read at the first
    // synchronisation, so no host round trip precedes it.
    double bn = -1.0;
    if (!x_zero) {
        bn = device_norm(b, n);
        if (!std::isfinite(bn)) return WWBI_EHIP;
    }
    double prev = HUGE_VAL;
    int status = WWBI_NOT_CONVERGED;
    bool inner_pending = false;
    for (int k = 0;; ++k) {
        double rn;
        const bool cold = k == 0 && x_zero;
        if (cold) {
            rn = -1.0;
        } else {
            apply(op64, x, nullptr, b, r, nullptr);
            launch_norm_partial(r, n, Pn, G, stream);
            if (hipMemcpyAsync(hst, Pn, sizeof(double) * G, hipMemcpyDeviceToHost, stream) !=
                hipSuccess)
                return WWBI_EHIP;
            if (hipStreamSynchronize(stream) != hipSuccess) return WWBI_EHIP;
            const double *h = (const double *)hst;
            double s2 = 0.0;
            for (int i = 0; i < G; ++i) s2 += h[i];
            rn = std::sqrt(s2);
            if (inner_pending) {
                GState fin;                    // the inner solve's final state
                if (final_state(fin)) return WWBI_EHIP;
                st.iters += fin.its;
                if (last_cycle >= 0 && last_cycle < (int)cyc_done.size())
                    cyc_done[last_cycle] = fin.its;
                inner_pending = false;
                if (bn < 0.0) {
                    bn = fin.bnorm;     // the first inner solve's right-hand side was b
                    prev = bn;
                }
                // the first solve's basis, rotated Hessenberg and rotations are
                // still in place (nothing since has written them)
                if (first_inner && recycle && fin.jdone >= 1 && fin.jdone <= vpre &&
                    !fin.breakdown && std::isfinite(fin.resid)) {
                    kc = fin.jdone;
                    double *Vb = V + (long)vpre * ldv;
                    launch_recycle_build(Vb, ldv, n, kc, H, o.restart + 1, cs, sn,
                                         Vb - (long)kc * ldv, Urec, stream);
                }
                first_inner = false;
            }
        }
        if (!cold) {
            st.rel_resid = bn > 0 ? rn / bn : 0.0;
            note_resid(st.rel_resid);
            if (trace)
                std::fprintf(stderr, "wwbi: refine step %d its %d rel_resid %.3e\n", k,
                             st.iters, st.rel_resid);
            if (rn <= o.tol * bn) { status = WWBI_OK; break; }
            if (!std::isfinite(rn) || (k > 0 && rn > 0.5 * prev)) {
                status = WWBI_REFINE_STALLED;
                break;
            }
        }
        if (k >= o.max_refine || st.iters >= o.max_iter) { status = WWBI_NOT_CONVERGED; break; }
        if (!cold) prev = rn;
        SolveStats in{};
        // for the cold step rn = ||b||, where the inner tolerance does not depend on ||b||
        const double itol = cold ? inner_tolerance(o, 1.0, 1.0) : inner_tolerance(o, bn, rn);
        const int rc = gmres(op32, cold ? b : r, cold ? x : d, true, itol, o.restart,
                             o.max_iter - st.iters, o.poll_every, false, in, kc);
        if (rc < 0) return rc;
        inner_pending = true;
        st.cycles += in.cycles;
        st.refine_steps += 1;
        if (!cold) launch_axpy(x, d, n, 1.0, stream);
    }
    return status;
}

// U on the surface from the surface-and-wall vortex sheets gamma (Sec. 3.4,
// Sec. 4.1): U = (u_mv + H gamma_0 / 2 + T gamma) / s.
void Ctx::eval_U_from_gamma(const double *gamma, double *U) {
    const int n0 = L.off[1];
    double *hg = vec[VHG], *um = vec[VUM];
    launch_circulant_apply(L, rowH, gamma, hg, 1.0, 0.0, 0, 0, stream);
    launch_umv(N, F, 0, n0, um, stream);
    launch_rflavour(L, N, hrow, 2, 0, 0, n0, 0, L.n, gamma, part, nullptr, stream);
    launch_U_finalize(n0, s, um, hg, part, rflavour_nsplit(N, n0, L.n, 0), U, stream);
}

void Ctx::gamma_from_omega(const double *omega, double *gamma) {
    launch_circulant_apply2(L, rowD, omega, gamma, -1.0, 1.0, 0.0, 0, L.nb - 1, stream);
}

int Ctx::check_opts(const wwbi_opts *o) {
    if (!o) return WWBI_EINVAL_NULL;
    if (!(o->tol > 0.0) || !(o->tol < 1.0)) return WWBI_EINVAL_OPTS;
    if (o->restart < 1 || o->restart > WWBI_MAX_RESTART) return WWBI_EINVAL_OPTS;
    if (o->max_iter < 1 || o->poll_every < 1) return WWBI_EINVAL_OPTS;
    if (o->precision != WWBI_FP64 && o->precision != WWBI_FP32_REFINED) return WWBI_EINVAL_OPTS;
    if (o->matvec < 0 || o->matvec > 2) return WWBI_EINVAL_OPTS;
    if (o->band < 0) return WWBI_EINVAL_OPTS;
    if (o->precision == WWBI_FP32_REFINED && (!(o->inner_tol > 0.0) || !(o->inner_tol < 1.0)))
        return WWBI_EINVAL_OPTS;
    return WWBI_OK;
}

void Ctx::begin_report(bool prof) {
    profiling = prof;
    nprof = 0;
    cyc_done.clear();
    hist.clear();
    cur_cycle = -1;
    cur_step = 0;
    hipEventRecord(ev[0], stream);
}

static float ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

void Ctx::finish_report(wwbi_report *rep, int status, const SolveStats &st, double bytes) {
    hipStreamSynchronize(stream);
    if (!rep) return;
    std::memset(rep, 0, sizeof(*rep));
    rep->status = status;
    rep->iters = st.iters;
    rep->restarts = st.cycles;
    rep->refine_steps = st.refine_steps;
    rep->rel_resid = st.rel_resid;
    rep->ms_prep = ev_ms(ev[0], ev[1]);
    rep->ms_assemble = ev_ms(ev[1], ev[2]);
    rep->ms_solve = ev_ms(ev[2], ev[3]);
    rep->ms_U = ev_ms(ev[3], ev[4]);
    rep->ms_total = ev_ms(ev[0], ev[4]);
    double t = 0.0;
    int cnt = 0;
    for (int i = 0; i < nprof; ++i) {
        const int c = prof_cycle[i];
        const bool real = c < 0 || c >= (int)cyc_done.size() || cyc_done[c] < 0 ||
                          prof_step[i] < cyc_done[c];
        if (!real) continue;
        t += ev_ms(prof[2 * i], prof[2 * i + 1]);
        ++cnt;
    }
    rep->n_matvec = cnt;
    rep->ms_matvec = t;
    rep->bytes_matvec = bytes;
    rep->n_hist = (int32_t)std::min<size_t>(hist.size(), WWBI_HIST_MAX);
    for (int i = 0; i < rep->n_hist; ++i) rep->resid_hist[i] = hist[i];
}

// ---------------------------------------------------------------------------
// several right-hand sides in lockstep
// ---------------------------------------------------------------------------

int Ctx::ensure_multi(int n, int nr, int restart) {
    const size_t ldv = (size_t)round_up(n, 64), rr = (size_t)restart;
    const size_t ldp = rr + 1;
    int rc = WWBI_OK;
    MultiWS &m = mw;
    auto G = [&](double *&p, size_t &c, size_t w) { if (rc == WWBI_OK) rc = grow(p, c, w); };
    auto Gf = [&](float *&p, size_t &c, size_t w) { if (rc == WWBI_OK) rc = grow(p, c, w); };
    G(m.V, m.cV, nr * (rr + 1) * ldv);
    Gf(m.v32, m.cv32, nr * ldv);
    Gf(m.x32, m.cx32, nr * ldv);
    G(m.w, m.cw, nr * ldv);
    G(m.r, m.cr, nr * ldv);
    G(m.x, m.cx, nr * ldv);
    G(m.b, m.cb, nr * ldv);
    G(m.d, m.cd, nr * ldv);
    G(m.rr, m.crr, nr * ldv);
    G(m.P, m.cP, nr * 3 * 64 * ldp);
    G(m.H, m.cH, nr * ldp * ldp);
    G(m.cs, m.ccs, nr * (rr + 2));
    G(m.sn, m.csn, nr * (rr + 2));
    G(m.g, m.cg, nr * (rr + 2));
    G(m.y, m.cy, nr * (rr + 2));
    G(m.part, m.cpart, (size_t)multi_part_size(n, nr) + 64);
    G(m.nrm, m.cnrm, nr * 64 + 64);
    if (rc == WWBI_OK && (m.cgs < (size_t)nr || !m.gs)) {
        if (m.gs) hipFree(m.gs);
        m.gs = nullptr;
        m.cgs = 0;
        if (hipMalloc((void **)&m.gs, sizeof(GState) * nr) != hipSuccess) {
            (void)hipGetLastError();
            return WWBI_ECAPACITY;
        }
        m.cgs = nr;
    }
    return rc;
}

// Y_s = c_s - A X_s (or A X_s) with the stored matrix of the given kind.
void Ctx::apply_multi(int kind, int n, long ld, const double *X, const float *X32, long xs, int nr,
                      const double *c, double *Y) {
    const long ldv = round_up(n, 64);
    if (kind == OP_A_S64) {
        launch_mfma_multi64((const double *)A, ld, n, X, xs, nr, c, ldv, Y, ldv, mw.part, stream);
    } else {
        if (!X32) {
            launch_to_f32_batched(X, xs, mw.x32, ldv, n, nr, stream);
            X32 = mw.x32;
            xs = ldv;
        }
        launch_mfma_multi32((const float *)A, ld, n, X32, xs, nr, c, ldv, Y, ldv, mw.part, stream);
    }
}

int Ctx::read_states(GState *out, int nr) {
    GState *slot = reinterpret_cast<GState *>((char *)hst + kStateSlotOffset);
    if (hipMemcpyAsync(slot, mw.gs, sizeof(GState) * nr, hipMemcpyDeviceToHost, stream) !=
        hipSuccess)
        return WWBI_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return WWBI_EHIP;
    std::memcpy(out, slot, sizeof(GState) * nr);
    return WWBI_OK;
}

// nr restarted GMRES solves in lockstep sharing every matrix pass (the matrix
// is read once per Arnoldi step for all systems).  B and X are batched with
// stride round_up(n, 64); X starts at zero.
int Ctx::gmres_multi(int kind, int n, long ld, const double *B, double *X, int nr, double tol,
                     int restart, int max_iter, int poll, bool verify, SolveStats &st) {
    const int G = gmres_nblocks(n);
    const int ldp = restart + 1;
    const long ldv = round_up(n, 64);
    MultiWS &m = mw;
    const Bat bt{nr, (long)(restart + 1) * ldv, ldv, ldv, 3L * 64 * ldp, (long)ldp * ldp,
                 (long)restart + 2};
    double *P1 = m.P, *P2 = m.P + 64 * ldp, *P3 = m.P + 2 * 64 * ldp;
    float *x32 = kind == OP_A_S32 ? m.v32 : nullptr;
    launch_fill(X, 0.0, (int)(nr * ldv), stream);
    launch_norm_partial(B, n, P3, G, stream, bt);
    launch_set_tol(P3, G, tol, m.gs, stream, bt);
    std::vector<GState> h(nr);
    bool first = true;
    double prev = HUGE_VAL;
    int status = WWBI_NOT_CONVERGED;
    GState *slot = reinterpret_cast<GState *>((char *)hst + kStateSlotOffset);
    for (;;) {
        if (first)
            launch_copy(m.r, B, (int)(nr * ldv), stream);
        else
            apply_multi(kind, n, ld, X, nullptr, ldv, nr, B, m.r);
        launch_norm_partial(m.r, n, P3, G, stream, bt);
        launch_cycle_start(m.r, n, P3, G, m.V, x32, m.g, restart + 1, m.gs, 0, nullptr,
                           stream, bt);
        int rc;
        double worst = 0.0;
        // an inner solve (one cycle, no verification) leaves the per-system
        // flags to the device and reads the states once, after its cycle
        if (verify || !first) {
            rc = read_states(h.data(), nr);
            if (rc) return rc;
            bool any = false;
            double bsum = 0.0;
            for (int s = 0; s < nr; ++s) {
                any = any || h[s].active;
                worst = std::max(worst, h[s].bnorm > 0 ? h[s].beta / h[s].bnorm : 0.0);
                bsum += h[s].beta;
            }
            st.rel_resid = worst;
            if (!any) { status = WWBI_OK; break; }
            if (!std::isfinite(bsum)) { status = WWBI_STAGNATED; break; }
            if (st.iters >= max_iter) { status = WWBI_NOT_CONVERGED; break; }
            if (!first && bsum > 0.99 * prev) { status = WWBI_STAGNATED; break; }
            prev = bsum;
        }
        const int jmax = std::min(restart, max_iter - st.iters);
        int pending = -1;
        bool ended = false;
        for (int j0 = 0; j0 < jmax && !ended; j0 += poll) {
            const int j1 = std::min(jmax, j0 + poll);
            for (int j = j0; j < j1; ++j) {
                // the product's K-split slices are summed by the first Gram-Schmidt kernel
                prof_begin();
                const int ks =
                    kind == OP_A_S64
                        ? launch_mfma_parts64((const double *)A, ld, n, m.V + (long)j * ldv,
                                              bt.v, nr, m.part, stream)
                        : launch_mfma_parts32((const float *)A, ld, n, x32, ldv, nr, m.part,
                                              stream);
                prof_end();
                launch_cgs_dot(m.V, ldv, m.w, n, j, P1, P3, G, m.gs, stream, bt, m.part, ks, nr);
                if (x32) {
                    // FP32 inner solves: one Gram-Schmidt pass, as for one system
                    launch_cgs_final(m.V, ldv, m.w, n, j, P1, P3, G, x32, m.H, ldp, false, m.cs,
                                     m.sn, m.g, jmax, m.gs, 0, nullptr, stream, bt);
                } else {
                    launch_cgs_first(m.V, ldv, m.w, n, j, P1, P2, P3, G, m.H, ldp, m.gs, stream,
                                     bt);
                    launch_cgs_final(m.V, ldv, m.w, n, j, P2, P3, G, x32, m.H, ldp, true, m.cs,
                                     m.sn, m.g, jmax, m.gs, 0, nullptr, stream, bt);
                }
            }
            const int cur = (j0 / poll) & 1;
            GState *dst = reinterpret_cast<GState *>((char *)slot + cur * kStateSlotBytes);
            if (hipMemcpyAsync(dst, m.gs, sizeof(GState) * nr, hipMemcpyDeviceToHost, stream) !=
                hipSuccess)
                return WWBI_EHIP;
            if (hipEventRecord(pollev[cur], stream) != hipSuccess) return WWBI_EHIP;
            if (pending >= 0) {
                if (hipEventSynchronize(pollev[pending]) != hipSuccess) return WWBI_EHIP;
                const GState *ps =
                    reinterpret_cast<const GState *>((char *)slot + pending * kStateSlotBytes);
                bool act = false;
                for (int s = 0; s < nr; ++s) act = act || ps[s].active;
                if (!act) ended = true;
            }
            pending = cur;
        }
        // the states are read after the update (a full synchronisation)
        launch_hsolve(m.H, ldp, m.g, m.y, m.gs, stream, bt);
        launch_xupdate(X, m.V, ldv, n, m.y, false, m.gs, stream, bt);
        rc = read_states(h.data(), nr);
        if (rc) return rc;
        int jd = 0;
        bool all_ok = true;
        worst = 0.0;
        for (int s = 0; s < nr; ++s) {
            jd = std::max(jd, h[s].jdone);
            all_ok = all_ok && h[s].resid <= h[s].tol_abs;
            worst = std::max(worst, h[s].bnorm > 0 ? h[s].resid / h[s].bnorm : 0.0);
        }
        st.iters += jd;
        st.cycles += 1;
        first = false;
        if (!verify) {
            st.rel_resid = worst;
            status = all_ok ? WWBI_OK : WWBI_NOT_CONVERGED;
            break;
        }
    }
    return status;
}

// FP64 refinement of nr systems around batched FP32 inner solves.  With
// stored64 the FP64 residuals of all systems come from one matrix-core pass
// over the FP64 copy A64; otherwise each is formed on the fly.
int Ctx::refine_multi(int n, long ld, const double *B, double *X, int nr, const wwbi_opts &o,
                      bool stored64, SolveStats &st) {
    const long ldv = round_up(n, 64);
    const int G = gmres_nblocks(n);
    MultiWS &m = mw;
    const Bat bn{nr, 0, 0, ldv, 64, 0, 0};
    launch_fill(X, 0.0, (int)(nr * ldv), stream);
    auto norms = [&](const double *v, std::vector<double> &out) -> int {
        launch_norm_partial(v, n, m.nrm, G, stream, bn);
        double *h = (double *)hst;
        if (hipMemcpyAsync(h, m.nrm, sizeof(double) * 64 * nr, hipMemcpyDeviceToHost, stream) !=
            hipSuccess)
            return WWBI_EHIP;
        if (hipStreamSynchronize(stream) != hipSuccess) return WWBI_EHIP;
        out.assign(nr, 0.0);
        for (int s = 0; s < nr; ++s) {
            double a = 0.0;
            for (int b = 0; b < G; ++b) a += h[s * 64 + b];
            out[s] = std::sqrt(a);
        }
        return WWBI_OK;
    };
    std::vector<double> bnrm, rn, prev(nr, HUGE_VAL);
    int rc = norms(B, bnrm);
    if (rc) return rc;
    int status = WWBI_NOT_CONVERGED;
    for (int k = 0;; ++k) {
        if (k == 0) {
            launch_copy(m.rr, B, (int)(nr * ldv), stream);
            rn = bnrm;
        } else {
            if (stored64)
                launch_mfma_multi64(A64, ld, n, X, ldv, nr, B, ldv, m.rr, ldv, m.part, stream);
            else
                for (int s = 0; s < nr; ++s)
                    launch_otf_matvec(L, N, o.flags, 0, o.band, 0, X + s * ldv, B + s * ldv,
                                      m.rr + s * ldv, part, nullptr, stream);
            rc = norms(m.rr, rn);
            if (rc) return rc;
        }
        double worst = 0.0;
        bool done = true, stalled = false;
        for (int s = 0; s < nr; ++s) {
            const double rel = bnrm[s] > 0 ? rn[s] / bnrm[s] : 0.0;
            worst = std::max(worst, rel);
            done = done && rel <= o.tol;
            stalled = stalled || !std::isfinite(rn[s]) ||
                      (k > 0 && rel > o.tol && rn[s] > 0.5 * prev[s]);
        }
        st.rel_resid = worst;
        note_resid(worst);
        if (done) { status = WWBI_OK; break; }
        if (stalled) { status = WWBI_REFINE_STALLED; break; }
        if (k >= o.max_refine || st.iters >= o.max_iter) { status = WWBI_NOT_CONVERGED; break; }
        prev = rn;
        SolveStats in{};
        in.iters = st.iters;
        double itol = 0.0;
        for (int s = 0; s < nr; ++s)
            if (bnrm[s] > 0 && rn[s] > o.tol * bnrm[s])
                itol = std::max(itol, inner_tolerance(o, bnrm[s], rn[s]));
        // the matrix-core products accumulate in FP32, which holds their
        // contraction near kMulti32Floor
        itol = std::max(itol > 0 ? itol : o.inner_tol, kMulti32Floor);
        rc = gmres_multi(OP_A_S32, n, ld, m.rr, m.d, nr, itol, o.restart, o.max_iter,
                         o.poll_every, false, in);
        if (rc < 0) return rc;
        st.iters = in.iters;
        st.cycles += in.cycles;
        st.refine_steps += 1;
        launch_axpy(X, m.d, (int)(nr * ldv), 1.0, stream);
    }
    return status;
}

}  // namespace wwbi

// ---------------------------------------------------------------------------
// C entry points
// ---------------------------------------------------------------------------

extern "C" {

void wwbi_default_opts(wwbi_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-13;
    o->inner_tol = 1e-7;
    o->restart = 100;
    o->max_iter = 2000;
    o->precision = WWBI_FP64;
    o->matvec = WWBI_MATVEC_AUTO;
    o->poll_every = 2;
    o->max_refine = 8;
    o->band = 16;
    o->flags = 0;
    o->x0 = nullptr;
}

const char *wwbi_status_str(int s) {
    switch (s) {
    case WWBI_OK: return "ok";
    case WWBI_EINVAL_NULL: return "invalid argument: null pointer";
    case WWBI_EINVAL_SIZE: return "invalid argument: sizes (nb, or M_k odd or < 8)";
    case WWBI_EINVAL_NONFINITE: return "invalid argument: non-finite input";
    case WWBI_EINVAL_ORIENTATION: return "invalid argument: boundary orientation";
    case WWBI_ECAPACITY: return "out of device memory";
    case WWBI_EHIP: return "HIP runtime error";
    case WWBI_EINVAL_OPTS: return "invalid options";
    case WWBI_EINVAL_RANGE: return "invalid argument: a node lies more than 30 above or below y = 0";
    case WWBI_ESCRATCH: return "workspace exceeds the allocation-free entry point's static scratch";
    case WWBI_NOT_CONVERGED: return "not converged";
    case WWBI_STAGNATED: return "stagnated";
    case WWBI_REFINE_STALLED: return "iterative refinement stalled";
    case WWBI_WARN_UNDERRESOLVED: return "warning: omega not resolved by the grid (Fourier tail)";
    default: return "unknown status";
    }
}

int wwbi_create(wwbi_ctx **out, int32_t device, void *stream) {
    if (!out) return WWBI_EINVAL_NULL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return WWBI_EHIP;
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return WWBI_ECAPACITY;
    c->device = device;
    c->stream = (hipStream_t)stream;
    // the per-cycle bookkeeping never grows inside a solve of up to 4096 cycles
    c->cyc_done.reserve(4096);
    c->hist.reserve(WWBI_HIST_MAX);
    // device address of the allocation-free entry point's static scratch array
    scratch_init(device);
    int rc = WWBI_OK;
    if (hipMalloc((void **)&c->gs, sizeof(GState)) != hipSuccess) rc = WWBI_ECAPACITY;
    if (!rc && hipHostMalloc(&c->hst, kHostStaging) != hipSuccess) rc = WWBI_ECAPACITY;
    if (!rc && hipHostMalloc((void **)&c->hmir, sizeof(GState),
                             hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        rc = WWBI_ECAPACITY;
    if (!rc) {
        std::memset(c->hmir, 0, sizeof(GState));
        if (hipHostGetDevicePointer((void **)&c->dmir, c->hmir, 0) != hipSuccess) rc = WWBI_EHIP;
    }
    // the phase markers and the matvec timing pairs only time (the report is
    // read after a full synchronisation of the stream), so they skip the
    // system-scope fence, whose cache write-back would be timed with the work
    for (auto &e : c->ev)
        if (!rc && hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
            rc = WWBI_EHIP;
    for (auto &e : c->prof)
        if (!rc && hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
            rc = WWBI_EHIP;
    for (auto &e : c->pollev)
        if (!rc && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = WWBI_EHIP;
    for (auto &e : c->stepev)
        if (!rc && hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence) !=
                       hipSuccess)
            rc = WWBI_EHIP;
    if (rc) {
        c->release();
        delete c;
        return rc;
    }
    *out = reinterpret_cast<wwbi_ctx *>(c);
    return WWBI_OK;
}

int wwbi_set_stream(wwbi_ctx *ctx, void *stream) {
    if (!ctx) return WWBI_EINVAL_NULL;
    reinterpret_cast<Ctx *>(ctx)->stream = (hipStream_t)stream;
    return WWBI_OK;
}

int wwbi_destroy(wwbi_ctx *ctx) {
    if (!ctx) return WWBI_OK;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    hipStreamSynchronize(c->stream);
    c->release();
    delete c;
    return WWBI_OK;
}

int wwbi_reserve(wwbi_ctx *ctx, int64_t max_unknowns, int32_t max_restart, int32_t precision) {
    if (!ctx) return WWBI_EINVAL_NULL;
    if (max_unknowns < 8 || max_unknowns > (1L << 28)) return WWBI_EINVAL_SIZE;
    if (max_restart < 1 || max_restart > WWBI_MAX_RESTART) return WWBI_EINVAL_OPTS;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->restart_cap = std::max(c->restart_cap, (int)max_restart);
    int rc = c->ensure((int)max_unknowns, c->restart_cap);
    if (rc) return rc;
    if (precision >= 0) {
        const size_t ld = round_up((long)max_unknowns, 64);
        const size_t es = precision == WWBI_FP64 ? 8 : 4;
        rc = c->ensure_matrix((size_t)max_unknowns * ld * es);
    }
    return rc;
}

}  // extern "C"

namespace wwbi {

int solve_phi_impl(Ctx *c, const wwbi_geom *g, const double *phi, const wwbi_opts *o,
                   double *U, double *omega, double *psi_k, wwbi_report *rep) {
    SolveStats st{};
    int rc = Ctx::check_opts(o);
    if (!rc && (!phi || !U)) rc = WWBI_EINVAL_NULL;
    if (!rc) {
        c->restart_cap = std::max(c->restart_cap, o->restart);
        c->begin_report((o->flags & WWBI_FLAG_PROFILE) != 0);
        rc = c->setup(g, phi, g ? g->M[0] : 0, false);
    }
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    const int n = c->L.n;
    const long ld = round_up(n, 64);
    double *b = c->vec[VB], *x = c->vec[VX];
    // the right-hand side, circulant rows and matrix go into internal buffers
    // only, so they are queued before the input checks are read back
    launch_rhs_phi(c->L, c->N, c->F, phi, c->psi_wall, b, c->stream);
    launch_circulant_rows(c->L, WWBI_OP_D, c->rowD, c->stream);
    launch_circulant_rows(c->L, WWBI_OP_H, c->rowH, c->stream);
    hipEventRecord(c->ev[1], c->stream);
    const bool stored = o->matvec != WWBI_MATVEC_ON_THE_FLY;
    const bool fp32 = o->precision == WWBI_FP32_REFINED;
    if (stored) {
        rc = c->ensure_matrix((size_t)n * ld * (fp32 ? 4 : 8));
        if (rc) { c->finish_report(rep, rc, st, 0); return rc; }
        if (fp32)
            launch_assemble32(c->L, c->N, o->flags, o->band, (float *)c->A, ld, c->stream);
        else
            launch_assemble64(c->L, c->N, o->flags, (double *)c->A, ld, c->stream);
    }
    hipEventRecord(c->ev[2], c->stream);
    rc = c->setup_check();
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    const bool xz = o->x0 == nullptr;
    if (!xz) launch_copy(x, o->x0, n, c->stream);
    Op op64{stored ? OP_A_S64 : OP_A_O64, n, ld, o->flags, o->band};
    int status;
    double bytes;
    if (!fp32) {
        status = c->gmres(op64, b, x, xz, o->tol, o->restart, o->max_iter, o->poll_every, true, st);
        bytes = c->op_bytes(op64);
    } else {
        Op op32{stored ? OP_A_S32 : OP_A_O32, n, ld, o->flags, o->band};
        Op opres{OP_A_O64, n, ld, o->flags, o->band};
        status = c->refine(op32, opres, b, x, xz, *o, st);
        bytes = c->op_bytes(op32);
    }
    hipEventRecord(c->ev[3], c->stream);
    if (status < 0) { c->finish_report(rep, status, st, bytes); return status; }
    double *gam = c->vec[VG];
    c->gamma_from_omega(x, gam);
    c->eval_U_from_gamma(gam, U);
    if (omega) launch_copy(omega, x, n, c->stream);
    if (psi_k && c->L.nb > 2) {
        double *means = c->vec[VTMP];
        launch_block_means(c->L, x, means, c->stream);
        hipMemcpyAsync(c->hst, means, sizeof(double) * (c->L.nb - 2), hipMemcpyDeviceToHost,
                       c->stream);
    }
    // resolution check: the Fourier tail of omega on every boundary
    double *tails = (double *)((char *)c->hst + kTailOffset);
    launch_tail_monitor(c->L, x, c->part, c->val, c->stream);
    hipMemcpyAsync(tails, c->val, sizeof(double) * 2 * c->L.nb, hipMemcpyDeviceToHost, c->stream);
    hipEventRecord(c->ev[4], c->stream);
    c->finish_report(rep, status, st, bytes);
    if (psi_k && c->L.nb > 2) std::memcpy(psi_k, c->hst, sizeof(double) * (c->L.nb - 2));
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    // per boundary: the root of its tail energy over M_k^2 times the largest
    // mean square of omega on any boundary, i.e. its tail in units of the
    // solution's scale.  On the boundary carrying that largest mean square this
    // is the energy fraction of its own tail; a boundary whose omega is at the
    // solver's noise level (a bottom far below the surface) is not flagged by
    // the spectrum of that noise
    double tail = 0.0, smax = 0.0;
    bool finite = true;
    for (int k = 0; k < c->L.nb; ++k) {
        const double M = (double)(c->L.off[k + 1] - c->L.off[k]);
        smax = std::max(smax, tails[2 * k + 1] / (M * M));
        finite = finite && std::isfinite(tails[2 * k]) && std::isfinite(tails[2 * k + 1]);
    }
    for (int k = 0; k < c->L.nb && smax > 0.0; ++k) {
        const double M = (double)(c->L.off[k + 1] - c->L.off[k]);
        tail = std::max(tail, std::sqrt(tails[2 * k] / (smax * M * M)));
    }
    if (!finite || !std::isfinite(tail)) tail = HUGE_VAL;
    if (status == WWBI_OK && tail > std::max(1e-12, 10.0 * o->tol))
        status = WWBI_WARN_UNDERRESOLVED;
    if (rep) {
        rep->tail_ratio = tail;
        rep->status = status;
    }
    return status;
}

}  // namespace wwbi

extern "C" {

int wwbi_solve_phi(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi, const wwbi_opts *o,
                   double *U, double *omega, double *psi_k, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    return solve_phi_impl(reinterpret_cast<Ctx *>(ctx), g, phi, o, U, omega, psi_k, rep);
}

int wwbi_solve_gamma(wwbi_ctx *ctx, const wwbi_geom *g, const double *gamma0, const wwbi_opts *o,
                     double *U, double *gamma_wall, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    SolveStats st{};
    int rc = Ctx::check_opts(o);
    if (!rc && (!gamma0 || !U)) rc = WWBI_EINVAL_NULL;
    if (!rc) {
        c->restart_cap = std::max(c->restart_cap, o->restart);
        c->begin_report((o->flags & WWBI_FLAG_PROFILE) != 0);
        rc = c->setup(g, gamma0, g ? g->M[0] : 0);
    }
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    const int n = c->L.n, n0 = c->L.off[1], nw = n - n0;
    const long ldw = round_up(nw, 64);
    double *gam = c->vec[VG], *rhs = c->vec[VB], *um = c->vec[VUM];
    launch_circulant_rows(c->L, WWBI_OP_H, c->rowH, c->stream);
    // wall right-hand side: -G_0k^dagger gamma_0 - s dphi_mv/dn on every wall
    launch_umv(c->N, c->F, n0, nw, um, c->stream);
    launch_rflavour(c->L, c->N, c->hrow, 2, 0, n0, nw, 0, n0, gamma0, c->part, nullptr, c->stream);
    launch_wall_rhs_finalize(nw, um, c->part, rflavour_nsplit(c->N, nw, n0, 0), rhs, c->stream);
    hipEventRecord(c->ev[1], c->stream);
    // the wall operator: GMRES in FP64 (stored or on the fly), or (stored,
    // FP32_REFINED) FP32 products inside FP64 refinement with on-the-fly FP64
    // residuals
    const bool stored = o->matvec != WWBI_MATVEC_ON_THE_FLY;
    const bool refined = stored && o->precision == WWBI_FP32_REFINED;
    if (stored) {
        rc = c->ensure_matrix((size_t)nw * ldw * (refined ? 4 : 8));
        if (rc) { c->finish_report(rep, rc, st, 0); return rc; }
        if (refined)
            launch_assemble_wall32(c->L, c->N, c->hrow, (float *)c->A, ldw, c->stream);
        else
            launch_assemble_wall64(c->L, c->N, c->hrow, (double *)c->A, ldw, c->stream);
    }
    hipEventRecord(c->ev[2], c->stream);
    double *gw = gam + n0;
    const bool xz = o->x0 == nullptr;
    if (!xz) launch_copy(gw, o->x0, nw, c->stream);
    Op op{refined ? OP_W_S32 : (stored ? OP_W_S64 : OP_W_O64), nw, ldw, o->flags, o->band};
    int status;
    if (refined) {
        const Op op64{OP_W_O64, nw, ldw, o->flags, o->band};
        status = c->refine(op, op64, rhs, gw, xz, *o, st);
    } else {
        status = c->gmres(op, rhs, gw, xz, o->tol, o->restart, o->max_iter, o->poll_every,
                          true, st);
    }
    hipEventRecord(c->ev[3], c->stream);
    if (status < 0) { c->finish_report(rep, status, st, c->op_bytes(op)); return status; }
    launch_copy(gam, gamma0, n0, c->stream);
    c->eval_U_from_gamma(gam, U);
    if (gamma_wall) launch_copy(gamma_wall, gw, nw, c->stream);
    hipEventRecord(c->ev[4], c->stream);
    c->finish_report(rep, status, st, c->op_bytes(op));
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    return status;
}

int wwbi_tangential_energy(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi,
                           const double *omega, double tau, double grav, double *dphids,
                           double *energy, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    SolveStats st{};
    int rc = WWBI_OK;
    if (!omega || (!dphids && !energy) || (energy && !phi)) rc = WWBI_EINVAL_NULL;
    if (!rc && energy && !(std::isfinite(tau) && std::isfinite(grav))) rc = WWBI_EINVAL_NONFINITE;
    if (!rc) {
        c->begin_report(false);
        rc = c->setup(g, energy ? phi : nullptr, g ? g->M[0] : 0);
    }
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    hipStream_t sm = c->stream;
    const int n = c->L.n, n0 = c->L.off[1];
    double *gam = c->vec[VG], *tm = c->vec[VUM], *hg = c->vec[VHG];
    launch_circulant_rows(c->L, WWBI_OP_D, c->rowD, sm);
    launch_circulant_rows(c->L, WWBI_OP_H, c->rowH, sm);
    launch_tmv(c->N, c->F, 0, n, tm, sm);
    hipEventRecord(c->ev[1], sm);
    hipEventRecord(c->ev[2], sm);
    if (dphids) {
        // s dphi/ds on every boundary from gamma = (-D omega_0, D omega_j)
        c->gamma_from_omega(omega, gam);
        if (c->L.nb > 1)
            launch_circulant_apply(c->L, c->rowH, gam, hg, 1.0, 0.0, 1, c->L.nb - 1, sm);
        launch_rflavour(c->L, c->N, c->hrow, 5, 0, 0, n, 0, n, gam, c->part, nullptr, sm);
        launch_tangential_finalize(n, n0, c->s, tm, gam, hg, c->part,
                                   rflavour_nsplit(c->N, n, n, 0), dphids, sm);
    }
    hipEventRecord(c->ev[3], sm);
    if (energy) {
        double *hw = c->vec[VTMP], *dphi = c->vec[VTMP2], *e = c->vec[VD];
        double *means = c->vec[VRR], *E = c->val;
        launch_circulant_apply(c->L, c->rowH, omega, hw, 1.0, 0.0, 0, 0, sm);
        launch_circulant_apply(c->L, c->rowD, phi, dphi, 1.0, 0.0, 0, 0, sm);
        launch_block_means(c->L, omega, means, sm);
        launch_rflavour(c->L, c->N, c->hrow, 4, 0, 0, n0, 0, n, omega, c->part, nullptr, sm);
        launch_energy(n0, c->N, c->F, tau, grav, hw, c->part, rflavour_nsplit(c->N, n0, n, 0),
                      dphi, tm, means, e, E, sm);
        if (hipMemcpyAsync(c->hst, E, sizeof(double), hipMemcpyDeviceToHost, sm) != hipSuccess)
            return WWBI_EHIP;
    }
    hipEventRecord(c->ev[4], sm);
    c->finish_report(rep, WWBI_OK, st, 0.0);
    if (energy) std::memcpy(energy, c->hst, sizeof(double));
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    return WWBI_OK;
}

int wwbi_solve_gamma_t(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi, const double *V,
                       double tau, double grav, const wwbi_opts *o, double *gamma_t, double *U,
                       wwbi_report *rep_phi, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    SolveStats st{};
    int rc = Ctx::check_opts(o);
    if (!rc && (!phi || !V || !gamma_t)) rc = WWBI_EINVAL_NULL;
    if (!rc && !(std::isfinite(tau) && std::isfinite(grav))) rc = WWBI_EINVAL_NONFINITE;
    if (!rc && (!g || !g->M)) rc = WWBI_EINVAL_NULL;
    if (!rc && (g->nb < 2 || g->nb > kMaxB)) rc = WWBI_EINVAL_SIZE;
    long nsum = 0;
    for (int k = 0; !rc && k < g->nb; ++k) {
        if (g->M[k] < 8 || (g->M[k] & 1)) rc = WWBI_EINVAL_SIZE;
        nsum += g->M[k];
    }
    if (!rc && nsum > (1L << 28)) rc = WWBI_EINVAL_SIZE;
    if (!rc) {
        // size the workspace before the velocity-potential solve: it writes
        // into workspace vectors, which must not move when the workspace grows
        c->restart_cap = std::max(c->restart_cap, o->restart);
        rc = c->ensure((int)nsum, c->restart_cap);
    }
    if (rc) {
        if (rep_phi) { std::memset(rep_phi, 0, sizeof(*rep_phi)); rep_phi->status = rc; }
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    // 1. velocity-potential solve at the current state: omega and U
    wwbi_report r1{};
    const int s1 = solve_phi_impl(c, g, phi, o, c->vec[VU0], c->vec[VOM], nullptr, &r1);
    if (rep_phi) *rep_phi = r1;
    if (s1 < 0) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = s1; }
        return s1;
    }
    hipStream_t sm = c->stream;
    const Layout &L = c->L;
    const int n = L.n, n0 = L.off[1], nw = n - n0;
    const long ld = round_up(n, 64);
    double *om = c->vec[VOM], *u0 = c->vec[VU0], *gam = c->vec[VG];
    double *fV = c->vec[VFV], *fU = c->vec[VFU], *kfv = c->vec[VKF], *gfu = c->vec[VGF];
    double *hfu = c->vec[VHF], *qg = c->vec[VQG], *tm = c->vec[VTM], *e = c->vec[VE];
    double *b = c->vec[VB], *x = c->vec[VX];
    c->begin_report((o->flags & WWBI_FLAG_PROFILE) != 0);
    // 2. right-hand side (Sec. 4.2)
    c->gamma_from_omega(om, gam);
    launch_tmv(c->N, c->F, 0, n0, tm, sm);
    launch_rflavour(L, c->N, c->hrow, 5, 0, 0, n0, 0, n, gam, c->part, nullptr, sm);
    launch_reduce_partials(n0, c->part, rflavour_nsplit(c->N, n0, n, 0), nullptr, 1.0, qg,
                           nullptr, sm);
    launch_gt_vectors(n0, V, u0, gam, c->s, fV, fU, sm);
    launch_circulant_apply(L, c->rowH, fU, hfu, 1.0, 0.0, 0, 0, sm);
    const int nss = rflavour_nsplit(c->N, n0, n0, 0), nsw = rflavour_nsplit(c->N, nw, n0, 0);
    launch_rflavour(L, c->N, c->hrow, 6, 0, 0, n0, 0, n0, fV, c->part, nullptr, sm);
    launch_reduce_partials(n0, c->part, nss, nullptr, 1.0, kfv, nullptr, sm);
    launch_rflavour(L, c->N, c->hrow, 7, 0, 0, n0, 0, n0, fU, c->part, nullptr, sm);
    launch_reduce_partials(n0, c->part, nss, nullptr, 1.0, gfu, nullptr, sm);
    launch_gt_surface(n0, c->N, tau, grav, V, u0, gam, tm, qg, 1, hfu, kfv, gfu, e, sm);
    if (nw > 0) {
        // wall k: -F_k0 gamma_0 = KS fU - GS fV
        launch_rflavour(L, c->N, c->hrow, 6, 0, n0, nw, 0, n0, fU, c->part, nullptr, sm);
        launch_reduce_partials(nw, c->part, nsw, nullptr, 1.0, e + n0, nullptr, sm);
        launch_rflavour(L, c->N, c->hrow, 7, 0, n0, nw, 0, n0, fV, c->part, nullptr, sm);
        launch_reduce_partials(nw, c->part, nsw, e + n0, 1.0, e + n0, nullptr, sm);
    }
    launch_circulant_apply(L, c->rowD, e, b, 1.0, 0.0, 0, L.nb - 1, sm);
    hipEventRecord(c->ev[1], sm);
    // 3. the gamma_t operator, stored or on the fly: GMRES in FP64, or (stored,
    // FP32_REFINED) FP32 products inside FP64 refinement with on-the-fly
    // FP64 residuals
    const bool stored = o->matvec != WWBI_MATVEC_ON_THE_FLY;
    const bool refined = stored && o->precision == WWBI_FP32_REFINED;
    if (stored) {
        rc = c->ensure_matrix((size_t)n * ld * (refined ? 4 : 8));
        if (rc) { c->finish_report(rep, rc, st, 0); return rc; }
        if (refined)
            launch_assemble_gt32(L, c->N, (float *)c->A, ld, sm);
        else
            launch_assemble_gt64(L, c->N, (double *)c->A, ld, sm);
    }
    hipEventRecord(c->ev[2], sm);
    Op op{refined ? OP_GT_S32 : (stored ? OP_GT_S64 : OP_GT_O64), n, ld, o->flags, o->band};
    int status;
    if (refined) {
        const Op op64{OP_GT_O64, n, ld, o->flags, o->band};
        status = c->refine(op, op64, b, x, true, *o, st);
    } else {
        status = c->gmres(op, b, x, true, o->tol, o->restart, o->max_iter, o->poll_every, true, st);
    }
    hipEventRecord(c->ev[3], sm);
    if (status < 0) { c->finish_report(rep, status, st, c->op_bytes(op)); return status; }
    launch_copy(gamma_t, x, n, sm);
    if (U) launch_copy(U, u0, n0, sm);
    hipEventRecord(c->ev[4], sm);
    c->finish_report(rep, status, st, c->op_bytes(op));
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    return status != WWBI_OK ? status : s1;
}

// ---------------------------------------------------------------------------
// evolution of the free surface: one Runge-Kutta stage and one step
// (Sec. 2.1, 2.2, 3.5, 5)
// ---------------------------------------------------------------------------

namespace {
enum EvVec { EW_U = 0, EW_V, EW_T1, EW_T2, EW_T3, EW_T4, EW_DPHI, EW_SC, kEw };
}

// Workspace and the D / antiderivative / filter rows of the M_0 grid.
static int evolve_prepare(Ctx *c, int M0) {
    const size_t M = (size_t)M0;
    int rc = grow(c->ew, c->capew, kEw * M + 64);
    if (!rc && c->ev_M != M0) {
        rc = grow(c->evrow, c->capevrow, 4 * M + 64);
        if (!rc) {
            launch_circ_row1(M0, WWBI_OP_D, c->evrow, c->stream);
            launch_evolve_rows(M0, c->evrow + 3 * M, c->evrow + M, c->evrow + 2 * M, c->stream);
            c->ev_M = M0;
        }
    }
    return rc;
}

static int check_stage_geom(const wwbi_geom *g, int mode) {
    if (!g || !g->M || !g->x || !g->y || !g->dx || !g->dy || !g->ddx || !g->ddy)
        return WWBI_EINVAL_NULL;
    if (g->nb < 2 || g->nb > kMaxB) return WWBI_EINVAL_SIZE;
    if (g->M[0] < 8 || (g->M[0] & 1)) return WWBI_EINVAL_SIZE;
    if (mode != WWBI_SURF_GRAPH && mode != WWBI_SURF_HLS) return WWBI_EINVAL_OPTS;
    return WWBI_OK;
}

// Surface of the stage state written into the first M_0 entries of the
// geometry arrays, the velocity-potential solve there, then the rates.
static int stage_impl(Ctx *c, const wwbi_geom *g, int mode, const double *q, const double *phi,
                      double tau, double grav, const wwbi_opts *o, double *qt, double *phit,
                      double *Uout, double *Vout, wwbi_report *rep) {
    const int M0 = g->M[0];
    const size_t M = (size_t)M0;
    int rc = evolve_prepare(c, M0);
    if (rc) return rc;
    hipStream_t st = c->stream;
    double *x = const_cast<double *>(g->x), *y = const_cast<double *>(g->y);
    double *dx = const_cast<double *>(g->dx), *dy = const_cast<double *>(g->dy);
    double *ddx = const_cast<double *>(g->ddx), *ddy = const_cast<double *>(g->ddy);
    const double *rD = c->evrow, *rI = c->evrow + M;
    double *U = c->ew + EW_U * M, *V = c->ew + EW_V * M;
    double *t1 = c->ew + EW_T1 * M, *t2 = c->ew + EW_T2 * M, *t3 = c->ew + EW_T3 * M;
    double *t4 = c->ew + EW_T4 * M, *dphi = c->ew + EW_DPHI * M, *sc = c->ew + EW_SC * M;
    if (mode == WWBI_SURF_GRAPH) {
        // zeta = alpha + i eta (Sec. 2.1)
        launch_graph_base(M0, q, x, y, dx, ddx, st);
        launch_circ_apply1(M0, rD, q, dy, 1.0, 0.0, st);
        launch_circ_apply1(M0, rD, dy, ddy, 1.0, 0.0, st);
    } else {
        // the curve from P theta (Sec. 2.2)
        launch_mean_cs(M0, q, sc, st);
        launch_hls_slope(M0, q, sc, dx, dy, t1, st);
        launch_circ_apply1(M0, rI, t1, t2, 1.0, 0.0, st);      // xi^aux
        launch_circ_apply1(M0, rI, dy, t3, 1.0, 0.0, st);      // eta^aux
        launch_mean_prod(M0, t3, dx, sc + 2, st);
        launch_hls_xy(M0, t2, t3, sc + 2, x, y, st);
        launch_circ_apply1(M0, rD, q, t4, 1.0, 0.0, st);       // theta_alpha
        launch_hls_curv(M0, t4, dx, dy, ddx, ddy, st);
    }
    wwbi_report r{};
    const int s1 = solve_phi_impl(c, g, phi, o, U, nullptr, nullptr, &r);
    if (rep) *rep = r;
    if (s1 < 0) return s1;
    if (mode == WWBI_SURF_GRAPH) {
        launch_graph_rates(M0, U, dy, V, qt, st);
    } else {
        // V (Sec. 5) and (P theta)_t = P[(U_alpha + V theta_alpha) / s_alpha]
        launch_mul(M0, t4, U, t1, st);
        launch_circ_apply1(M0, rI, t1, t2, 1.0, 0.0, st);
        launch_hls_V(M0, t2, U, dx, dy, V, st);
        launch_circ_apply1(M0, rD, U, t3, 1.0, 0.0, st);
        launch_hls_f(M0, t3, V, t4, dx, dy, t1, st);
        launch_mean_prod(M0, t1, nullptr, sc + 3, st);
        launch_sub_mean(M0, t1, sc + 3, qt, st);
    }
    launch_circ_apply1(M0, rD, phi, dphi, 1.0, 0.0, st);
    launch_phit(M0, c->N, c->F, dphi, U, V, tau, grav, phit, st);
    if (Uout) launch_copy(Uout, U, M0, st);
    if (Vout) launch_copy(Vout, V, M0, st);
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    return s1;
}

int wwbi_stage_rhs(wwbi_ctx *ctx, const wwbi_geom *g, int32_t mode, const double *q,
                   const double *phi, double tau, double grav, const wwbi_opts *o, double *q_t,
                   double *phi_t, double *U, double *V, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    int rc = check_stage_geom(g, mode);
    if (!rc) rc = Ctx::check_opts(o);
    if (!rc && (!q || !phi || !q_t || !phi_t)) rc = WWBI_EINVAL_NULL;
    if (!rc && !(std::isfinite(tau) && std::isfinite(grav))) rc = WWBI_EINVAL_NONFINITE;
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    rc = stage_impl(c, g, mode, q, phi, tau, grav, o, q_t, phi_t, U, V, rep);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return WWBI_EHIP;
    return rc;
}

int wwbi_rk_step(wwbi_ctx *ctx, const wwbi_geom *g, int32_t mode, int32_t nstage,
                 const double *A, const double *b, double h, double *q, double *phi, double tau,
                 double grav, int32_t filter, const wwbi_opts *o, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    int rc = check_stage_geom(g, mode);
    if (!rc) rc = Ctx::check_opts(o);
    if (!rc && (!A || !b || !q || !phi)) rc = WWBI_EINVAL_NULL;
    if (!rc && (nstage < 1 || nstage > kMaxStages)) rc = WWBI_EINVAL_OPTS;
    if (!rc && !(std::isfinite(h) && std::isfinite(tau) && std::isfinite(grav)))
        rc = WWBI_EINVAL_NONFINITE;
    for (int i = 0; !rc && i < nstage; ++i) {
        if (!std::isfinite(b[i])) rc = WWBI_EINVAL_NONFINITE;
        for (int j = 0; j < i; ++j)
            if (!std::isfinite(A[i * nstage + j])) rc = WWBI_EINVAL_NONFINITE;
    }
    const int M0 = rc ? 0 : g->M[0];
    const size_t M = (size_t)M0;
    if (!rc) rc = grow(c->ek, c->capek, (2 * (size_t)nstage + 2) * M + 64);
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = c->stream;
    double *Kq = c->ek, *Kp = c->ek + nstage * M;
    double *qi = c->ek + 2 * nstage * M, *pi = qi + M;
    wwbi_report total{};
    int status = WWBI_OK;
    for (int i = 0; i < nstage; ++i) {
        RkCoef co{};
        co.ns = i;
        co.h = h;
        for (int j = 0; j < i; ++j) co.c[j] = A[i * nstage + j];
        launch_rk_combine(M0, q, Kq, (long)M, co, qi, st);
        launch_rk_combine(M0, phi, Kp, (long)M, co, pi, st);
        wwbi_report r{};
        const int s = stage_impl(c, g, mode, qi, pi, tau, grav, o, Kq + i * M, Kp + i * M,
                                 nullptr, nullptr, &r);
        total.iters += r.iters;
        total.restarts += r.restarts;
        total.refine_steps += r.refine_steps;
        total.rel_resid = std::max(total.rel_resid, r.rel_resid);
        total.n_matvec += r.n_matvec;
        total.ms_matvec += r.ms_matvec;
        total.ms_solve += r.ms_total;
        if (s < 0) { status = s; break; }
        if (s > 0 && status == WWBI_OK) status = s;
    }
    if (status >= 0) {
        RkCoef co{};
        co.ns = nstage;
        co.h = h;
        for (int j = 0; j < nstage; ++j) co.c[j] = b[j];
        launch_rk_combine(M0, q, Kq, (long)M, co, qi, st);
        launch_rk_combine(M0, phi, Kp, (long)M, co, pi, st);
        if (filter) {
            // the 36th-order filter at the end of the step (Sec. 5)
            const double *rF = c->evrow + 2 * M;
            launch_circ_apply1(M0, rF, qi, q, 1.0, 0.0, st);
            launch_circ_apply1(M0, rF, pi, phi, 1.0, 0.0, st);
        } else {
            launch_copy(q, qi, M0, st);
            launch_copy(phi, pi, M0, st);
        }
    }
    const bool ok = hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess;
    total.status = ok ? status : WWBI_EHIP;
    total.ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = total;
    return ok ? status : WWBI_EHIP;
}

// ---------------------------------------------------------------------------
// velocity on the boundaries and inside the fluid (Sec. 4.1, 5.1 and the
// Helsing-Ojala appendix)
// ---------------------------------------------------------------------------

// s dphi/ds and s dphi/dn on every node from the densities omega
static void boundary_derivs(Ctx *c, const double *omega, double *sds, double *sdn) {
    hipStream_t sm = c->stream;
    const Layout &L = c->L;
    const int n = L.n, n0 = L.off[1];
    double *gam = c->vec[VG], *hg = c->vec[VHG], *tm = c->vec[VTM], *um = c->vec[VUM];
    launch_circulant_rows(L, WWBI_OP_D, c->rowD, sm);
    launch_circulant_rows(L, WWBI_OP_H, c->rowH, sm);
    c->gamma_from_omega(omega, gam);
    launch_circulant_apply(L, c->rowH, gam, hg, 1.0, 0.0, 0, L.nb - 1, sm);
    launch_tmv(c->N, c->F, 0, n, tm, sm);
    launch_umv(c->N, c->F, 0, n, um, sm);
    const int ns = rflavour_nsplit(c->N, n, n, 0);
    launch_rflavour(L, c->N, c->hrow, 5, 0, 0, n, 0, n, gam, c->part, nullptr, sm);
    launch_tangential_finalize(n, n0, nullptr, tm, gam, hg, c->part, ns, sds, sm);
    launch_rflavour(L, c->N, c->hrow, 2, 0, 0, n, 0, n, gam, c->part, nullptr, sm);
    launch_normal_finalize(n, n0, um, gam, hg, c->part, ns, sdn, sm);
}

static int interior_common(Ctx *c, const wwbi_geom *g, int32_t npts, const double *zx,
                           const double *zy) {
    if (!zx || !zy) return WWBI_EINVAL_NULL;
    if (npts < 1 || npts > (1 << 26)) return WWBI_EINVAL_SIZE;
    int rc = c->setup(g, nullptr, 0);
    if (rc) return rc;
    // the points: finite, and within the node height limit (a point inside
    // the fluid lies between the bottom and the surface anyway)
    launch_check_points(npts, zx, zy, c->val, c->stream);
    if (hipMemcpyAsync(c->hst, c->val, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return WWBI_EHIP;
    const double *h = (const double *)c->hst;
    if (h[0] != 0.0) return WWBI_EINVAL_NONFINITE;
    if (h[1] != 0.0) return WWBI_EINVAL_RANGE;
    const size_t ns = (size_t)ho_slices(npts, c->L.n);
    rc = grow(c->hop, c->caphop, 4 * ns * npts + 64);
    if (!rc) rc = grow(c->hoi, c->caphoi, ns * npts + 64);
    return rc;
}

int wwbi_boundary_velocity(wwbi_ctx *ctx, const wwbi_geom *g, const double *omega, double *u,
                           double *v) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!omega || !u || !v) return WWBI_EINVAL_NULL;
    int rc = c->setup(g, nullptr, 0);
    if (rc) return rc;
    double *sds = c->vec[VE], *sdn = c->vec[VQG];
    boundary_derivs(c, omega, sds, sdn);
    launch_boundary_velocity(c->L.n, g->dx, g->dy, sds, sdn, false, u, v, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return WWBI_EHIP;
    return hip_ok(hipGetLastError());
}

int wwbi_interior_eval(wwbi_ctx *ctx, const wwbi_geom *g, const double *f_re,
                       const double *f_im, int32_t npts, const double *zx, const double *zy,
                       double *out_re, double *out_im) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!f_re || !f_im || !out_re || !out_im) return WWBI_EINVAL_NULL;
    int rc = interior_common(c, g, npts, zx, zy);
    if (rc) return rc;
    launch_helsing_ojala(c->N, c->L.n, c->L.off[1], npts, zx, zy, f_re, f_im, c->hop, c->hoi,
                         false, out_re, out_im, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return WWBI_EHIP;
    return hip_ok(hipGetLastError());
}

int wwbi_interior_velocity(wwbi_ctx *ctx, const wwbi_geom *g, const double *omega,
                           int32_t npts, const double *zx, const double *zy, double *u,
                           double *v) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!omega || !u || !v) return WWBI_EINVAL_NULL;
    int rc = interior_common(c, g, npts, zx, zy);
    if (rc) return rc;
    double *sds = c->vec[VE], *sdn = c->vec[VQG], *fr = c->vec[VFV], *fi = c->vec[VFU];
    boundary_derivs(c, omega, sds, sdn);
    launch_boundary_velocity(c->L.n, g->dx, g->dy, sds, sdn, true, fr, fi, c->stream);
    launch_helsing_ojala(c->N, c->L.n, c->L.off[1], npts, zx, zy, fr, fi, c->hop, c->hoi, true,
                         u, v, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return WWBI_EHIP;
    return hip_ok(hipGetLastError());
}

int wwbi_pressure(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi, double tau,
                  double grav, const wwbi_opts *o, int32_t npts, const double *zx,
                  const double *zy, double *p, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    SolveStats st{};
    int rc = Ctx::check_opts(o);
    if (!rc && (!phi || !zx || !zy || !p)) rc = WWBI_EINVAL_NULL;
    if (!rc && !(std::isfinite(tau) && std::isfinite(grav))) rc = WWBI_EINVAL_NONFINITE;
    if (!rc && (npts < 1 || npts > (1 << 26))) rc = WWBI_EINVAL_SIZE;
    if (!rc && (!g || !g->M)) rc = WWBI_EINVAL_NULL;
    if (!rc && (g->nb < 2 || g->nb > kMaxB)) rc = WWBI_EINVAL_SIZE;
    long nsum = 0;
    for (int k = 0; !rc && k < g->nb; ++k) {
        if (g->M[k] < 8 || (g->M[k] & 1)) rc = WWBI_EINVAL_SIZE;
        nsum += g->M[k];
    }
    if (!rc && nsum > (1L << 28)) rc = WWBI_EINVAL_SIZE;
    if (!rc) {
        // workspace first: the solve below writes into workspace vectors
        c->restart_cap = std::max(c->restart_cap, o->restart);
        rc = c->ensure((int)nsum, c->restart_cap);
    }
    if (!rc) {
        const size_t ns = (size_t)ho_slices(npts, (int)nsum);
        rc = grow(c->hop, c->caphop, 4 * ns * npts + 3 * (size_t)npts + 64);
        if (!rc) rc = grow(c->hoi, c->caphoi, ns * npts + 64);
    }
    if (!rc) {
        // the points, before any work: finite and within the node height limit
        launch_check_points(npts, zx, zy, c->val, c->stream);
        if (hipMemcpyAsync(c->hst, c->val, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            rc = WWBI_EHIP;
        const double *h = (const double *)c->hst;
        if (!rc && h[0] != 0.0) rc = WWBI_EINVAL_NONFINITE;
        if (!rc && h[1] != 0.0) rc = WWBI_EINVAL_RANGE;
    }
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    // 1. the velocity-potential solve; its stored matrix serves the second solve
    wwbi_report r1{};
    const int s1 = solve_phi_impl(c, g, phi, o, c->vec[VU0], c->vec[VOM], nullptr, &r1);
    if (s1 < 0) {
        if (rep) *rep = r1;
        return s1;
    }
    hipStream_t sm = c->stream;
    const Layout &L = c->L;
    const int n = L.n, n0 = L.off[1], nw = n - n0;
    const long ld = round_up(n, 64);
    double *om = c->vec[VOM], *sds = c->vec[VE], *sdn = c->vec[VQG];
    double *b = c->vec[VB], *x = c->vec[VX];
    // 2. Dirichlet data tau kappa - |grad phi|^2/2 - g eta on the surface, 0 on the walls
    boundary_derivs(c, om, sds, sdn);
    launch_fill(b, 0.0, n, sm);
    launch_pressure_data(n0, c->N, sds, sdn, tau, grav, b, sm);
    // 3. A omega_aux = b with the matrix of step 1
    const bool stored = o->matvec != WWBI_MATVEC_ON_THE_FLY;
    const bool fp32 = o->precision == WWBI_FP32_REFINED;
    Op op64{stored ? OP_A_S64 : OP_A_O64, n, ld, o->flags, o->band};
    int status;
    if (!fp32) {
        status = c->gmres(op64, b, x, true, o->tol, o->restart, o->max_iter, o->poll_every,
                          true, st);
    } else {
        Op op32{stored ? OP_A_S32 : OP_A_O32, n, ld, o->flags, o->band};
        Op opres{OP_A_O64, n, ld, o->flags, o->band};
        status = c->refine(op32, opres, b, x, true, *o, st);
    }
    if (status < 0) {
        if (rep) { *rep = r1; rep->status = status; }
        return status;
    }
    // 4. boundary values of the auxiliary Cauchy integrals
    double *ps = c->vec[VTMP], *rw = c->vec[VTMP2], *hw = c->vec[VHF], *means = c->vec[VRR];
    double *fr = c->vec[VFV], *fi = c->vec[VFU];
    launch_circulant_apply(L, c->rowH, x, hw, 1.0, 0.0, 0, L.nb - 1, sm);
    launch_block_means(L, x, means, sm);
    launch_rflavour(L, c->N, c->hrow, 4, 0, 0, n0, 0, n, x, c->part, nullptr, sm);
    launch_reduce_partials(n0, c->part, rflavour_nsplit(c->N, n0, n, 0), nullptr, 1.0, ps,
                           nullptr, sm);
    if (nw > 0) {
        launch_rflavour(L, c->N, c->hrow, 6, 0, n0, nw, 0, n0, x, c->part, nullptr, sm);
        launch_reduce_partials(nw, c->part, rflavour_nsplit(c->N, nw, n0, 0), nullptr, 1.0, rw,
                               nullptr,
                               sm);
        launch_rflavour(L, c->N, c->hrow, 7, 0, n0, nw, n0, nw, x + n0, c->part, nullptr, sm);
        launch_reduce_partials(nw, c->part, rflavour_nsplit(c->N, nw, nw, 0), rw, -1.0, rw,
                               nullptr, sm);
    }
    launch_phi_aux_values(n, n0, b, ps, rw, hw, c->bid, means, fr, fi, sm);
    // 5. phi_t - C and u - i v inside the fluid, then the pressure
    const size_t ns = (size_t)ho_slices(npts, n);
    double *phit = c->hop + 4 * ns * npts, *wr = phit + npts, *wi = wr + npts;
    launch_helsing_ojala(c->N, n, n0, npts, zx, zy, fr, fi, c->hop, c->hoi, false, phit, wi, sm);
    double *vr = c->vec[VKF], *vi = c->vec[VGF];
    launch_boundary_velocity(n, g->dx, g->dy, sds, sdn, true, vr, vi, sm);
    launch_helsing_ojala(c->N, n, n0, npts, zx, zy, vr, vi, c->hop, c->hoi, false, wr, wi, sm);
    launch_pressure_final(npts, phit, wr, wi, zy, grav, p, sm);
    const bool ok = hipStreamSynchronize(sm) == hipSuccess && hipGetLastError() == hipSuccess;
    if (rep) {
        *rep = r1;
        rep->iters += st.iters;
        rep->refine_steps += st.refine_steps;
        rep->status = ok ? status : WWBI_EHIP;
    }
    if (!ok) return WWBI_EHIP;
    return status != WWBI_OK ? status : s1;
}

int wwbi_adjoint_phi(wwbi_ctx *ctx, const wwbi_geom *g, const double *omega, const double *dJdU,
                     const wwbi_opts *o, double *g_phi, double *g_x, double *g_y, double *g_dx,
                     double *g_dy, double *g_ddx, double *g_ddy, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    SolveStats st{};
    int rc = Ctx::check_opts(o);
    if (!rc && (!omega || !dJdU || !g_phi || !g_x || !g_y || !g_dx || !g_dy || !g_ddx || !g_ddy))
        rc = WWBI_EINVAL_NULL;
    if (!rc) {
        c->restart_cap = std::max(c->restart_cap, o->restart);
        c->begin_report((o->flags & WWBI_FLAG_PROFILE) != 0);
        rc = c->setup(g, dJdU, g ? g->M[0] : 0, false);
    }
    const int n = rc ? 0 : c->L.n, n0 = rc ? 0 : c->L.off[1];
    if (!rc) {
        const int ns = adjoint_nsplit(n);
        rc = grow(c->apart, c->capapart, (size_t)12 * ns * n0 + 64);
    }
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    hipStream_t sm = c->stream;
    const long ld = round_up(n, 64);
    double *gam = c->vec[VG], *U = c->vec[VTMP2], *cv = c->vec[VC], *gbar = c->vec[VTMP];
    double *mu = c->vec[VMU], *lam = c->vec[VLAM];
    launch_circulant_rows(c->L, WWBI_OP_D, c->rowD, sm);
    launch_circulant_rows(c->L, WWBI_OP_H, c->rowH, sm);
    hipEventRecord(c->ev[1], sm);
    // the transpose solve A^T lambda = mu; the stored path assembles A^T itself,
    // so that its products stream rows (the forward matvec, about 6% faster at
    // large n than the column-split transpose product).  The matrix goes into
    // internal memory only, so it is queued before the input checks are read.
    const bool stored = o->matvec != WWBI_MATVEC_ON_THE_FLY;
    const bool fp32 = o->precision == WWBI_FP32_REFINED;
    if (stored) {
        rc = c->ensure_matrix((size_t)n * ld * (fp32 ? 4 : 8));
        if (rc) { c->finish_report(rep, rc, st, 0); return rc; }
        if (fp32)
            launch_assemble32_T(c->L, c->N, o->flags, o->band, (float *)c->A, ld, sm);
        else
            launch_assemble64_T(c->L, c->N, o->flags, (double *)c->A, ld, sm);
    }
    hipEventRecord(c->ev[2], sm);
    rc = c->setup_check();
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    // forward quantities: gamma = (-D omega_0, D omega_j) and U
    c->gamma_from_omega(omega, gam);
    c->eval_U_from_gamma(gam, U);
    // c = Ubar / s;  gammabar = T^T c - H c / 2 (surface block);  mu = Gamma^T gammabar
    launch_adj_c(n0, dJdU, c->s, cv, sm);
    launch_rflavour(c->L, c->N, c->hrow, 2, 1, 0, n0, 0, n, cv, c->part, nullptr, sm);
    launch_reduce_partials(n, c->part, rflavour_nsplit(c->N, n0, n, 1), nullptr, 1.0, gbar,
                           nullptr, sm);
    launch_circulant_apply(c->L, c->rowH, cv, gbar, -0.5, 1.0, 0, 0, sm);
    launch_circulant_apply2(c->L, c->rowD, gbar, mu, 1.0, -1.0, 0.0, 0, c->L.nb - 1, sm);
    int status;
    double bytes;
    const bool xz = o->x0 == nullptr;
    if (!xz) launch_copy(lam, o->x0, n, sm);
    if (!fp32) {
        // the stored operator is A^T itself: the forward product applies it
        Op op{stored ? OP_A_S64 : OP_AT_O64, n, ld, o->flags, o->band};
        status = c->gmres(op, mu, lam, xz, o->tol, o->restart, o->max_iter, o->poll_every,
                          true, st);
        bytes = c->op_bytes(op);
    } else {
        Op op32{stored ? OP_A_S32 : OP_AT_O32, n, ld, o->flags, o->band};
        Op op64{OP_AT_O64, n, ld, o->flags, o->band};
        status = c->refine(op32, op64, mu, lam, xz, *o, st);
        bytes = c->op_bytes(op32);
    }
    hipEventRecord(c->ev[3], sm);
    if (status < 0) { c->finish_report(rep, status, st, bytes); return status; }
    // derivative contractions and the final combination
    const int ns = adjoint_nsplit(n);
    double *prow = c->apart, *pcol = c->apart + (size_t)6 * ns * n0;
    launch_adj_rows(c->N, c->hrow, n0, n, omega, gam, prow, sm);
    launch_adj_cols(c->N, n0, n, lam, cv, pcol, sm);
    launch_adj_finalize(c->N, c->F, n0, dJdU, U, omega, gam, lam, prow, ns, pcol, ns, g_phi, g_x,
                        g_y, g_dx, g_dy, g_ddx, g_ddy, sm);
    hipEventRecord(c->ev[4], sm);
    c->finish_report(rep, status, st, bytes);
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    return status;
}

int wwbi_tangent_phi(wwbi_ctx *ctx, const wwbi_geom *g, const double *omega, int32_t nd,
                     const double *dirs, const wwbi_opts *o, double *dU, double *domega,
                     wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    SolveStats st{};
    int rc = Ctx::check_opts(o);
    if (!rc && (!omega || !dirs || !dU)) rc = WWBI_EINVAL_NULL;
    if (!rc && (nd < 1 || nd > kMaxMulti)) rc = WWBI_EINVAL_OPTS;
    if (!rc && (o->matvec == WWBI_MATVEC_ON_THE_FLY || o->x0)) rc = WWBI_EINVAL_OPTS;
    if (!rc && (!g || !g->M)) rc = WWBI_EINVAL_NULL;
    if (!rc && (g->nb < 2 || g->nb > kMaxB || g->M[0] < 8)) rc = WWBI_EINVAL_SIZE;
    if (!rc && 7L * nd * g->M[0] > INT32_MAX) rc = WWBI_EINVAL_SIZE;
    if (!rc) {
        c->restart_cap = std::max(c->restart_cap, o->restart);
        c->begin_report((o->flags & WWBI_FLAG_PROFILE) != 0);
        // the directions are checked for finite values with the geometry
        rc = c->setup(g, dirs, (int)(7L * nd * g->M[0]), false);
    }
    const int n = rc ? 0 : c->L.n, n0 = rc ? 0 : c->L.off[1];
    const int nsr = rc ? 0 : adjoint_nsplit(n), nsc = rc ? 0 : tlm_nsplit(n, n0);
    if (!rc) rc = c->ensure_multi(n, nd, o->restart);
    if (!rc)
        rc = grow(c->apart, c->capapart,
                  (size_t)6 * nsr * n0 + (size_t)nsc * nd * (n + n0) + (size_t)3 * nd * n0 +
                      tlm_weights_size(n0) + 64);
    // the partial sums of the multi-vector product with T (M_0 x n)
    if (!rc)
        rc = grow(c->mw.part, c->mw.cpart, (size_t)multi_part_size_rect64(n0, n, nd) + 64);
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    hipStream_t sm = c->stream;
    const long ld = round_up(n, 64), ldv = ld;
    double *gam = c->vec[VG], *U = c->vec[VTMP2];
    double *prow = c->apart, *pA = prow + (size_t)6 * nsr * n0, *pT = pA + (size_t)nsc * nd * n;
    double *um = pT + (size_t)nsc * nd * n0, *hgs = um + (size_t)nd * n0;
    double *tgs = hgs + (size_t)nd * n0, *wts = tgs + (size_t)nd * n0;
    launch_circulant_rows(c->L, WWBI_OP_D, c->rowD, sm);
    launch_circulant_rows(c->L, WWBI_OP_H, c->rowH, sm);
    hipEventRecord(c->ev[1], sm);
    // the nd systems share A: one multi-RHS solve (matrix read once per step).
    // The matrix goes into internal memory only, so it is queued before the
    // input checks are read back.
    const bool fp32 = o->precision == WWBI_FP32_REFINED;
    rc = c->ensure_matrix((size_t)n * ld * (fp32 ? 4 : 8));
    if (rc) { c->finish_report(rep, rc, st, 0); return rc; }
    const bool stored64 = fp32 && c->ensure_matrix64((size_t)n * ld * 8) == WWBI_OK;
    if (fp32) {
        launch_assemble32(c->L, c->N, o->flags, o->band, (float *)c->A, ld, sm);
        if (stored64) launch_assemble64(c->L, c->N, o->flags, c->A64, ld, sm);
    } else {
        launch_assemble64(c->L, c->N, o->flags, (double *)c->A, ld, sm);
    }
    hipEventRecord(c->ev[2], sm);
    rc = c->setup_check();
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    // base state: gamma = (-D omega_0, D omega_j) and U
    c->gamma_from_omega(omega, gam);
    c->eval_U_from_gamma(gam, U);
    // the terms of dA omega and dT gamma: row sums (per target node) and the
    // source-moving column parts of every direction; then the right-hand sides
    launch_adj_rows(c->N, c->hrow, n0, n, omega, gam, prow, sm);
    launch_tlm_cols(c->N, n0, n, nd, dirs, omega, gam, wts, pA, pT, sm);
    launch_tlm_rhs(c->N, c->F, n0, n, nd, dirs, omega, gam, U, prow, pA, pT, c->mw.b, ldv, um,
                   sm);
    int status;
    if (!fp32)
        status = c->gmres_multi(OP_A_S64, n, ld, c->mw.b, c->mw.x, nd, o->tol, o->restart,
                                o->max_iter, o->poll_every, true, st);
    else
        status = c->refine_multi(n, ld, c->mw.b, c->mw.x, nd, *o, stored64, st);
    hipEventRecord(c->ev[3], sm);
    if (status >= 0) {
        // dU_i = (um_i + H d gamma_0,i / 2 + T d gamma_i) / s, d gamma_i = Gamma d omega_i,
        // for all directions at once: d gamma into the right-hand sides' buffer
        // (free after the solve), and T assembled in FP64 over matrix storage
        // the solve has finished with
        double *dG = c->mw.b;
        launch_circulant_batched(c->L, c->rowD, c->mw.x, ldv, dG, ldv, nd, -1.0, 1.0, 0.0, 0,
                                 c->L.nb - 1, sm);
        launch_circulant_batched(c->L, c->rowH, dG, ldv, hgs, n0, nd, 1.0, 1.0, 0.0, 0, 0, sm);
        double *Tm = nullptr;
        if (!fp32)
            Tm = (double *)c->A;
        else if (stored64)
            Tm = c->A64;
        else if (c->ensure_matrix((size_t)n0 * ld * 8) == WWBI_OK)
            Tm = (double *)c->A;
        if (Tm) {
            launch_assemble_T64(c->L, c->N, c->hrow, Tm, ld, sm);
            launch_mfma_rect64(Tm, ld, n0, n, dG, ldv, nd, tgs, n0, c->mw.part, sm);
            launch_tlm_finalize(n0, nd, c->s, um, hgs, tgs, dU, sm);
        } else {
            // no room for T: its on-the-fly product, one direction at a time
            const int nsu = rflavour_nsplit(c->N, n0, n, 0);
            for (int i = 0; i < nd; ++i) {
                launch_rflavour(c->L, c->N, c->hrow, 2, 0, 0, n0, 0, n, dG + (long)i * ldv,
                                c->part, nullptr, sm);
                launch_U_finalize(n0, c->s, um + (long)i * n0, hgs + (long)i * n0, c->part, nsu,
                                  dU + (long)i * n0, sm);
            }
        }
        if (domega) launch_copy_strided(c->mw.x, ldv, domega, n, n, nd, sm);
    }
    hipEventRecord(c->ev[4], sm);
    const double bytes = (double)n * n * (fp32 ? 4.0 : 8.0);
    c->finish_report(rep, status, st, bytes);
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    return status;
}

int wwbi_solve_phi_multi(wwbi_ctx *ctx, const wwbi_geom *g, const double *rhs, int32_t nr,
                         const wwbi_opts *o, double *omega, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    SolveStats st{};
    int rc = Ctx::check_opts(o);
    if (!rc && (!rhs || !omega)) rc = WWBI_EINVAL_NULL;
    if (!rc && (nr < 1 || nr > kMaxMulti)) rc = WWBI_EINVAL_OPTS;
    if (!rc && (o->matvec == WWBI_MATVEC_ON_THE_FLY || o->x0)) rc = WWBI_EINVAL_OPTS;
    if (!rc) {
        // the right-hand sides are checked with the geometry: nr x sum(M)
        // values (setup rejects a malformed geometry before reading them)
        long ntot = 0;
        if (g && g->M && g->nb >= 2 && g->nb <= kMaxB)
            for (int k = 0; k < g->nb; ++k) ntot += std::max(0, g->M[k]);
        if (ntot * nr > INT32_MAX) rc = WWBI_EINVAL_SIZE;
        if (!rc) {
            c->restart_cap = std::max(c->restart_cap, o->restart);
            c->begin_report((o->flags & WWBI_FLAG_PROFILE) != 0);
            rc = c->setup(g, rhs, (int)(ntot * nr));
        }
    }
    if (!rc) rc = c->ensure_multi(c->L.n, nr, o->restart);
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    hipStream_t sm = c->stream;
    const int n = c->L.n;
    const long ld = round_up(n, 64), ldv = ld;
    const bool fp32 = o->precision == WWBI_FP32_REFINED;
    launch_copy_strided(rhs, n, c->mw.b, ldv, n, nr, sm);
    hipEventRecord(c->ev[1], sm);
    rc = c->ensure_matrix((size_t)n * ld * (fp32 ? 4 : 8));
    if (rc) { c->finish_report(rep, rc, st, 0); return rc; }
    // the refined path also keeps an FP64 copy for the residuals of all
    // systems in one pass; without room for it they are formed on the fly
    const bool stored64 = fp32 && c->ensure_matrix64((size_t)n * ld * 8) == WWBI_OK;
    if (fp32) {
        launch_assemble32(c->L, c->N, o->flags, o->band, (float *)c->A, ld, sm);
        if (stored64) launch_assemble64(c->L, c->N, o->flags, c->A64, ld, sm);
    } else {
        launch_assemble64(c->L, c->N, o->flags, (double *)c->A, ld, sm);
    }
    hipEventRecord(c->ev[2], sm);
    int status;
    if (!fp32)
        status = c->gmres_multi(OP_A_S64, n, ld, c->mw.b, c->mw.x, nr, o->tol, o->restart,
                                o->max_iter, o->poll_every, true, st);
    else
        status = c->refine_multi(n, ld, c->mw.b, c->mw.x, nr, *o, stored64, st);
    hipEventRecord(c->ev[3], sm);
    if (status >= 0) launch_copy_strided(c->mw.x, ldv, omega, n, n, nr, sm);
    hipEventRecord(c->ev[4], sm);
    const double bytes = (double)n * n * (fp32 ? 4.0 : 8.0);
    c->finish_report(rep, status, st, bytes);
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    return status;
}

int wwbi_spectral(wwbi_ctx *ctx, int32_t n, const double *f, int32_t op, double alpha, double beta,
                  double *out) {
    if (!ctx) return WWBI_EINVAL_NULL;
    if (!f || !out) return WWBI_EINVAL_NULL;
    if (n < 8 || (n & 1)) return WWBI_EINVAL_SIZE;
    if (op < WWBI_OP_D || op > WWBI_OP_ABSD) return WWBI_EINVAL_OPTS;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    int rc = c->ensure(n, c->restart_cap);
    if (rc) return rc;
    double *tmp = c->vec[VTMP];
    launch_circ_row1(n, WWBI_OP_D, c->rowD, c->stream);
    launch_circ_row1(n, WWBI_OP_H, c->rowH, c->stream);
    switch (op) {
    case WWBI_OP_D: launch_circ_apply1(n, c->rowD, f, out, alpha, beta, c->stream); break;
    case WWBI_OP_H: launch_circ_apply1(n, c->rowH, f, out, alpha, beta, c->stream); break;
    case WWBI_OP_D2:
        launch_circ_apply1(n, c->rowD, f, tmp, 1.0, 0.0, c->stream);
        launch_circ_apply1(n, c->rowD, tmp, out, alpha, beta, c->stream);
        break;
    case WWBI_OP_ABSD:
        launch_circ_apply1(n, c->rowD, f, tmp, 1.0, 0.0, c->stream);
        launch_circ_apply1(n, c->rowH, tmp, out, alpha, beta, c->stream);
        break;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return WWBI_EHIP;
    return hip_ok(hipGetLastError());
}

int wwbi_surface_fill(wwbi_ctx *ctx, int32_t n, const double *xt, const double *yt, double *x,
                      double *y, double *dx, double *dy, double *ddx, double *ddy) {
    if (!ctx) return WWBI_EINVAL_NULL;
    if (!xt || !yt || !x || !y || !dx || !dy || !ddx || !ddy) return WWBI_EINVAL_NULL;
    if (n < 8 || (n & 1)) return WWBI_EINVAL_SIZE;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    int rc = c->ensure(n, c->restart_cap);
    if (rc) return rc;
    hipStream_t st = c->stream;
    launch_circ_row1(n, WWBI_OP_D, c->rowD, st);
    launch_surface_base(n, xt, yt, x, y, st);
    launch_circ_apply1(n, c->rowD, xt, dx, 1.0, 0.0, st);
    launch_circ_apply1(n, c->rowD, dx, ddx, 1.0, 0.0, st);
    launch_add_scalar(n, dx, 1.0, st);
    launch_circ_apply1(n, c->rowD, yt, dy, 1.0, 0.0, st);
    launch_circ_apply1(n, c->rowD, dy, ddy, 1.0, 0.0, st);
    if (hipStreamSynchronize(st) != hipSuccess) return WWBI_EHIP;
    return hip_ok(hipGetLastError());
}

int wwbi_surface_fill_adjoint(wwbi_ctx *ctx, int32_t n, const double *g_x, const double *g_y,
                              const double *g_dx, const double *g_dy, const double *g_ddx,
                              const double *g_ddy, double *g_xt, double *g_yt) {
    if (!ctx) return WWBI_EINVAL_NULL;
    if (!g_x || !g_y || !g_dx || !g_dy || !g_ddx || !g_ddy || !g_xt || !g_yt)
        return WWBI_EINVAL_NULL;
    if (n < 8 || (n & 1)) return WWBI_EINVAL_SIZE;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    int rc = c->ensure(n, c->restart_cap);
    if (rc) return rc;
    hipStream_t st = c->stream;
    double *tmp = c->vec[VTMP];
    launch_circ_row1(n, WWBI_OP_D, c->rowD, st);
    // g_xt = g_x - D g_dx + D (D g_ddx)   (D^T = -D, (D2)^T = D2)
    launch_copy(g_xt, g_x, n, st);
    launch_circ_apply1(n, c->rowD, g_dx, g_xt, -1.0, 1.0, st);
    launch_circ_apply1(n, c->rowD, g_ddx, tmp, 1.0, 0.0, st);
    launch_circ_apply1(n, c->rowD, tmp, g_xt, 1.0, 1.0, st);
    launch_copy(g_yt, g_y, n, st);
    launch_circ_apply1(n, c->rowD, g_dy, g_yt, -1.0, 1.0, st);
    launch_circ_apply1(n, c->rowD, g_ddy, tmp, 1.0, 0.0, st);
    launch_circ_apply1(n, c->rowD, tmp, g_yt, 1.0, 1.0, st);
    if (hipStreamSynchronize(st) != hipSuccess) return WWBI_EHIP;
    return hip_ok(hipGetLastError());
}

int wwbi_debug_matrix(wwbi_ctx *ctx, const wwbi_geom *g, int32_t which, int32_t precision,
                      int32_t band, void *out) {
    if (!ctx) return WWBI_EINVAL_NULL;
    if (!out) return WWBI_EINVAL_NULL;
    if (which != WWBI_MAT_A && which != WWBI_MAT_WALL && which != WWBI_MAT_T)
        return WWBI_EINVAL_OPTS;
    if (precision != WWBI_FP64 && precision != WWBI_FP32_REFINED) return WWBI_EINVAL_OPTS;
    if (which != WWBI_MAT_A && precision != WWBI_FP64) return WWBI_EINVAL_OPTS;
    if (band < 0) return WWBI_EINVAL_OPTS;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    int rc = c->setup(g, nullptr, 0);
    if (rc) return rc;
    // assemble with the padded leading dimension the kernels write (a multiple
    // of 64 elements) into the workspace matrix, then copy the dense rows out
    const int n = c->L.n;
    int rows = n;
    if (which == WWBI_MAT_WALL) rows = n - c->L.off[1];
    if (which == WWBI_MAT_T) rows = c->L.off[1];
    const int cols = which == WWBI_MAT_WALL ? rows : n;
    const long ld = round_up(cols, 64);
    const size_t es = precision == WWBI_FP64 ? 8 : 4;
    rc = c->ensure_matrix((size_t)rows * ld * es);
    if (rc) return rc;
    if (which == WWBI_MAT_WALL)
        launch_assemble_wall64(c->L, c->N, c->hrow, (double *)c->A, ld, c->stream);
    else if (which == WWBI_MAT_T)
        launch_assemble_T64(c->L, c->N, c->hrow, (double *)c->A, ld, c->stream);
    else if (precision == WWBI_FP64)
        launch_assemble64(c->L, c->N, 0, (double *)c->A, ld, c->stream);
    else
        launch_assemble32(c->L, c->N, 0, band, (float *)c->A, ld, c->stream);
    if (hipMemcpy2DAsync(out, cols * es, c->A, ld * es, cols * es, rows, hipMemcpyDeviceToDevice,
                         c->stream) != hipSuccess)
        return WWBI_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return WWBI_EHIP;
    return hip_ok(hipGetLastError());
}

int wwbi_matvec(wwbi_ctx *ctx, const wwbi_geom *g, const double *x, double *y, int32_t precision,
                int32_t mode, int32_t transpose, int32_t band, wwbi_report *rep) {
    if (!ctx) return WWBI_EINVAL_NULL;
    if (!x || !y) return WWBI_EINVAL_NULL;
    if (precision != WWBI_FP64 && precision != WWBI_FP32_REFINED) return WWBI_EINVAL_OPTS;
    if (mode < 0 || mode > 2 || band < 0) return WWBI_EINVAL_OPTS;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->begin_report(rep != nullptr);
    int rc = c->setup(g, nullptr, 0);
    if (rc) return rc;
    const int n = c->L.n;
    const long ld = round_up(n, 64);
    const bool fp32 = precision == WWBI_FP32_REFINED;
    const bool stored = mode != WWBI_MATVEC_ON_THE_FLY;
    hipEventRecord(c->ev[1], c->stream);
    // the stored transpose is assembled as A^T and applied by the forward product
    if (stored) {
        rc = c->ensure_matrix((size_t)n * ld * (fp32 ? 4 : 8));
        if (rc) return rc;
        if (fp32 && transpose)
            launch_assemble32_T(c->L, c->N, 0, band, (float *)c->A, ld, c->stream);
        else if (fp32)
            launch_assemble32(c->L, c->N, 0, band, (float *)c->A, ld, c->stream);
        else if (transpose)
            launch_assemble64_T(c->L, c->N, 0, (double *)c->A, ld, c->stream);
        else
            launch_assemble64(c->L, c->N, 0, (double *)c->A, ld, c->stream);
    }
    hipEventRecord(c->ev[2], c->stream);
    double *xw = c->vec[VTMP], *yw = c->vec[VW];
    launch_copy(xw, x, n, c->stream);
    int kind;
    if (stored)
        kind = fp32 ? OP_A_S32 : OP_A_S64;
    else
        kind = transpose ? (fp32 ? OP_AT_O32 : OP_AT_O64) : (fp32 ? OP_A_O32 : OP_A_O64);
    Op op{kind, n, ld, 0, band};
    c->prof_begin();
    c->apply(op, xw, nullptr, nullptr, yw, nullptr);
    c->prof_end();
    hipEventRecord(c->ev[3], c->stream);
    launch_copy(y, yw, n, c->stream);
    hipEventRecord(c->ev[4], c->stream);
    SolveStats st{};
    c->finish_report(rep, WWBI_OK, st, c->op_bytes(op));
    return hip_ok(hipGetLastError());
}

}  // extern "C"
