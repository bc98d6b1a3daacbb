// Host side of libwwbi: context and workspace, input validation, the GMRES
// and iterative-refinement drivers, and the C entry points of wwbi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
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

int Ctx::ensure(int n, int restart) {
    trace = std::getenv("WWBI_TRACE") != nullptr;
    const size_t nn = (size_t)round_up(n, 64);
    const size_t rr = (size_t)std::max(restart, 8);
    int rc = WWBI_OK;
    auto G = [&](double *&p, size_t &c, size_t w) { if (rc == WWBI_OK) rc = grow(p, c, w); };
    auto Gi = [&](int *&p, size_t &c, size_t w) { if (rc == WWBI_OK) rc = grow(p, c, w); };
    auto Gf = [&](float *&p, size_t &c, size_t w) { if (rc == WWBI_OK) rc = grow(p, c, w); };
    G(V, capV, (rr + 1) * nn);
    Gf(v32, capv32, nn);
    for (int i = 0; i < kNumVec; ++i) G(vec[i], capvec[i], nn);
    G(H, capH, (rr + 1) * (rr + 1));
    G(cs, capcs, rr + 1);
    G(sn, capsn, rr + 1);
    G(gv, capg, rr + 1);
    G(yv, capy, rr + 1);
    G(P, capP, 3 * 64 * (rr + 1) + 64);
    G(part, cappart, 64 * nn + 64);
    Gi(bid, capbid, nn);
    Gi(loc, caploc, nn);
    Gi(Mk, capMk, nn);
    G(wq, capwq, nn);
    G(s, caps, nn);
    G(lre, caplre, nn);
    G(lim, caplim, nn);
    G(rowD, caprowD, nn);
    G(rowH, caprowH, nn);
    G(hrow, caphrow, nn);
    G(eR, capeR, nn);
    G(eI, capeI, nn);
    G(val, capval, 3 * kMaxB + 8);
    return rc;
}

int Ctx::ensure_matrix(size_t bytes) {
    if (bytes <= capA && A) return WWBI_OK;
    if (A) hipFree(A);
    A = nullptr;
    capA = 0;
    if (hipMalloc(&A, bytes) != hipSuccess) {
        A = nullptr;
        (void)hipGetLastError();
        return WWBI_ECAPACITY;
    }
    capA = bytes;
    return WWBI_OK;
}

void Ctx::release() {
    auto F = [](auto *&p) { if (p) hipFree((void *)p); p = nullptr; };
    F(A);
    F(V);
    F(v32);
    for (int i = 0; i < kNumVec; ++i) F(vec[i]);
    F(H); F(cs); F(sn); F(gv); F(yv); F(P); F(part);
    F(bid); F(loc); F(Mk); F(wq); F(s); F(lre); F(lim); F(rowD); F(rowH); F(val); F(apart);
    F(hrow); F(eR); F(eI);
    if (gs) hipFree(gs);
    gs = nullptr;
    if (hst) hipHostFree(hst);
    hst = nullptr;
    for (auto &e : ev) if (e) hipEventDestroy(e);
    for (auto &e : prof) if (e) hipEventDestroy(e);
    for (auto &e : pollev) if (e) hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// geometry set-up and validation
// ---------------------------------------------------------------------------

int Ctx::setup(const wwbi_geom *g, const double *phi, int nphi) {
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
    N.ex = eR; N.ey = eI;
    N.n = L.n;
    psi_wall = g->psi_wall;
    launch_prep_nodes(L, g->x, g->y, g->dx, g->dy, g->ddx, g->ddy, bid, loc, Mk, wq, s, lre, lim,
                      eR, eI, stream);
    launch_circ_row1(L.off[1], kOpHalfCot, hrow, stream);
    launch_validate(L, N, phi, phi ? nphi : 0, val, stream);
    if (hipMemcpyAsync(hst, val, sizeof(double) * (3 * L.nb + 1), hipMemcpyDeviceToHost,
                       stream) != hipSuccess)
        return WWBI_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return WWBI_EHIP;
    const double *h = (const double *)hst;
    for (int k = 0; k < L.nb; ++k)
        if (h[3 * k] != 0.0) return WWBI_EINVAL_NONFINITE;
    if (h[3 * L.nb] != 0.0) return WWBI_EINVAL_NONFINITE;
    for (int k = 0; k < L.nb; ++k) {
        if (k <= 1 && !(h[3 * k + 2] > 0.0)) return WWBI_EINVAL_ORIENTATION;
        if (k >= 2 && !(h[3 * k + 1] < 0.0)) return WWBI_EINVAL_ORIENTATION;
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
        if (x32)
            launch_gemv32((const float *)A, ld, op.n, x32, c, y, active, stream);
        else
            launch_gemv32_x64((const float *)A, ld, op.n, x, c, y, active, stream);
        break;
    case OP_A_O64:
        launch_otf_matvec(L, N, op.flags, 0, op.band, 0, x, c, y, part, active, stream);
        break;
    case OP_A_O32:
        launch_otf_matvec(L, N, op.flags, 1, op.band, 0, x, c, y, part, active, stream);
        break;
    case OP_AT_S64:
        launch_gemvT64((const double *)A, ld, op.n, x, c, y, part, active, stream);
        break;
    case OP_AT_S32:
        launch_gemvT32((const float *)A, ld, op.n, x, c, y, part, active, stream);
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
        launch_reduce_partials(nw, part, rflavour_nsplit(nw), c, 1.0, y, active, stream);
        break;
    }
    }
}

double Ctx::op_bytes(const Op &op) const {
    const double n = op.n;
    switch (op.kind) {
    case OP_A_S64: case OP_AT_S64: case OP_W_S64: return n * n * 8.0 + 2.0 * n * 8.0;
    case OP_A_S32: case OP_AT_S32: return n * n * 4.0 + n * 4.0 + n * 8.0;
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

void Ctx::prof_begin() {
    if (profiling && nprof < kProfPairs) hipEventRecord(prof[2 * nprof], stream);
}
void Ctx::prof_end() {
    if (profiling && nprof < kProfPairs) {
        hipEventRecord(prof[2 * nprof + 1], stream);
        ++nprof;
    }
}

// Restarted GMRES on op: x <- solution of op x = b.  x must hold the initial
// guess unless x_zero.  With verify, every cycle starts from the true residual
// b - op x and convergence is declared only on it; without verify a single
// cycle runs and its residual estimate is returned (inner solves of the
// iterative refinement, whose outer loop checks the FP64 residual itself).
//
// The host enqueues `poll` Arnoldi steps at a time.  After each batch it
// queues an asynchronous copy of the cycle flag, enqueues the next batch and
// only then waits for the previous copy, so the device never idles on the
// host; steps enqueued after convergence return at once on the device flag.
int Ctx::gmres(const Op &op, const double *b, double *x, bool x_zero, double tol, int restart,
               int max_iter, int poll, bool fp32_basis, bool verify, SolveStats &st) {
    const int n = op.n;
    const int G = gmres_nblocks(n);
    const int ldp = restart + 1;
    const long ldv = round_up(n, 64);
    double *r = vec[VR], *w = vec[VW];
    double *P1 = P, *P2 = P + 64 * ldp, *P3 = P + 2 * 64 * ldp;   // P[i*G + b] layout
    float *x32 = fp32_basis ? v32 : nullptr;
    if (x_zero) launch_fill(x, 0.0, n, stream);
    launch_norm_partial(b, n, P3, G, stream);
    launch_set_tol(P3, G, tol, gs, stream);
    bool first = true;
    double prev_beta = HUGE_VAL;
    int status = WWBI_NOT_CONVERGED;
    GState h{};
    GState *slot = reinterpret_cast<GState *>((char *)hst + kStateSlotOffset);
    for (;;) {
        if (first && x_zero)
            launch_copy(r, b, n, stream);
        else
            apply(op, x, nullptr, b, r, nullptr);
        launch_norm_partial(r, n, P3, G, stream);
        launch_cycle_start(r, n, P3, G, V, x32, gv, restart + 1, gs, stream);
        int rc = read_state(h);
        if (rc) return rc;
        st.rel_resid = h.bnorm > 0 ? h.beta / h.bnorm : 0.0;
        if (trace)
            std::fprintf(stderr, "wwbi: op %d n %d cycle %d its %d beta/bnorm %.3e\n", op.kind, n,
                         st.cycles, st.iters, st.rel_resid);
        if (!h.active) { status = WWBI_OK; break; }
        if (!std::isfinite(h.beta)) { status = WWBI_STAGNATED; break; }
        if (st.iters >= max_iter) { status = WWBI_NOT_CONVERGED; break; }
        if (!first && h.beta > 0.99 * prev_beta) { status = WWBI_STAGNATED; break; }
        prev_beta = h.beta;
        const int jmax = std::min(restart, max_iter - st.iters);
        int pending = -1;          // slot of the flag copy not yet waited for
        bool ended = false;
        for (int j0 = 0; j0 < jmax && !ended; j0 += poll) {
            const int j1 = std::min(jmax, j0 + poll);
            for (int j = j0; j < j1; ++j) {
                const double *vj = V + (long)j * ldv;
                prof_begin();
                apply(op, vj, x32, nullptr, w, &gs->active);
                prof_end();
                launch_cgs_dot(V, ldv, w, n, j, P1, ldp, G, gs, stream);
                launch_cgs_update(V, ldv, w, n, j, P1, P2, ldp, G, H, restart + 1, 0, gs, stream);
                launch_cgs_update(V, ldv, w, n, j, P2, P3, ldp, G, H, restart + 1, 1, gs, stream);
                launch_givens_scale(w, n, j, P3, G, V, ldv, x32, H, restart + 1, cs, sn, gv, jmax,
                                    gs, stream);
            }
            const int cur = (j0 / poll) & 1;
            if (hipMemcpyAsync(slot + cur, gs, sizeof(GState), hipMemcpyDeviceToHost, stream) !=
                hipSuccess)
                return WWBI_EHIP;
            if (hipEventRecord(pollev[cur], stream) != hipSuccess) return WWBI_EHIP;
            if (pending >= 0) {
                if (hipEventSynchronize(pollev[pending]) != hipSuccess) return WWBI_EHIP;
                if (!slot[pending].active) ended = true;
            }
            pending = cur;
        }
        if (hipEventSynchronize(pollev[pending]) != hipSuccess) return WWBI_EHIP;
        launch_hsolve(H, restart + 1, gv, yv, gs, stream);
        launch_xupdate(x, V, ldv, n, yv, gs, stream);
        rc = read_state(h);
        if (rc) return rc;
        st.iters += h.jdone;
        st.cycles += 1;
        first = false;
        if (!verify) {
            st.rel_resid = h.bnorm > 0 ? h.resid / h.bnorm : 0.0;
            status = h.resid <= h.tol_abs ? WWBI_OK : WWBI_NOT_CONVERGED;
            break;
        }
    }
    return status;
}

double Ctx::device_norm(const double *v, int n) {
    const int G = gmres_nblocks(n);
    double *P3 = P + 2 * 64 * (restart_cap + 1);
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
//   solve A32 d = r by GMRES to inner_tol; x += d.
int Ctx::refine(const Op &op32, const Op &op64, const double *b, double *x, bool x_zero,
                const wwbi_opts &o, SolveStats &st) {
    const int n = op64.n;
    double *r = vec[VRR], *d = vec[VD];
    if (x_zero) launch_fill(x, 0.0, n, stream);   // the inner GMRES zeroes d itself
    const double bn = device_norm(b, n);
    if (!std::isfinite(bn)) return WWBI_EHIP;
    double prev = HUGE_VAL;
    int status = WWBI_NOT_CONVERGED;
    for (int k = 0;; ++k) {
        double rn;
        if (k == 0 && x_zero) {
            launch_copy(r, b, n, stream);    // r = b - A 0
            rn = bn;
        } else {
            apply(op64, x, nullptr, b, r, nullptr);
            rn = device_norm(r, n);
        }
        st.rel_resid = bn > 0 ? rn / bn : 0.0;
        if (rn <= o.tol * bn) { status = WWBI_OK; break; }
        if (!std::isfinite(rn) || (k > 0 && rn > 0.5 * prev)) { status = WWBI_REFINE_STALLED; break; }
        if (k >= o.max_refine || st.iters >= o.max_iter) { status = WWBI_NOT_CONVERGED; break; }
        prev = rn;
        SolveStats in{};
        in.iters = st.iters;
        const int rc = gmres(op32, r, d, true, o.inner_tol, o.restart, o.max_iter, o.poll_every,
                             op32.kind == OP_A_S32, false, in);
        if (rc < 0) return rc;
        st.iters = in.iters;
        st.cycles += in.cycles;
        st.refine_steps += 1;
        launch_axpy(x, d, n, 1.0, stream);
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
    launch_U_finalize(n0, s, um, hg, part, rflavour_nsplit(L.n), U, stream);
}

void Ctx::gamma_from_omega(const double *omega, double *gamma) {
    launch_circulant_apply(L, rowD, omega, gamma, -1.0, 0.0, 0, 0, stream);
    launch_circulant_apply(L, rowD, omega, gamma, 1.0, 0.0, 1, L.nb - 1, stream);
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
    rep->n_matvec = nprof;
    double t = 0.0;
    for (int i = 0; i < nprof; ++i) t += ev_ms(prof[2 * i], prof[2 * i + 1]);
    rep->ms_matvec = t;
    rep->bytes_matvec = bytes;
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
    o->inner_tol = 3e-7;
    o->restart = 100;
    o->max_iter = 2000;
    o->precision = WWBI_FP64;
    o->matvec = WWBI_MATVEC_AUTO;
    o->poll_every = 4;
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
    case WWBI_NOT_CONVERGED: return "not converged";
    case WWBI_STAGNATED: return "stagnated";
    case WWBI_REFINE_STALLED: return "iterative refinement stalled";
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
    int rc = WWBI_OK;
    if (hipMalloc((void **)&c->gs, sizeof(GState)) != hipSuccess) rc = WWBI_ECAPACITY;
    if (!rc && hipHostMalloc(&c->hst, 4096) != hipSuccess) rc = WWBI_ECAPACITY;
    for (auto &e : c->ev)
        if (!rc && hipEventCreate(&e) != hipSuccess) rc = WWBI_EHIP;
    for (auto &e : c->prof)
        if (!rc && hipEventCreate(&e) != hipSuccess) rc = WWBI_EHIP;
    for (auto &e : c->pollev)
        if (!rc && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = WWBI_EHIP;
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

static int solve_phi_impl(Ctx *c, const wwbi_geom *g, const double *phi, const wwbi_opts *o,
                          double *U, double *omega, double *psi_k, wwbi_report *rep) {
    SolveStats st{};
    int rc = Ctx::check_opts(o);
    if (!rc && (!phi || !U)) rc = WWBI_EINVAL_NULL;
    if (!rc) {
        c->restart_cap = std::max(c->restart_cap, o->restart);
        c->begin_report((o->flags & WWBI_FLAG_PROFILE) != 0);
        rc = c->setup(g, phi, g ? g->M[0] : 0);
    }
    if (rc) {
        if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->status = rc; }
        return rc;
    }
    const int n = c->L.n;
    const long ld = round_up(n, 64);
    double *b = c->vec[VB], *x = c->vec[VX];
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
    const bool xz = o->x0 == nullptr;
    if (!xz) launch_copy(x, o->x0, n, c->stream);
    Op op64{stored ? OP_A_S64 : OP_A_O64, n, ld, o->flags, o->band};
    int status;
    double bytes;
    if (!fp32) {
        status = c->gmres(op64, b, x, xz, o->tol, o->restart, o->max_iter, o->poll_every, false,
                          true, st);
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
    hipEventRecord(c->ev[4], c->stream);
    c->finish_report(rep, status, st, bytes);
    if (psi_k && c->L.nb > 2) std::memcpy(psi_k, c->hst, sizeof(double) * (c->L.nb - 2));
    if (hipGetLastError() != hipSuccess) return WWBI_EHIP;
    return status;
}

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
    if (!rc && o->precision != WWBI_FP64) rc = WWBI_EINVAL_OPTS;
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
    launch_wall_rhs_finalize(nw, um, c->part, rflavour_nsplit(n0), rhs, c->stream);
    hipEventRecord(c->ev[1], c->stream);
    const bool stored = o->matvec != WWBI_MATVEC_ON_THE_FLY;
    if (stored) {
        rc = c->ensure_matrix((size_t)nw * ldw * 8);
        if (rc) { c->finish_report(rep, rc, st, 0); return rc; }
        launch_assemble_wall64(c->L, c->N, c->hrow, (double *)c->A, ldw, c->stream);
    }
    hipEventRecord(c->ev[2], c->stream);
    double *gw = gam + n0;
    const bool xz = o->x0 == nullptr;
    if (!xz) launch_copy(gw, o->x0, nw, c->stream);
    Op op{stored ? OP_W_S64 : OP_W_O64, nw, ldw, o->flags, o->band};
    const int status =
        c->gmres(op, rhs, gw, xz, o->tol, o->restart, o->max_iter, o->poll_every, false, true, st);
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
        rc = c->setup(g, dJdU, g ? g->M[0] : 0);
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
    // forward quantities: gamma = (-D omega_0, D omega_j) and U
    c->gamma_from_omega(omega, gam);
    c->eval_U_from_gamma(gam, U);
    // c = Ubar / s;  gammabar = T^T c - H c / 2 (surface block);  mu = Gamma^T gammabar
    launch_adj_c(n0, dJdU, c->s, cv, sm);
    launch_rflavour(c->L, c->N, c->hrow, 2, 1, 0, n0, 0, n, cv, c->part, nullptr, sm);
    launch_reduce_partials(n, c->part, rflavour_nsplit(n0), nullptr, 1.0, gbar, nullptr, sm);
    launch_circulant_apply(c->L, c->rowH, cv, gbar, -0.5, 1.0, 0, 0, sm);
    launch_circulant_apply(c->L, c->rowD, gbar, mu, 1.0, 0.0, 0, 0, sm);
    launch_circulant_apply(c->L, c->rowD, gbar, mu, -1.0, 0.0, 1, c->L.nb - 1, sm);
    hipEventRecord(c->ev[1], sm);
    // transpose solve A^T lambda = mu
    const bool stored = o->matvec != WWBI_MATVEC_ON_THE_FLY;
    const bool fp32 = o->precision == WWBI_FP32_REFINED;
    if (stored) {
        rc = c->ensure_matrix((size_t)n * ld * (fp32 ? 4 : 8));
        if (rc) { c->finish_report(rep, rc, st, 0); return rc; }
        if (fp32)
            launch_assemble32(c->L, c->N, o->flags, o->band, (float *)c->A, ld, sm);
        else
            launch_assemble64(c->L, c->N, o->flags, (double *)c->A, ld, sm);
    }
    hipEventRecord(c->ev[2], sm);
    int status;
    double bytes;
    const bool xz = o->x0 == nullptr;
    if (!xz) launch_copy(lam, o->x0, n, sm);
    if (!fp32) {
        Op op{stored ? OP_AT_S64 : OP_AT_O64, n, ld, o->flags, o->band};
        status = c->gmres(op, mu, lam, xz, o->tol, o->restart, o->max_iter, o->poll_every, false,
                          true, st);
        bytes = c->op_bytes(op);
    } else {
        Op op32{stored ? OP_AT_S32 : OP_AT_O32, n, ld, o->flags, o->band};
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
    if (which != WWBI_MAT_A && which != WWBI_MAT_WALL) return WWBI_EINVAL_OPTS;
    if (precision != WWBI_FP64 && precision != WWBI_FP32_REFINED) return WWBI_EINVAL_OPTS;
    if (which == WWBI_MAT_WALL && precision != WWBI_FP64) return WWBI_EINVAL_OPTS;
    if (band < 0) return WWBI_EINVAL_OPTS;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    int rc = c->setup(g, nullptr, 0);
    if (rc) return rc;
    const int n = c->L.n;
    if (which == WWBI_MAT_WALL) {
        const int nw = n - c->L.off[1];
        launch_assemble_wall64(c->L, c->N, c->hrow, (double *)out, nw, c->stream);
    } else if (precision == WWBI_FP64) {
        launch_assemble64(c->L, c->N, 0, (double *)out, n, c->stream);
    } else {
        launch_assemble32(c->L, c->N, 0, band, (float *)out, n, c->stream);
    }
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
    if (stored) {
        rc = c->ensure_matrix((size_t)n * ld * (fp32 ? 4 : 8));
        if (rc) return rc;
        if (fp32)
            launch_assemble32(c->L, c->N, 0, band, (float *)c->A, ld, c->stream);
        else
            launch_assemble64(c->L, c->N, 0, (double *)c->A, ld, c->stream);
    }
    hipEventRecord(c->ev[2], c->stream);
    double *xw = c->vec[VTMP], *yw = c->vec[VW];
    launch_copy(xw, x, n, c->stream);
    int kind;
    if (stored)
        kind = transpose ? (fp32 ? OP_AT_S32 : OP_AT_S64) : (fp32 ? OP_A_S32 : OP_A_S64);
    else
        kind = transpose ? (fp32 ? OP_AT_O32 : OP_AT_O64) : (fp32 ? OP_A_O32 : OP_A_O64);
    Op op{kind, n, ld, 0, band};
    float *x32 = nullptr;
    if (kind == OP_A_S32) {
        x32 = c->v32;
        launch_to_f32(xw, x32, n, c->stream);
    }
    c->prof_begin();
    c->apply(op, xw, x32, nullptr, yw, nullptr);
    c->prof_end();
    hipEventRecord(c->ev[3], c->stream);
    launch_copy(y, yw, n, c->stream);
    hipEventRecord(c->ev[4], c->stream);
    SolveStats st{};
    c->finish_report(rep, WWBI_OK, st, c->op_bytes(op));
    return hip_ok(hipGetLastError());
}

}  // extern "C"
