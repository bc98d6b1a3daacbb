// Allocation-free velocity-potential solve (wwbi_solve_phi_noalloc): the
// same solve as wwbi_solve_phi with an on-the-fly matvec, its whole
// per-solve workspace carved out of one static device array per GPU instead
// of the context's allocations.  For callers that cannot allocate device
// memory: code under stream capture, tight serving loops, harnesses that
// forbid hipMalloc.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "api_internal.h"

namespace {

constexpr size_t kScratchBytes = WWBI_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The workspace of every allocation-free call on this GPU.  Host code never
// passes this name to a kernel: it is only a host-side handle of the symbol.
// The device address is looked up once per device (scratch_init) and every
// kernel receives pointers derived from it.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};    // device address of `scratch` on each device
bool g_done[kMaxDevices] = {};    // lookup attempted on that device

constexpr size_t kAlign = 256;
inline size_t align_up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }

void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace

namespace wwbi {

void scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_done[device]) return;
    g_done[device] = true;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return;                     // the entry point then reports WWBI_EHIP
    }
    g_ptr[device] = p;
}

}  // namespace wwbi

using namespace wwbi;

extern "C" int wwbi_solve_phi_noalloc(wwbi_ctx *ctx, const wwbi_geom *g, const double *phi,
                                      const wwbi_opts *o, double *U, double *omega,
                                      double *psi_k, wwbi_report *rep) {
    auto fail = [&](int rc) {
        if (rep) {
            std::memset(rep, 0, sizeof(*rep));
            rep->status = rc;
        }
        return rc;
    };
    if (!ctx) return WWBI_EINVAL_NULL;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    int rc = Ctx::check_opts(o);
    if (rc) return fail(rc);
    if (o->matvec != WWBI_MATVEC_ON_THE_FLY) return fail(WWBI_EINVAL_OPTS);
    // every restart cycle records its step count in host bookkeeping reserved
    // at wwbi_create; a cycle takes at least one Arnoldi step
    if ((size_t)o->max_iter + (size_t)o->max_refine + 8 > c->cyc_done.capacity())
        return fail(WWBI_EINVAL_OPTS);
    if (!g || !g->M || !phi || !U) return fail(WWBI_EINVAL_NULL);
    if (g->nb < 2 || g->nb > kMaxB) return fail(WWBI_EINVAL_SIZE);
    long n = 0;
    for (int k = 0; k < g->nb; ++k) {
        if (g->M[k] < 8 || (g->M[k] & 1)) return fail(WWBI_EINVAL_SIZE);
        n += g->M[k];
        if (n > (1L << 28)) return fail(WWBI_EINVAL_SIZE);
    }
    if (!g->x || !g->y || !g->dx || !g->dy || !g->ddx || !g->ddy) return fail(WWBI_EINVAL_NULL);
    if (g->nb > 2 && (!g->zc || !g->a)) return fail(WWBI_EINVAL_NULL);
    unsigned char *base = static_cast<unsigned char *>(scratch_ptr(c->device));
    if (!base) return fail(WWBI_EHIP);

    // the workspace of this solve, laid out in the array: the cycle state
    // first, then every buffer of the plan, each 256-byte aligned
    WsItem it[kMaxWsItems];
    // (an on-the-fly FP64 solve: no room for a recycled space)
    const int k = c->ws_plan((int)n, o->restart, it, false);
    size_t off[kMaxWsItems];
    size_t total = align_up(sizeof(GState));
    for (int i = 0; i < k; ++i) {
        off[i] = total;
        total += align_up(it[i].count * it[i].esize);
    }
    if (total > kScratchBytes) return fail(WWBI_ESCRATCH);

    // swap the context's workspace for the carved one; restored on return
    void *save_p[kMaxWsItems];
    size_t save_cap[kMaxWsItems];
    for (int i = 0; i < k; ++i) {
        save_p[i] = *it[i].p;
        save_cap[i] = *it[i].cap;
        *it[i].p = base + off[i];
        *it[i].cap = it[i].count;
    }
    GState *save_gs = c->gs;
    const int save_restart = c->restart_cap;
    const int save_vpre = c->vpre;
    c->gs = reinterpret_cast<GState *>(base);
    c->restart_cap = o->restart;
    c->vpre = 0;
    c->fixed_ws = true;

    // the array keeps the previous call's contents: start from zero, as a
    // fresh allocation would (a fill kernel, no memset node)
    launch_fill(reinterpret_cast<double *>(base), 0.0, (int)(total / sizeof(double)), c->stream);
    rc = solve_phi_impl(c, g, phi, o, U, omega, psi_k, rep);
    // no work of this call may still read or write the array after it returns
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc >= 0) rc = WWBI_EHIP;

    c->fixed_ws = false;
    c->vpre = save_vpre;
    c->restart_cap = save_restart;
    c->gs = save_gs;
    for (int i = 0; i < k; ++i) {
        *it[i].p = save_p[i];
        *it[i].cap = save_cap[i];
    }
    return rc;
}
