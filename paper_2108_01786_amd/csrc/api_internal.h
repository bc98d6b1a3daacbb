// Host context of libwwbi (shared by the translation units of the host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "internal.h"

namespace wwbi {

inline long round_up(long a, long b) { return (a + b - 1) / b * b; }

// Linear operators GMRES can run on.
enum OpKind {
    OP_A_S64 = 0,   // velocity-potential A, stored FP64
    OP_A_S32,       // stored FP32 (FP32 accumulation)
    OP_A_O64,       // on the fly FP64
    OP_A_O32,       // on the fly FP32 (FP64 band and limits)
    OP_AT_O64,      // transposes on the fly (a stored transpose is assembled as
    OP_AT_O32,      // A^T and applied with OP_A_S64 / OP_A_S32)
    OP_W_S64,       // vortex-sheet wall operator, stored FP64
    OP_W_O64,       // on the fly FP64
    OP_GT_S64,      // gamma_t operator (Sec. 4.2), stored FP64
    OP_GT_O64,      // on the fly FP64
    OP_GT_S32,      // stored FP32 (FP32 accumulation), inside FP64 refinement
    OP_W_S32,       // wall operator, stored FP32, inside FP64 refinement
};

// stored FP64 operators
inline bool stored_fp64(int kind) {
    return kind == OP_A_S64 || kind == OP_GT_S64 || kind == OP_W_S64;
}

// stored FP32 operators, whose products can read the FP32 copy of a basis vector
inline bool stored_fp32(int kind) {
    return kind == OP_A_S32 || kind == OP_GT_S32 || kind == OP_W_S32;
}

struct Op {
    int kind;
    int n;          // operator size
    long ld;        // leading dimension of the stored matrix
    int flags;
    int band;
};

struct SolveStats {
    int iters = 0;
    int cycles = 0;
    int refine_steps = 0;
    double rel_resid = 0.0;
};

// workspace vectors (each round_up(n, 64) doubles)
enum VecId { VR = 0, VW, VB, VX, VRR, VD, VG, VHG, VUM, VTMP, VTMP2, VLAM, VMU, VC,
             VOM, VU0, VFV, VFU, VKF, VGF, VHF, VQG, VTM, VE, kNumVec };

constexpr int kProfPairs = 2048;
constexpr int kStateSlotOffset = 8192;   // byte offset of the two polled GState slots in hst
constexpr int kStateSlotBytes = 8192;    // bytes per slot (up to kMaxMulti states)
constexpr int kTailOffset = 24576;       // byte offset of the Fourier-tail energies in hst
constexpr int kHostStaging = 32768;      // pinned host staging bytes
constexpr int kMaxMulti = 32;            // right-hand sides per multi solve

double inner_tolerance(const wwbi_opts &o, double bnorm, double rnorm);

// One buffer of the per-solve workspace: the context's pointer and capacity
// (elements) and the element count and size a solve needs.
struct WsItem {
    void **p;
    size_t *cap;
    size_t count;
    size_t esize;
};
constexpr int kMaxWsItems = 64;

// Batched Krylov workspace of a multi right-hand-side solve.
struct MultiWS {
    double *V = nullptr; size_t cV = 0;
    float *v32 = nullptr; size_t cv32 = 0;
    float *x32 = nullptr; size_t cx32 = 0;
    double *w = nullptr, *r = nullptr, *x = nullptr, *b = nullptr, *d = nullptr, *rr = nullptr;
    size_t cw = 0, cr = 0, cx = 0, cb = 0, cd = 0, crr = 0;
    double *P = nullptr; size_t cP = 0;
    double *H = nullptr; size_t cH = 0;
    double *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
    size_t ccs = 0, csn = 0, cg = 0, cy = 0;
    double *part = nullptr; size_t cpart = 0;
    double *nrm = nullptr; size_t cnrm = 0;
    GState *gs = nullptr; size_t cgs = 0;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int restart_cap = 100;

    Layout L{};
    Flow F{};
    Nodes N{};
    const double *psi_wall = nullptr;

    void *A = nullptr;      size_t capA = 0;
    double *A64 = nullptr;  size_t capA64 = 0;   // FP64 copy beside an FP32 A (multi refine)
    double *V = nullptr;    size_t capV = 0;      // vpre recycled rows, then the basis
    int vpre = 0;
    float *v32 = nullptr;   size_t capv32 = 0;
    double *Urec = nullptr; size_t capUrec = 0;   // U of the recycled space (A U = C)
    double *Brec = nullptr; size_t capBrec = 0;   // B (kRecycleMax x restart) | z
    double *vec[kNumVec] = {};  size_t capvec[kNumVec] = {};
    double *H = nullptr;    size_t capH = 0;
    double *cs = nullptr;   size_t capcs = 0;
    double *sn = nullptr;   size_t capsn = 0;
    double *gv = nullptr;   size_t capg = 0;
    double *yv = nullptr;   size_t capy = 0;
    double *P = nullptr;    size_t capP = 0;
    double *part = nullptr; size_t cappart = 0;
    double *pw = nullptr;   size_t cappw = 0;     // partials of the fused Arnoldi product
    double *hsum = nullptr; size_t caphsum = 0;   // their row sums
    int *bid = nullptr;     size_t capbid = 0;
    int *loc = nullptr;     size_t caploc = 0;
    int *Mk = nullptr;      size_t capMk = 0;
    double *wq = nullptr;   size_t capwq = 0;
    double *s = nullptr;    size_t caps = 0;
    double *lre = nullptr;  size_t caplre = 0;
    double *lim = nullptr;  size_t caplim = 0;
    double *rowD = nullptr; size_t caprowD = 0;
    double *rowH = nullptr; size_t caprowH = 0;
    double *hrow = nullptr; size_t caphrow = 0;     // (1/2) cot(pi n / M_0)
    double *eR = nullptr;   size_t capeR = 0;       // E = e^{i zeta}
    double *eI = nullptr;   size_t capeI = 0;
    double *eRl = nullptr;  size_t capeRl = 0;      // trailing parts of E
    double *eIl = nullptr;  size_t capeIl = 0;
    double *cell = nullptr; size_t capcell = 0;     // E discs of the 64-node cells
    int *nlist = nullptr;   size_t capnlist = 0;    // near-pair cell lists
    double *val = nullptr;  size_t capval = 0;
    double *apart = nullptr; size_t capapart = 0;   // adjoint partial sums
    // surface evolution: rows of D, the antiderivative and the filter on the
    // M_0 grid (recomputed when M_0 changes), stage work vectors and the
    // Runge-Kutta stage derivatives
    int ev_M = 0;
    double *evrow = nullptr; size_t capevrow = 0;    // D | INT | FILTER | sigma
    double *ew = nullptr;    size_t capew = 0;
    double *ek = nullptr;    size_t capek = 0;
    double *hop = nullptr;   size_t caphop = 0;      // interior evaluation partials
    int *hoi = nullptr;      size_t caphoi = 0;
    MultiWS mw;
    GState *gs = nullptr;
    void *hst = nullptr;    // pinned host staging (4 KiB)
    // host-mapped coherent copy of the single-solve cycle state, written by
    // the device kernels (hmir on the host, dmir its device address)
    GState *hmir = nullptr;
    GState *dmir = nullptr;
    int cyc_id = 0;            // id of the latest GMRES cycle enqueued on gs

    hipEvent_t ev[5] = {};
    hipEvent_t pollev[3] = {};   // two convergence polls and the input checks' copy
    // the single-system solve's two step polls: they only pace the host, which
    // then reads the coherent host mirror, so they skip the system-scope fence
    hipEvent_t stepev[2] = {};
    hipEvent_t prof[2 * kProfPairs] = {};
    bool profiling = false;
    // launch -> (cycle, step) of every profiled matvec; steps at or beyond a
    // cycle's completed count were no-ops (enqueued ahead of the flag poll)
    int prof_cycle[kProfPairs] = {};
    int prof_step[kProfPairs] = {};
    std::vector<int> cyc_done;   // completed steps per cycle, -1 while unknown
    // relative residuals for wwbi_report.resid_hist (capacity reserved at
    // creation; values past it are dropped, never reallocated)
    std::vector<double> hist;
    void note_resid(double r) {
        if (hist.size() < hist.capacity()) hist.push_back(r);
    }
    int cur_cycle = -1;
    int cur_step = 0;
    int last_cycle = -1;
    bool trace = false;     // WWBI_TRACE set: one stderr line per GMRES cycle
    int nprof = 0;

    long near_pairs = 0;       // near pairs outside the band of the last geometry
    int val_blocks = 1;        // blocks of the data check of the last setup
    // workspace carved from a fixed region for one call (the allocation-free
    // entry point): ensure() then checks capacities and never allocates
    bool fixed_ws = false;

    // recycle: room for the recycled space of the refinement's inner solves
    int ws_plan(int n, int restart, WsItem *it, bool recycle = true);
    // 128 doubles of norm partials behind the Gram-Schmidt partials
    double *norm_partials() const { return P + 3L * 64 * (restart_cap + 1 + vpre); }
    int ensure(int n, int restart);
    int ensure_matrix(size_t bytes);
    int ensure_matrix64(size_t bytes);
    void release();
    // check = false leaves the device-side input checks to setup_check(), so
    // that work which writes only internal buffers can be queued meanwhile
    int setup(const wwbi_geom *g, const double *phi, int nphi, bool check = true);
    int setup_check();
    // x32 (may be null): an FP32 copy of x for the stored FP32 operators
    void apply(const Op &op, const double *x, const float *x32, const double *c, double *y,
               const int *active);
    double op_bytes(const Op &op) const;
    int read_state(GState &out);
    // state at the end of the latest cycle: the published copy when it is that
    // cycle's (after a synchronisation past the cycle's end), else a copy of gs
    int final_state(GState &out);
    void prof_begin();
    void prof_end();
    // kc > 0: deflate the kc recycled vectors in front of the basis (one
    // cycle, no verification, x = the solution from zero)
    int gmres(const Op &op, const double *b, double *x, bool x_zero, double tol, int restart,
              int max_iter, int poll, bool verify, SolveStats &st, int kc = 0);
    double device_norm(const double *v, int n);
    int refine(const Op &op32, const Op &op64, const double *b, double *x, bool x_zero,
               const wwbi_opts &o, SolveStats &st);
    int ensure_multi(int n, int nr, int restart);
    void apply_multi(int kind, int n, long ld, const double *X, const float *X32, long xs, int nr,
                     const double *c, double *Y);
    int read_states(GState *out, int nr);
    int gmres_multi(int kind, int n, long ld, const double *B, double *X, int nr, double tol,
                    int restart, int max_iter, int poll, bool verify, SolveStats &st);
    int refine_multi(int n, long ld, const double *B, double *X, int nr, const wwbi_opts &o,
                     bool stored64, SolveStats &st);
    void eval_U_from_gamma(const double *gamma, double *U);
    void gamma_from_omega(const double *omega, double *gamma);
    static int check_opts(const wwbi_opts *o);
    void begin_report(bool prof);
    void finish_report(wwbi_report *rep, int status, const SolveStats &st, double bytes);
};

// The velocity-potential solve behind wwbi_solve_phi (its workspace is the
// context's, grown on demand unless Ctx::fixed_ws).
int solve_phi_impl(Ctx *c, const wwbi_geom *g, const double *phi, const wwbi_opts *o,
                   double *U, double *omega, double *psi_k, wwbi_report *rep);

// Looks up, once per device and with that device current, the device address
// of the allocation-free entry point's static scratch array.
void scratch_init(int device);

}  // namespace wwbi
