#!/usr/bin/env python3
"""Throughput of the boundary-integral solve (assembly + GMRES + U) on one GPU.

One step = one complete velocity-potential solve from device-resident inputs:
right-hand side, assembly of the dense collocated system, GMRES (inside FP64
iterative refinement for the FP32 path) and the normal velocity U.  The
matrix is re-assembled every step, as in a time-stepping stage.

Workload: the refined-FP32 cell of M = 10240 unknowns (surface 4096 nodes,
flat bottom 2048, four ellipses of 1024), refinement to a relative residual
of 1e-14 (the extra decade keeps the FP32 noise of the last correction
out of U).  The same steps are also timed in plain FP64 (GMRES to 1e-13).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_k_gemv_fp32_config3_M10240.md")
TRAFFIC_FILE_LARGE = os.path.join(ROOT, "profiles", "hbm_traffic_k_gemv_fp32_large_M40960.md")


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch of the stored FP32 matvec from a committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by a
    1 GiB copy), or None when the kernel source changed since it was taken."""
    import hashlib
    try:
        text = open(path).read()
        src = open(os.path.join(ROOT, "paper_2108_01786_amd", "csrc", "kernels_gemv.hip"), "rb").read()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith(("*", "#")))
    if vals.get("kernels_gemv_sha256", "").strip() != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


INFINITY_CACHE_BYTES = 256 << 20


def copy_bandwidth(dev, mib=1024, reps=5):
    """Achievable HBM bandwidth of a plain device copy (read + write bytes per
    second, GB/s), timed with events on torch's stream after the timed region."""
    src = torch.empty(mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    nbytes = 2 * src.numel() * 4
    del src, dst
    return nbytes / (float(np.median(ts)) * 1e-3) / 1e9


def add_copy_reference(roof, dev, matrix_bytes):
    """Put the copy kernel's bandwidth beside the published peak, and label a
    matrix that fits the 256 MB Infinity Cache as cache-resident (its figure is
    an effective bandwidth, not an HBM one)."""
    cb = copy_bandwidth(dev)
    roof["copy_GBs"] = cb
    roof["copy_kind"] = "torch device copy of 1 GiB, read + write bytes, median of 5"
    roof["frac_of_copy"] = roof["achieved"] / cb if cb > 0 else None
    roof["cache_resident"] = matrix_bytes <= INFINITY_CACHE_BYTES
    if roof["cache_resident"]:
        roof["note"] = "effective (cache-resident) bandwidth: the matrix fits the Infinity Cache"
    return roof


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--mode", default="stored", choices=["stored", "otf"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--inner-tol", type=float, default=1e-7)
    ap.add_argument("--poll", type=int, default=2)
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--workload", default="solve", choices=["solve", "adjoint", "large-stages"],
                    help="solve: one solve on the cell --config names (default: M = 10240); "
                         "adjoint: forward + adjoint gradient on the M = 4608 cell; "
                         "large-stages: forward + adjoint stages on the M = 40960 cell")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip timing the diagnostics and the gamma_t stage")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum host time spent on the oracle baseline sample")
    return ap.parse_args()


def stats_ms(reps, key="ms_total"):
    v = np.array([r[key] for r in reps])
    q1, med, q3 = np.percentile(v, [25, 50, 75])
    return {"median": float(med), "iqr": float(q3 - q1), "min": float(v.min()), "max": float(v.max())}


def timed_solves(ctx, dg, phi, steps, warmup, flags=0, **kw):
    """Warm up, then time `steps` solves bracketed by device synchronisation.

    The first timed step also brackets every launch of the dominant matvec
    with HIP events on the library's stream (the report's n_matvec and
    ms_matvec); the event records add a short gap around each launch, so the
    other steps run without them."""
    from paper_2108_01786_amd import wwbi
    # outputs allocated once, as a time-stepping caller would
    U = torch.empty(dg.M[0], dtype=torch.float64, device=phi.device)
    om = torch.empty(dg.n, dtype=torch.float64, device=phi.device)
    for _ in range(warmup):
        ctx.solve_phi(dg, phi, flags=flags, U=U, omega=om, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    out = None
    for k in range(steps):
        f = flags | (wwbi.FLAG_PROFILE if k == 0 else 0)
        out = ctx.solve_phi(dg, phi, flags=f, U=U, omega=om, **kw)
        reps.append(out[3].as_dict())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, reps, out


def time_extras(ctx, dg, geom, phi, a, reps=5):
    """Per-call times, on the same cell, of the other entry points: the
    vortex-sheet solve, the diagnostics (tangential velocity on every node and the energy), the
    gamma_t stage (its own velocity-potential solve plus the right-hand side
    and the n x n FP64 system), one evolution stage and one DOP853 step (HLS
    surface), velocity and pressure at 4096 points inside the fluid, and
    solves with 1, 8 and 32 right-hand sides against one matrix."""
    from paper_2108_01786_amd import wwbi
    M0 = geom.M[0]
    al = torch.arange(M0, dtype=torch.float64, device=phi.device) * (2 * np.pi / M0)
    V = 0.1 * torch.sin(al) + 0.03 * torch.cos(2 * al)
    U64, omega, _, _ = ctx.solve_phi(dg, phi, tol=1e-13)
    out = {}
    # the vortex-sheet entry on the same cell, gamma_0 = -D omega_0 from the
    # FP64 velocity-potential solve; both formulations give the same U
    gam0 = ctx.spectral(omega[:M0].contiguous(), wwbi.OP_D, alpha=-1.0)
    gs = []
    for _ in range(reps + 1):
        Ug, _, r = ctx.solve_gamma(dg, gam0, tol=1e-13, restart=100, poll_every=a.poll)
        gs.append(r.as_dict())
    out["solve_gamma_ms"] = stats_ms(gs[1:])
    out["solve_gamma_iters"] = gs[-1]["iters"]
    out["solve_gamma_phases_ms"] = {k: gs[-1][k] for k in ("ms_prep", "ms_assemble", "ms_solve", "ms_U")}
    out["solve_gamma_U_vs_solve_phi_U"] = float((Ug - U64).abs().max() / U64.abs().max())
    gr = []
    for _ in range(reps + 1):
        Ugr, _, r = ctx.solve_gamma(dg, gam0, tol=1e-14, restart=100, poll_every=a.poll,
                                    precision=wwbi.FP32_REFINED, inner_tol=a.inner_tol)
        gr.append(r.as_dict())
    out["solve_gamma_refined_ms"] = stats_ms(gr[1:])
    out["solve_gamma_refined_iters"] = gr[-1]["iters"]
    out["solve_gamma_refined_U_vs_solve_phi_U"] = float((Ugr - U64).abs().max() / U64.abs().max())
    te = []
    for _ in range(reps + 1):
        _, _, r = ctx.tangential_energy(dg, omega, phi, tau=0.1, grav=1.0)
        te.append(r.as_dict())
    out["tangential_energy_ms"] = stats_ms(te[1:])
    gt, gp = [], []
    for _ in range(reps + 1):
        _, _, r1, r2 = ctx.solve_gamma_t(dg, phi, V, tau=0.1, tol=1e-13, restart=100,
                                         poll_every=a.poll)
        gt.append(r2.as_dict())
        gp.append(r1.as_dict())
    out["gamma_t_stage_ms"] = stats_ms(gt[1:])
    out["gamma_t_phi_solve_ms"] = stats_ms(gp[1:])
    out["gamma_t_iters"] = gt[-1]["iters"]
    out["gamma_t_phases_ms"] = {k: gt[-1][k] for k in ("ms_prep", "ms_assemble", "ms_solve")}
    # the same stage with both solves in refined FP32
    gr, gpr = [], []
    for _ in range(reps + 1):
        _, _, r1, r2 = ctx.solve_gamma_t(dg, phi, V, tau=0.1, tol=1e-14, restart=100,
                                         precision=wwbi.FP32_REFINED, inner_tol=a.inner_tol,
                                         poll_every=a.poll)
        gr.append(r2.as_dict())
        gpr.append(r1.as_dict())
    out["gamma_t_stage_refined_ms"] = stats_ms(gr[1:])
    out["gamma_t_phi_solve_refined_ms"] = stats_ms(gpr[1:])
    out["gamma_t_refined_iters"] = gr[-1]["iters"]
    out["gamma_t_refined_refine_steps"] = gr[-1]["refine_steps"]
    # one evolution stage (HLS surface, refined FP32 solve) and one DOP853 step
    # (tableau from tests/golden/dop853_tableau.json) on the same walls; the stage's surface is
    # written into a copy of the geometry
    dg2 = wwbi.DeviceGeometry.from_synth(geom, phi.device)
    Pt = (0.15 * torch.sin(al) + 0.05 * torch.cos(2 * al)).contiguous()
    kw = dict(precision=wwbi.FP32_REFINED, tol=1e-14, inner_tol=a.inner_tol, restart=100,
              poll_every=a.poll)
    st_ms = []
    for _ in range(reps + 1):
        t0 = time.perf_counter()
        ctx.stage_rhs(dg2, wwbi.SURF_HLS, Pt, phi, tau=0.1, **kw)
        torch.cuda.synchronize()
        st_ms.append(1e3 * (time.perf_counter() - t0))
    out["stage_hls_ms"] = float(np.median(st_ms[1:]))
    try:
        with open(os.path.join(ROOT, "tests", "golden", "dop853_tableau.json")) as f:
            tab = json.load(f)
        A = np.array(tab["A"], dtype=np.float64)
        b = np.array(tab["b"], dtype=np.float64)
        q, p = Pt.clone(), phi.clone().contiguous()
        # the capillary mode at k = M0/2 turns at about sqrt(tau k^3) = 2.9e4
        # rad per unit time and DOP853 is stable to |h omega| ~ 5.9 on the
        # imaginary axis; h = 1e-5 also keeps the stages' high modes at the
        # FP64 floor
        rep = ctx.rk_step(dg2, wwbi.SURF_HLS, A, b, 1e-5, q, p, tau=0.1, **kw)
        out["dop853_step_ms"] = rep.ms_total
        out["dop853_step_iters"] = rep.iters
    except OSError:
        pass
    # velocity and pressure at 4096 points inside the fluid (Helsing-Ojala rule)
    g0 = geom.curves[0]
    Mq = 4096
    idx = np.arange(Mq) * (M0 // Mq if M0 >= Mq else 1) % M0
    nrm = -1j * g0.d[idx] / np.abs(g0.d[idx])
    zpts = torch.as_tensor(g0.z[idx] + np.geomspace(1e-6, 0.2, Mq) * nrm, device=phi.device)
    vel, prs = [], []
    for _ in range(reps + 1):
        t0 = time.perf_counter()
        ctx.interior_velocity(dg, omega, zpts)
        torch.cuda.synchronize()
        vel.append(1e3 * (time.perf_counter() - t0))
        t0 = time.perf_counter()
        ctx.pressure(dg, phi, zpts, tau=0.1, tol=1e-13, poll_every=a.poll)
        torch.cuda.synchronize()
        prs.append(1e3 * (time.perf_counter() - t0))
    out["interior_velocity_4096pts_ms"] = float(np.median(vel[1:]))
    out["pressure_4096pts_ms"] = float(np.median(prs[1:]))
    # several right-hand sides against one matrix (matrix-core product and
    # lockstep GMRES), refined FP32, seeded normal right-hand sides
    n = geom.Mtot
    mr = {}
    for nr in (1, 8, 32):
        rhs = torch.as_tensor(np.random.default_rng(178610 + nr).standard_normal((nr, n)),
                              device=phi.device)
        ts = []
        for _ in range(reps + 1):
            t0 = time.perf_counter()
            _, r = ctx.solve_phi_multi(dg, rhs, precision=wwbi.FP32_REFINED, tol=1e-14,
                                       inner_tol=a.inner_tol, restart=100, poll_every=a.poll)
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        med = float(np.median(ts[1:]))
        mr[str(nr)] = {"ms": med, "ms_per_rhs": med / nr, "iters": r.iters,
                       "refine_steps": r.refine_steps}
    out["multi_rhs_refined"] = mr
    return out


def large_cpu_baseline(geom, rows=4096, steps=55):
    """The oracle's forward solve on the large cell, timed on a bounded sample
    and scaled: `rows` of the 40960 rows of A assembled (oracle.A_rows),
    `steps` products of that row block with a vector (the oracle's GMRES took
    55 steps on this cell), and the U map's share for `rows` sources (the
    transposed G_00 block applied to them), all times n / rows.  The oracle's
    adjoint (its tangent-linear model) is left out, so the stage rate this
    gives is an upper bound for the oracle."""
    import oracle as O
    og = O.OGeom.from_synth(geom)
    n = geom.Mtot
    nthreads = torch.get_num_threads()
    t0 = time.perf_counter()
    blk = O.A_rows(og, range(rows))
    t1 = time.perf_counter()
    x = torch.ones(n, dtype=torch.float64)
    for _ in range(steps):
        _ = blk @ x
    t2 = time.perf_counter()
    src = torch.arange(min(rows, geom.M[0]))
    _ = O.G_block(og, 0, 0, src).T @ torch.ones(src.shape[0], dtype=torch.float64)
    t3 = time.perf_counter()
    scale = n / rows
    t_fwd = (t3 - t0) * scale
    return {"value": 1.0 / t_fwd, "unit": "stages/s", "cores": nthreads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"oracle forward only: {rows} of {n} rows of A assembled ({t1 - t0:.1f} s), "
                       f"{steps} products with that block ({t2 - t1:.1f} s), the U map for "
                       f"{src.shape[0]} sources ({t3 - t2:.1f} s), scaled by n / {rows} = "
                       f"{scale:.0f} to {t_fwd:.0f} s per forward solve; the adjoint is not "
                       f"included")}


def run_large(a):
    """Forward + adjoint stages on the M = 40960 cell (surface 16384, bottom
    8192, eight ellipses of 2048): stage s moves the surface and phi by
    s * 1e-3 times a seeded smooth displacement (degree <= 32), runs the
    refined-FP32 solve for U warm-started from the previous stage's omega, and
    the adjoint of J = sum w U^2 (weights ~ U[0, 1]).  One step is one stage."""
    from paper_2108_01786_amd import wwbi
    from paper_2108_01786_amd.autograd import SurfaceProblem
    from synth import make_config

    cfg = make_config(5)
    geom = cfg["geom"]
    dev = "cuda:0"
    ctx = wwbi.Context(0)
    prob = SurfaceProblem(ctx, geom, dev)
    M0 = geom.M[0]
    z0 = geom.curves[0].z
    al = 2 * np.pi * np.arange(M0) / M0
    xt0, yt0, ph0 = z0.real - al, z0.imag, np.asarray(cfg["phi"])
    disp = cfg["stage_disp"]
    w = torch.as_tensor(np.random.default_rng(178605).uniform(0.0, 1.0, M0), device=dev)
    ctx.reserve(geom.Mtot, 120, wwbi.FP32_REFINED)
    # the paper's tolerance (Sec. 7.4): U on this near-overturning surface
    # amplifies what the solve leaves in omega by up to about 3e4
    opts = dict(precision=wwbi.FP32_REFINED, tol=1e-15, inner_tol=a.inner_tol,
                matvec=wwbi.MATVEC_STORED, restart=120, poll_every=a.poll)
    inputs = []
    for s in range(4):
        f = s * 1e-3
        inputs.append([torch.as_tensor(v, device=dev) for v in
                       (xt0 + f * disp[0], yt0 + f * disp[1], ph0 + f * disp[2])])

    def stage(s, x0, flags=0):
        xt, yt, ph = inputs[s]
        g = prob.fill(xt, yt)
        U, om, _, rf = ctx.solve_phi(g, ph, x0=x0, flags=flags, **opts)
        grads, ra = ctx.adjoint_phi(g, om, 2.0 * w * U, **opts)
        ctx.surface_fill_adjoint([grads[k] for k in ("x", "y", "dx", "dy", "ddx", "ddy")])
        return om, rf.as_dict(), ra.as_dict()

    log(f"bench: large stages M={geom.Mtot}")
    om = None
    cold = None
    for k in range(a.warmup):
        om, rf, ra = stage(k % 4, om)
        cold = cold or rf
    torch.cuda.synchronize()
    fw, ad = [], []
    t0 = time.perf_counter()
    for k in range(a.steps):
        om, rf, ra = stage((a.warmup + k) % 4, om, wwbi.FLAG_PROFILE if k == 0 else 0)
        fw.append(rf)
        ad.append(ra)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / a.steps
    log(f"bench: {1e3 * t:.2f} ms per stage")
    p = fw[0]
    avg = p["ms_matvec"] / max(1, p["n_matvec"])
    achieved = p["bytes_matvec"] / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
    line = {
        "metric": "refined-FP32 forward+adjoint stages/s at 40960 unknowns",
        "value": 1.0 / t, "unit": "stages/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * t, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 matvec + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"forward+adjoint stages, M={geom.Mtot} (surface {M0}, bottom "
                               f"{geom.M[1]}, {geom.nb - 2} ellipses of {geom.M[2]})",
                   "unknowns": geom.Mtot, "matvec": "stored", "tol": 1e-15, "restart": 120,
                   "warm_start": True},
        "forward_ms": stats_ms(fw), "adjoint_ms": stats_ms(ad),
        "forward_iters_warm": [r["iters"] for r in fw],
        "forward_iters_cold": cold["iters"] if cold else None,
        "adjoint_iters": [r["iters"] for r in ad],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(TRAFFIC_FILE_LARGE),
                     "kernel": "k_gemv<float,float,double,2,4,true,4> (stored FP32 matvec, FP64 accumulation, with the first Gram-Schmidt dots)",
                     "avg_launch_ms": avg, "launches": p["n_matvec"],
                     "bytes_per_launch": p["bytes_matvec"]},
        "cpu_baseline": None if a.no_cpu_baseline else large_cpu_baseline(geom),
    }
    line["roofline"] = add_copy_reference(line["roofline"], dev, 4 * geom.Mtot * geom.Mtot)
    print(json.dumps(line), flush=True)
    ctx.close()


def run_adjoint(a):
    """Gradient of J = sum w U^2 with respect to the surface displacements and
    phi on the M = 4608 cell (surface 2048, bottom 1024, three ellipses of 512;
    weights ~ U[0, 1]).  One step is the forward solve plus the adjoint: the
    transpose solve, the kernel-derivative contractions and the chain rule
    through the spectral derivatives.  Timed in refined FP32 (the value) and
    in FP64.  Beside it, the tangent-linear model along the cell's 32 seeded
    directions in one call (32 systems sharing the matrix), with its dJ
    checked against the adjoint's gradient along the same directions."""
    from paper_2108_01786_amd import wwbi
    from paper_2108_01786_amd.autograd import SurfaceProblem
    from synth import make_config

    cfg = make_config(4)
    geom = cfg["geom"]
    dev = "cuda:0"
    ctx = wwbi.Context(0)
    prob = SurfaceProblem(ctx, geom, dev)
    M0 = geom.M[0]
    z0 = geom.curves[0].z
    al = 2 * np.pi * np.arange(M0) / M0
    xt_h, yt_h, ph_h = z0.real - al, z0.imag, np.asarray(cfg["phi"])
    xt, yt, ph = (torch.as_tensor(v, device=dev) for v in (xt_h, yt_h, ph_h))
    wt = torch.as_tensor(cfg["weights"], device=dev)
    ctx.reserve(geom.Mtot, 100, wwbi.FP64)

    def step(opts, flags=0):
        g = prob.fill(xt, yt)
        U, om, _, rf = ctx.solve_phi(g, ph, flags=flags, **opts)
        grads, ra = ctx.adjoint_phi(g, om, 2.0 * wt * U, flags=flags, **opts)
        gx, gy = ctx.surface_fill_adjoint([grads[k] for k in ("x", "y", "dx", "dy", "ddx", "ddy")])
        return (U, gx, gy, grads["phi"]), rf.as_dict(), ra.as_dict()

    def timed(opts, steps, warmup):
        for _ in range(warmup):
            step(opts)
        torch.cuda.synchronize()
        fw, ad, wall = [], [], []
        t0 = time.perf_counter()
        for k in range(steps):
            ts = time.perf_counter()
            out, rf, ra = step(opts, wwbi.FLAG_PROFILE if k == 0 else 0)
            torch.cuda.synchronize()
            wall.append({"ms_total": 1e3 * (time.perf_counter() - ts)})
            fw.append(rf)
            ad.append(ra)
        t = (time.perf_counter() - t0) / steps
        return t, out, fw, ad, wall

    o32 = dict(precision=wwbi.FP32_REFINED, tol=1e-14, inner_tol=a.inner_tol, restart=100,
               poll_every=a.poll)
    o64 = dict(precision=wwbi.FP64, tol=1e-13, restart=100, poll_every=a.poll)
    log(f"bench: adjoint M={geom.Mtot}")
    t32, out32, fw32, ad32, wall32 = timed(o32, a.steps, a.warmup)
    log(f"bench: refined fp32 forward+adjoint {1e3 * t32:.3f} ms")
    t64, out64, fw64, ad64, wall64 = timed(o64, a.steps, a.warmup)
    log(f"bench: fp64 forward+adjoint {1e3 * t64:.3f} ms")

    # the tangent-linear model along the cell's 32 seeded displacement
    # directions (x~, y~, phi~ with their spectral derivatives), one call: the
    # 32 systems A d omega_i = r_i share the matrix
    g = prob.fill(xt, yt)
    U32, om32, _, _ = ctx.solve_phi(g, ph, **o32)
    U64, om64, _, _ = ctx.solve_phi(g, ph, **o64)
    comp = []
    for d in cfg["directions"]:
        d0, d1 = (torch.as_tensor(v, device=dev) for v in (d[0], d[1]))
        d0p, d1p = ctx.spectral(d0, wwbi.OP_D), ctx.spectral(d1, wwbi.OP_D)
        comp.append(torch.stack([d0, d1, d0p, d1p, ctx.spectral(d0p, wwbi.OP_D),
                                 ctx.spectral(d1p, wwbi.OP_D), torch.as_tensor(d[2], device=dev)]))
    tdirs = torch.stack(comp, dim=1).contiguous()                  # 7 x 32 x M_0

    def tangent(om, opts, steps, warmup):
        for _ in range(warmup):
            ctx.tangent_phi(g, om, tdirs, **opts)
        torch.cuda.synchronize()
        reps, wall = [], []
        for k in range(steps):
            ts = time.perf_counter()
            dU, _, rt = ctx.tangent_phi(g, om, tdirs, flags=wwbi.FLAG_PROFILE if k == 0 else 0,
                                        **opts)
            torch.cuda.synchronize()
            wall.append({"ms_total": 1e3 * (time.perf_counter() - ts)})
            reps.append(rt.as_dict())
        return dU, reps, wall

    dU32, tr32, tw32 = tangent(om32, o32, a.steps, a.warmup)
    dU64, tr64, tw64 = tangent(om64, o64, a.steps, a.warmup)
    log(f"bench: tangent 32 directions refined {stats_ms(tw32)['median']:.3f} ms, "
        f"fp64 {stats_ms(tw64)['median']:.3f} ms")
    # dJ_i from the tangent against the adjoint's gradient along the same directions
    grads, _ = ctx.adjoint_phi(g, om64, 2.0 * wt * U64, **o64)
    gv = torch.stack([grads[k] for k in ("x", "y", "dx", "dy", "ddx", "ddy", "phi")])
    dJ_adj = (gv[:, None, :] * tdirs).sum(dim=(0, 2))
    tangent_info = {"directions": len(cfg["directions"])}
    for name, dU, tr, tw, U in (("refined", dU32, tr32, tw32, U32), ("fp64", dU64, tr64, tw64, U64)):
        dJ = (2.0 * wt * U * dU).sum(dim=1)
        mv = tr[0]["ms_matvec"] / max(1, tr[0]["n_matvec"])
        tangent_info[name] = {
            "ms_stats": stats_ms(tw), "iters": tr[-1]["iters"],
            "refine_steps": tr[-1]["refine_steps"],
            "multi_product_avg_ms": mv, "multi_product_launches": tr[0]["n_matvec"],
            "multi_product_GBps": tr[0]["bytes_matvec"] / (mv * 1e-3) / 1e9 if mv > 0 else None,
            "dJ_rel_diff_vs_adjoint": float((dJ - dJ_adj).abs().max() / dJ_adj.abs().max())}

    nmv = fw32[0]["n_matvec"] + ad32[0]["n_matvec"]
    msmv = fw32[0]["ms_matvec"] + ad32[0]["ms_matvec"]
    avg = msmv / max(1, nmv)
    bytes_mv = fw32[0]["bytes_matvec"]
    achieved = bytes_mv / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_gemv<float,float,double,2,4,true,4> (stored FP32 matvec, FP64 accumulation, with the first Gram-Schmidt dots, A and A^T)",
            "avg_launch_ms": avg, "launches": nmv, "bytes_per_launch": bytes_mv}

    res = {}
    cpu = None
    if not a.no_cpu_baseline:
        import oracle as O
        og = O.OGeom.from_synth(geom)
        n = 0
        t0 = time.perf_counter()
        while True:
            Jr, rx, ry, rp, Ur = O.J_and_grad(og, xt_h, yt_h, ph_h, cfg["weights"])
            n += 1
            tc = time.perf_counter() - t0
            if tc >= a.cpu_seconds:
                break
        cpu = {"value": n / tc, "unit": "gradients/s", "cores": torch.get_num_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{n} FP64 forward solves with autograd gradients of J on the same "
                         f"M={geom.Mtot} cell (dense LU and one extended-precision refinement step), {tc:.1f} s"}
        ref = [Ur.numpy(), rx.numpy(), ry.numpy(), rp.numpy()]
        for name, out in (("refined", out32), ("fp64", out64)):
            res[f"err_vs_oracle_{name}"] = {
                k: float(np.abs(o.cpu().numpy() - r).max() / np.abs(r).max())
                for k, o, r in zip(("U", "dJ_dxt", "dJ_dyt", "dJ_dphi"), out, ref)}

    roof = add_copy_reference(roof, dev, 4 * geom.Mtot * geom.Mtot)
    s32, s64 = stats_ms(wall32), stats_ms(wall64)
    line = {
        "metric": "refined-FP32 forward+adjoint gradients/s at 4608 unknowns",
        "value": 1.0 / t32, "unit": "gradients/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * t32, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 matvec + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"gradient of sum w U^2, M={geom.Mtot} (surface {M0}, bottom "
                               f"{geom.M[1]}, {geom.nb - 2} ellipses of {geom.M[2]})",
                   "unknowns": geom.Mtot, "matvec": "stored", "tol_refined": 1e-14,
                   "tol_fp64": 1e-13},
        "ms_per_step_stats": s32, "gradients_per_s_median": 1e3 / s32["median"],
        "forward_ms": stats_ms(fw32), "adjoint_ms": stats_ms(ad32),
        "forward_iters": fw32[-1]["iters"], "adjoint_iters": ad32[-1]["iters"],
        "refine_steps": [fw32[-1]["refine_steps"], ad32[-1]["refine_steps"]],
        "fp64_gradients_per_s": 1.0 / t64, "fp64_ms_per_step_stats": s64,
        "fp64_forward_iters": fw64[-1]["iters"], "fp64_adjoint_iters": ad64[-1]["iters"],
        "tangent_linear": tangent_info,
        "roofline": roof, "cpu_baseline": cpu,
    }
    line.update(res)
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: the solve runs on a single device; --gpus must be 1"}))
        sys.exit(2)
    if a.workload == "large-stages":
        return run_large(a)
    if a.workload == "adjoint":
        return run_adjoint(a)
    from paper_2108_01786_amd import wwbi
    from synth import make_config, CONFIG_NAMES

    cfg = make_config(a.config)
    geom = cfg["geom"]
    dev = "cuda:0"
    ctx = wwbi.Context(0)
    dg = wwbi.DeviceGeometry.from_synth(geom, dev)
    phi = torch.as_tensor(cfg["phi"], device=dev)
    mv = wwbi.MATVEC_STORED if a.mode == "stored" else wwbi.MATVEC_ON_THE_FLY
    ctx.reserve(geom.Mtot, 100, wwbi.FP64 if mv == wwbi.MATVEC_STORED else -1)
    kw32 = dict(precision=wwbi.FP32_REFINED, tol=1e-14, inner_tol=a.inner_tol, matvec=mv,
                restart=100, poll_every=a.poll)
    log(f"bench: config {a.config} ({CONFIG_NAMES.get(a.config)}) M={geom.Mtot} refined-fp32")
    t32, reps32, out32 = timed_solves(ctx, dg, phi, a.steps, a.warmup, **kw32)
    log(f"bench: refined fp32 {1e3 * t32:.3f} ms/solve")
    res = {}
    if not a.no_fp64:
        kw64 = dict(precision=wwbi.FP64, tol=1e-13, matvec=mv, restart=100,
                    poll_every=a.poll)
        t64, reps64, out64 = timed_solves(ctx, dg, phi, max(3, a.steps // 2), 1, **kw64)
        log(f"bench: fp64 {1e3 * t64:.3f} ms/solve")
        res["fp64_solves_per_s"] = 1.0 / t64
        res["fp64_ms_per_solve"] = 1e3 * t64
        res["fp64_iters"] = reps64[-1]["iters"]
        res["fp64_ms_per_solve_stats"] = stats_ms(reps64)
        res["fp64_solves_per_s_median"] = 1e3 / res["fp64_ms_per_solve_stats"]["median"]
        mv64 = sum(r["ms_matvec"] for r in reps64) / max(1, sum(r["n_matvec"] for r in reps64))
        res["fp64_matvec_ms"] = mv64
        res["fp64_matvec_GBs"] = reps64[-1]["bytes_matvec"] / (mv64 * 1e-3) / 1e9 if mv64 else None

    nmv = sum(r["n_matvec"] for r in reps32)
    msmv = sum(r["ms_matvec"] for r in reps32)
    avg = msmv / max(1, nmv)
    bytes_mv = reps32[-1]["bytes_matvec"]
    achieved = bytes_mv / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
    traffic = measured_traffic() if (a.config == 3 and a.mode == "stored") else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_gemv<float,float,double,2,4,true,4> (stored FP32 matvec, FP64 accumulation, with the first Gram-Schmidt dots)",
            "avg_launch_ms": avg, "launches": nmv, "bytes_per_launch": bytes_mv}

    cpu = None
    if not a.no_cpu_baseline:
        import oracle as O
        og = O.OGeom.from_synth(geom)
        nsol = 0
        t0 = time.perf_counter()
        while True:
            ref = O.solve_phi(og, torch.as_tensor(cfg["phi"]))
            nsol += 1
            tcpu = time.perf_counter() - t0
            if tcpu >= a.cpu_seconds:
                break
        cpu = {"value": nsol / tcpu, "unit": "solves/s", "cores": torch.get_num_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{nsol} full FP64 solves of the same M={geom.Mtot} cell (assembly, "
                         f"dense LU with one extended-precision refinement step, U), {tcpu:.1f} s"}
        if geom.Mtot <= 4608:
            # the small cells are also timed on one host thread
            nt = torch.get_num_threads()
            torch.set_num_threads(1)
            try:
                n1 = 0
                t0 = time.perf_counter()
                while time.perf_counter() - t0 < min(a.cpu_seconds, 10.0) or n1 == 0:
                    O.solve_phi(og, torch.as_tensor(cfg["phi"]))
                    n1 += 1
                cpu["value_1_thread"] = n1 / (time.perf_counter() - t0)
            finally:
                torch.set_num_threads(nt)
        U, omega, psi, _ = out32
        Ur, wr = ref["U"].numpy(), ref["omega"].numpy()
        res["err_vs_oracle_refined"] = {
            "U": float(np.abs(U.cpu().numpy() - Ur).max() / np.abs(Ur).max()),
            "omega": float(np.abs(omega.cpu().numpy() - wr).max() / np.abs(wr).max()),
            "psi_k": float(np.abs(psi - ref["psi_k"].numpy()).max() / np.abs(ref["psi_k"].numpy()).max()),
        }
        if not a.no_fp64:
            U, omega, psi, _ = out64
            res["err_vs_oracle_fp64"] = {
                "U": float(np.abs(U.cpu().numpy() - Ur).max() / np.abs(Ur).max()),
                "omega": float(np.abs(omega.cpu().numpy() - wr).max() / np.abs(wr).max()),
            }

    if not a.no_extras:
        res["extras"] = time_extras(ctx, dg, geom, phi, a)

    if a.copy_calib_mb:
        # a device copy of known size for scaling the HBM counters; a 1 GiB
        # write to another buffer first evicts the source from the MALL
        src = torch.empty(a.copy_calib_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        evict = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(2.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del evict
        log(f"bench: calibration copy of {a.copy_calib_mb} MiB done")

    roof = add_copy_reference(roof, dev, 4 * geom.Mtot * geom.Mtot)
    last = reps32[-1]
    line = {
        "metric": "assembly+GMRES solves/s at ~10k unknowns; refined FP32 vs FP64 at 1e-10 rel",
        "value": 1.0 / t32, "unit": "solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * t32, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 matvec + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"refined-FP32 cell M={geom.Mtot} "
                               f"(surface {geom.M[0]}, bottom {geom.M[1]}, "
                               f"{geom.nb - 2} ellipses of {geom.M[2]})",
                   "unknowns": geom.Mtot, "matvec": a.mode, "tol_refined": 1e-14,
                   "tol_fp64": 1e-13},
        "ms_per_solve_stats": stats_ms(reps32),
        "solves_per_s_median": 1e3 / stats_ms(reps32)["median"],
        "iters": last["iters"], "refine_steps": last["refine_steps"],
        "phase_ms": {k: last[k] for k in ("ms_prep", "ms_assemble", "ms_solve", "ms_U")},
        "roofline": roof, "cpu_baseline": cpu,
    }
    line.update(res)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
