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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--mode", default="stored", choices=["stored", "otf"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--inner-tol", type=float, default=3e-7)
    ap.add_argument("--poll", type=int, default=4)
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def timed_solves(ctx, dg, phi, steps, warmup, flags=0, **kw):
    """Warm up, then time `steps` solves bracketed by device synchronisation.

    The first timed step also brackets every launch of the dominant matvec
    with HIP events on the library's stream (the report's n_matvec and
    ms_matvec); the event records add a short gap around each launch, so the
    other steps run without them."""
    from paper_2108_01786_amd import wwbi
    for _ in range(warmup):
        ctx.solve_phi(dg, phi, flags=flags, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    out = None
    for k in range(steps):
        f = flags | (wwbi.FLAG_PROFILE if k == 0 else 0)
        out = ctx.solve_phi(dg, phi, flags=f, **kw)
        reps.append(out[3].as_dict())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, reps, out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
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
        mv64 = sum(r["ms_matvec"] for r in reps64) / max(1, sum(r["n_matvec"] for r in reps64))
        res["fp64_matvec_ms"] = mv64
        res["fp64_matvec_GBs"] = reps64[-1]["bytes_matvec"] / (mv64 * 1e-3) / 1e9 if mv64 else None

    nmv = sum(r["n_matvec"] for r in reps32)
    msmv = sum(r["ms_matvec"] for r in reps32)
    avg = msmv / max(1, nmv)
    bytes_mv = reps32[-1]["bytes_matvec"]
    achieved = bytes_mv / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_gemv<float,float,float,2,4> (stored FP32 matvec)",
            "avg_launch_ms": avg, "launches": nmv, "bytes_per_launch": bytes_mv}

    cpu = None
    if not a.no_cpu_baseline:
        import oracle as O
        og = O.OGeom.from_synth(geom)
        t0 = time.perf_counter()
        ref = O.solve_phi(og, torch.as_tensor(cfg["phi"]))
        tcpu = time.perf_counter() - t0
        cpu = {"value": 1.0 / tcpu, "unit": "solves/s", "cores": torch.get_num_threads(),
               "kind": "oracle",
               "sample": f"one full FP64 solve of the same M={geom.Mtot} cell (dense LU)"}
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
        "iters": last["iters"], "refine_steps": last["refine_steps"],
        "phase_ms": {k: last[k] for k in ("ms_prep", "ms_assemble", "ms_solve", "ms_U")},
        "roofline": roof, "cpu_baseline": cpu,
    }
    line.update(res)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
