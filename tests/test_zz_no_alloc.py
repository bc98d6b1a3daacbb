"""The allocation-free solve (wwbi_solve_phi_noalloc) against the solve it is a
variant of (wwbi_solve_phi with the on-the-fly matvec), through the C ABI.

Two calls in a row on one context, the second on a smaller problem (4608 then
640 unknowns), in FP64 and in refined FP32: U, omega and psi|_k must match
the ordinary entry point's to the parity bars of the solves (1e-11 FP64,
1e-10 refined; the kernels are the same, so the results agree to rounding),
and the first call's U matches the FP64 oracle.  The call must leave the
device's free memory unchanged (the ordinary solve on a fresh context, as a
control, visibly allocates its workspace), reject a stored matvec and a
problem beyond the static array, and leave the context's own workspace
working.
"""
import numpy as np
import pytest
import torch

import oracle as O
from synth import make_config

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BAR = {0: 1e-11, 1: 1e-10}


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def ww():
    from paper_2108_01786_amd import wwbi
    return wwbi


def _inputs(ww, c):
    cfg = make_config(c)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    return cfg, dg, phi


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_solve_phi_two_calls(ww, prec):
    ctx = ww.Context(0)
    try:
        kw = dict(precision=prec, matvec=ww.MATVEC_ON_THE_FLY,
                  tol=1e-14 if prec == 1 else 1e-13)
        for c in (2, 1):                       # the second call is the smaller one
            cfg, dg, phi = _inputs(ww, c)
            say(f"noalloc: config {c} n={dg.n} precision={prec}")
            U = torch.empty(dg.M[0], dtype=torch.float64, device=DEV)
            om = torch.empty(dg.n, dtype=torch.float64, device=DEV)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info(0)[0]
            Un, omn, psin, repn = ctx.solve_phi_noalloc(dg, phi, U=U, omega=om, **kw)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info(0)[0]
            if c == 1:
                # every module is loaded by now: the call changes nothing
                assert abs(free1 - free0) < (1 << 20), (free0, free1)
            Ur, omr, psir, repr_ = ctx.solve_phi(dg, phi, **kw)
            say(f"  iters {repn.iters}/{repr_.iters} resid {repn.rel_resid:.2e}/"
                f"{repr_.rel_resid:.2e} U {rel(Un.cpu(), Ur.cpu()):.2e}")
            assert repn.status == repr_.status
            assert repn.iters == repr_.iters
            assert rel(Un.cpu(), Ur.cpu()) <= BAR[prec]
            assert rel(omn.cpu(), omr.cpu()) <= BAR[prec]
            if len(psir):
                assert np.abs(psin - psir).max() <= BAR[prec] * max(1.0, np.abs(psir).max())
            if c == 2:
                og = O.OGeom.from_synth(cfg["geom"])
                ref = O.solve_phi(og, torch.as_tensor(cfg["phi"]))
                e = rel(Un.cpu().numpy(), ref["U"].numpy())
                say(f"  U vs oracle {e:.2e}")
                assert e <= BAR[prec]
    finally:
        ctx.close()


def test_noalloc_control_and_limits(ww):
    # control: the ordinary solve on a fresh context allocates its workspace,
    # and the free-memory measure sees it
    cfg, dg, phi = _inputs(ww, 2)
    ctx = ww.Context(0)
    try:
        ctx.solve_phi_noalloc(dg, phi)          # loads every module
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(0)[0]
        ctx.solve_phi(dg, phi, matvec=ww.MATVEC_ON_THE_FLY)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(0)[0]
        say(f"control: ordinary solve took {(free0 - free1) / 2**20:.1f} MiB")
        assert free0 - free1 > (8 << 20)
        # a stored matvec is refused, outputs untouched
        U = torch.full((dg.M[0],), 7.0, dtype=torch.float64, device=DEV)
        with pytest.raises(ww.WWBIError) as e:
            ctx.solve_phi_noalloc(dg, phi, U=U, matvec=ww.MATVEC_STORED)
        assert e.value.status == ww.EINVAL_OPTS
        assert bool((U == 7.0).all())
        # the longest restart still fits at 4608 unknowns
        _, _, _, rep = ctx.solve_phi_noalloc(dg, phi, check=False, restart=256)
        assert rep.status == ww.OK
    finally:
        ctx.close()


def test_noalloc_rejects_beyond_scratch(ww):
    # the large cell (40960 unknowns) needs about 125 MB of workspace at
    # restart 100, beyond the 48 MiB array: rejected by the size check, which
    # precedes any device work
    cfg5 = make_config(5)
    dg = ww.DeviceGeometry.from_synth(cfg5["geom"], DEV)
    phi = torch.as_tensor(cfg5["phi"], device=DEV)
    ctx = ww.Context(0)
    try:
        U = torch.full((dg.M[0],), 7.0, dtype=torch.float64, device=DEV)
        with pytest.raises(ww.WWBIError) as e:
            ctx.solve_phi_noalloc(dg, phi, U=U)
        say(f"{dg.n} unknowns at restart 100: status {e.value.status}")
        assert e.value.status == ww.ESCRATCH
        assert bool((U == 7.0).all())
    finally:
        ctx.close()
