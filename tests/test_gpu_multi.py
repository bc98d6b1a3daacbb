"""Several right-hand sides against one matrix (matrix-core product, batched
GMRES in lockstep) against dense LU of the oracle's matrix."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import make_config, ragged_config

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ww():
    from paper_2108_01786_amd import wwbi
    return wwbi


@pytest.fixture(scope="module")
def ctx(ww):
    c = ww.Context(0)
    yield c
    c.close()


_A = {}


def oracle_A(name, geom):
    if name not in _A:
        _A[name] = O.assemble_A(O.OGeom.from_synth(geom))
    return _A[name]


@pytest.mark.parametrize("name,nr,prec", [("ragged", 5, "fp64"), ("ragged", 17, "fp32"),
                                          ("c1", 20, "fp64"), ("c1", 32, "fp64"),
                                          ("c1", 7, "fp32"), ("c2", 16, "fp32"),
                                          ("c2", 32, "fp32"), ("c2", 4, "fp64")])
def test_multi_rhs_matches_dense_lu(ww, ctx, name, nr, prec):
    say(f"case multi {name} nr={nr} {prec}")
    cfg = ragged_config() if name == "ragged" else make_config(int(name[1]))
    geom = cfg["geom"]
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    n = geom.Mtot
    rhs = np.random.default_rng(nr).standard_normal((nr, n))
    tol = 1e-13 if prec == "fp64" else 1e-14
    out, rep = ctx.solve_phi_multi(dg, torch.as_tensor(rhs, device=DEV), tol=tol,
                                   precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED)
    assert rep.status == 0 and rep.rel_resid <= tol
    ref = torch.linalg.solve(oracle_A(name, geom), torch.as_tensor(rhs).T).T.numpy()
    err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
    say(f"  iters={rep.iters} refine={rep.refine_steps} err={err:.2e}")
    assert err <= 1e-11


def test_multi_equals_single_solves(ww, ctx):
    """Column s of the multi solve equals the single solve with b = rhs_s."""
    say("case multi vs single c1")
    cfg = make_config(1)
    geom = cfg["geom"]
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    og = O.OGeom.from_synth(geom)
    b = O.rhs(og, torch.as_tensor(cfg["phi"])).numpy()
    rhs = np.stack([b, 2 * b, -b])
    out, rep = ctx.solve_phi_multi(dg, torch.as_tensor(rhs, device=DEV), tol=1e-13)
    _, omega, _, _ = ctx.solve_phi(dg, torch.as_tensor(cfg["phi"], device=DEV), tol=1e-13)
    om = omega.cpu().numpy()
    o = out.cpu().numpy()
    for s, f in enumerate((1.0, 2.0, -1.0)):
        assert np.abs(o[s] - f * om).max() <= 1e-11 * np.abs(om).max()


def test_multi_errors(ww, ctx):
    """Invalid calls are rejected before any output is written."""
    say("case multi errors")
    cfg = make_config(1)
    geom = cfg["geom"]
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    n = geom.Mtot
    rhs = torch.as_tensor(np.random.default_rng(3).standard_normal((3, n)), device=DEV)
    for kw in (dict(matvec=ww.MATVEC_ON_THE_FLY), dict(x0=torch.zeros(n, dtype=torch.float64, device=DEV))):
        with pytest.raises(ww.WWBIError) as e:
            ctx.solve_phi_multi(dg, rhs, **kw)
        assert e.value.status == ww.EINVAL_OPTS
    with pytest.raises(ww.WWBIError) as e:
        ctx.solve_phi_multi(dg, torch.zeros((33, n), dtype=torch.float64, device=DEV))
    assert e.value.status == ww.EINVAL_OPTS
    bad = rhs.clone()
    bad[2, n - 1] = float("nan")
    with pytest.raises(ww.WWBIError) as e:
        ctx.solve_phi_multi(dg, bad)
    assert e.value.status == ww.EINVAL_NONFINITE
    # a valid call after the rejected ones still solves
    out, rep = ctx.solve_phi_multi(dg, rhs, tol=1e-13)
    assert rep.status == 0 and torch.isfinite(out).all()
