"""Parity on the headline cell (M = 10240: surface 4096, flat bottom 2048, four
ellipses of 1024) in the options the throughput bench times: every output
element against the oracle's refined dense solve of the same seeded inputs.

Bars: 1e-10 relative (max norm) for refined FP32 and 1e-11 for FP64, the
accuracy the method is asked to reach at this size.  The refined solve runs
both with the first inner solve's Krylov space recycled into the later ones
(the default) and without: same FP64 stopping test, fewer Arnoldi steps."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import make_config

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


@pytest.fixture(scope="module")
def cell():
    cfg = make_config(3)
    og = O.OGeom.from_synth(cfg["geom"])
    ref = O.solve_phi(og, torch.as_tensor(cfg["phi"]))
    return cfg, og, {k: v.numpy() for k, v in ref.items()}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def _opts(ww, prec, mode):
    mv = ww.MATVEC_STORED if mode == "stored" else ww.MATVEC_ON_THE_FLY
    if prec in ("refined", "refined-norecycle"):
        return dict(precision=ww.FP32_REFINED, tol=1e-14, inner_tol=1e-7, matvec=mv, restart=100,
                    poll_every=2, flags=ww.FLAG_NO_RECYCLE if prec == "refined-norecycle" else 0)
    return dict(precision=ww.FP64, tol=1e-13, matvec=mv, restart=100, poll_every=2)


@pytest.mark.parametrize("prec,mode", [("refined", "stored"), ("fp64", "stored"),
                                       ("refined", "otf"), ("refined-norecycle", "stored")])
def test_headline_cell_matches_oracle(ww, ctx, cell, prec, mode):
    say(f"case headline M=10240 {prec} {mode}")
    cfg, _, ref = cell
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    U, omega, psi, rep = ctx.solve_phi(dg, torch.as_tensor(cfg["phi"], device=DEV),
                                       **_opts(ww, prec, mode))
    bar = 1e-11 if prec == "fp64" else 1e-10
    errs = {"U": rel(U.cpu().numpy(), ref["U"]), "omega": rel(omega.cpu().numpy(), ref["omega"]),
            "psi": rel(np.asarray(psi), ref["psi_k"])}
    say("  " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()) +
        f"  iters {rep.iters} refine {rep.refine_steps} status {rep.status}")
    assert rep.status == 0
    for k, v in errs.items():
        assert v <= bar, (k, v)


def test_headline_cell_multi_rhs(ww, ctx, cell):
    """32 right-hand sides at full size (refined FP32, matrix-core products and
    stored FP64 residuals) against the oracle matrix's dense LU."""
    say("case headline M=10240 multi nr=32 refined")
    cfg, og, _ = cell
    n = cfg["geom"].Mtot
    rhs = np.random.default_rng(32).standard_normal((32, n))
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    out, rep = ctx.solve_phi_multi(dg, torch.as_tensor(rhs, device=DEV), precision=ww.FP32_REFINED,
                                   tol=1e-14, restart=100)
    assert rep.status == 0
    ref = torch.linalg.solve(O.assemble_A(og), torch.as_tensor(rhs).T).T.numpy()
    err = rel(out.cpu().numpy(), ref)
    say(f"  iters {rep.iters} refine {rep.refine_steps} err {err:.1e}")
    assert err <= 1e-11
