"""GPU path (HIP library through the C ABI) against the FP64 CPU oracle.

Error measure: relative max-norm error ||x_gpu - x_ref||_inf / ||x_ref||_inf per
output.  Bars: 1e-11 for FP64 solves, 1e-10 for refined FP32 solves.  FP64
GMRES runs to a relative residual of 1e-13 (cond_2(A) is a few units, so
omega is accurate to about 1e-12 and its error is smooth).  U applies a
spectral derivative to omega, which amplifies the high modes of the solution
error by up to M_0/2.  The last FP32 correction of the refinement carries
white noise of about 1e-7 of its size, so the refined solves run to 1e-14:
the final, short step then leaves noise far below the bar on U.
"""
import contextlib

import numpy as np
import pytest
import torch

import oracle as O
from manufactured import manufactured_case
from synth import make_config, ragged_config, tiny_config
from tails import check_tail_status, oracle_tail

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


def _cfg(name):
    if name == "c1":
        return make_config(1)
    if name == "c2":
        return make_config(2)
    if name == "ragged":
        return ragged_config()
    if name == "tiny":
        t = tiny_config()
        return {"geom": t["geom"], "phi": t["phi"]}
    raise KeyError(name)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


_ORACLE_CACHE = {}


def oracle_solution(name):
    if name not in _ORACLE_CACHE:
        cfg = _cfg(name)
        g = O.OGeom.from_synth(cfg["geom"])
        _ORACLE_CACHE[name] = O.solve_phi(g, torch.as_tensor(cfg["phi"]))
    return _ORACLE_CACHE[name]


@pytest.mark.parametrize("name", ["tiny", "ragged", "c1"])
def test_matrix_fp64_entrywise(ww, ctx, name):
    say(f"case matrix_fp64 {name}")
    cfg = _cfg(name)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    A = ctx.debug_matrix(dg, ww.MAT_A, ww.FP64).cpu().numpy()
    Ar = oracle_solution(name)["A"].numpy()
    assert np.abs(A - Ar).max() <= 1e-13, np.abs(A - Ar).max()


# tiny: every boundary fits inside the FP64 band (M <= 2 band + 1); ragged:
# tiles and waves that straddle boundary ends; c2: tiles on one boundary each,
# where the assembly takes its uniform fast entries
@pytest.mark.parametrize("name", ["tiny", "ragged", "c1", "c2"])
def test_matrix_fp32_band_and_offband(ww, ctx, name):
    say(f"case matrix_fp32 {name}")
    cfg = _cfg(name)
    geom = cfg["geom"]
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    band = 16
    A = ctx.debug_matrix(dg, ww.MAT_A, ww.FP32_REFINED, band).cpu().numpy().astype(np.float64)
    Ar = oracle_solution(name)["A"].numpy()
    # same-boundary pairs within the band are FP64 values rounded once to FP32
    n = geom.Mtot
    bid = np.concatenate([np.full(m, k) for k, m in enumerate(geom.M)])
    loc = np.concatenate([np.arange(m) for m in geom.M])
    Mk = np.concatenate([np.full(m, m) for m in geom.M])
    d = np.abs(loc[:, None] - loc[None, :])
    d = np.minimum(d, Mk[:, None] - d)
    inband = (bid[:, None] == bid[None, :]) & (d <= band)
    r32 = Ar.astype(np.float32).astype(np.float64)
    assert np.abs(A[inband] - r32[inband]).max() <= 2 * np.finfo(np.float32).eps * np.abs(Ar).max()
    # elsewhere FP32 evaluation of the kernel: a few FP32 ulps of the local scale
    err = np.abs(A - Ar)[~inband]
    assert err.max() <= 1e-6 * np.abs(Ar).max(), err.max()


# c2 has target blocks and source tiles inside single boundaries, so the
# on-the-fly products take their specialised far tiles there
@pytest.mark.parametrize("name", ["ragged", "c1", "c2"])
@pytest.mark.parametrize("mode", ["stored", "otf"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("transpose", [False, True])
def test_matvec(ww, ctx, name, mode, prec, transpose):
    say(f"case matvec {name} {mode} {prec} T={transpose}")
    cfg = _cfg(name)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    n = dg.n
    x = np.random.default_rng(11).standard_normal(n)
    y, _ = ctx.matvec(dg, torch.as_tensor(x, device=DEV),
                      precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED,
                      mode=ww.MATVEC_STORED if mode == "stored" else ww.MATVEC_ON_THE_FLY,
                      transpose=transpose)
    Ar = oracle_solution(name)["A"].numpy()
    ref = (Ar.T if transpose else Ar) @ x
    tol = 1e-13 if prec == "fp64" else 3e-6
    assert rel(y.cpu().numpy(), ref) <= tol


@pytest.mark.parametrize("name", ["tiny", "ragged", "c1", "c2"])
@pytest.mark.parametrize("mode", ["stored", "otf"])
def test_solve_phi_fp64(ww, ctx, name, mode):
    say(f"case solve_phi_fp64 {name} {mode}")
    cfg = _cfg(name)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    U, omega, psi, rep = ctx.solve_phi(
        dg, torch.as_tensor(cfg["phi"], device=DEV), tol=1e-13,
        matvec=ww.MATVEC_STORED if mode == "stored" else ww.MATVEC_ON_THE_FLY)
    ref = oracle_solution(name)
    assert rep.rel_resid <= 1e-13
    check_tail_status(ww, rep, 1e-13, oracle_tail(cfg["geom"], ref["omega"].numpy()))
    assert rel(U.cpu().numpy(), ref["U"].numpy()) <= 1e-11
    assert rel(omega.cpu().numpy(), ref["omega"].numpy()) <= 1e-11
    if cfg["geom"].nb > 2:
        assert rel(psi, ref["psi_k"].numpy()) <= 1e-11


@pytest.mark.parametrize("name", ["ragged", "c1", "c2"])
@pytest.mark.parametrize("mode", ["stored", "otf"])
def test_solve_phi_refined_fp32(ww, ctx, name, mode):
    say(f"case solve_phi_refined {name} {mode}")
    cfg = _cfg(name)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    U, omega, psi, rep = ctx.solve_phi(
        dg, torch.as_tensor(cfg["phi"], device=DEV), tol=1e-14, precision=ww.FP32_REFINED,
        matvec=ww.MATVEC_STORED if mode == "stored" else ww.MATVEC_ON_THE_FLY)
    ref = oracle_solution(name)
    say(f"  iters={rep.iters} refine={rep.refine_steps} resid={rep.rel_resid:.2e}")
    assert rep.rel_resid <= 1e-14
    check_tail_status(ww, rep, 1e-14, oracle_tail(cfg["geom"], ref["omega"].numpy()))
    assert rel(U.cpu().numpy(), ref["U"].numpy()) <= 1e-10
    assert rel(omega.cpu().numpy(), ref["omega"].numpy()) <= 1e-10


@pytest.mark.parametrize("name", ["ragged", "c1"])
def test_solve_gamma(ww, ctx, name):
    say(f"case solve_gamma {name}")
    cfg = _cfg(name)
    g = O.OGeom.from_synth(cfg["geom"])
    ref_vp = oracle_solution(name)
    gamma0 = -O.spectral(O.split(g, ref_vp["omega"])[0], "D")
    ref = O.solve_gamma(g, gamma0)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    for mode, prec in ((ww.MATVEC_STORED, ww.FP64), (ww.MATVEC_ON_THE_FLY, ww.FP64),
                       (ww.MATVEC_STORED, ww.FP32_REFINED)):
        refined = prec == ww.FP32_REFINED
        U, gw, rep = ctx.solve_gamma(dg, torch.as_tensor(gamma0.numpy(), device=DEV),
                                     tol=1e-14 if refined else 1e-13, matvec=mode, precision=prec)
        assert rep.status == 0 and (rep.refine_steps > 0) == refined
        bar = 1e-10 if refined else 1e-11
        assert rel(U.cpu().numpy(), ref["U"].numpy()) <= bar
        assert rel(gw.cpu().numpy(), ref["gamma_wall"].numpy()) <= bar
        # vortex-sheet U equals the velocity-potential U (Sec. 4.1 vs Sec. 3.4)
        assert rel(U.cpu().numpy(), ref_vp["U"].numpy()) <= bar


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_gamma_warm_start(ww, ctx, prec):
    """x0 = the converged wall strengths: the vortex-sheet solve stops at once
    with the same U; x0 from a nearby gamma_0 takes fewer steps to the same
    answer, in FP64 and in refined FP32."""
    say(f"case solve_gamma warm start {prec}")
    cfg = _cfg("c1")
    g = O.OGeom.from_synth(cfg["geom"])
    gamma0 = -O.spectral(O.split(g, oracle_solution("c1")["omega"])[0], "D").numpy()
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    kw = dict(tol=1e-13 if prec == "fp64" else 1e-14,
              precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED)
    g0 = torch.as_tensor(gamma0, device=DEV)
    U0, gw0, r0 = ctx.solve_gamma(dg, g0, **kw)
    U1, gw1, r1 = ctx.solve_gamma(dg, g0, x0=gw0.clone(), **kw)
    assert r1.status == 0 and r1.iters == 0
    assert rel(U1.cpu().numpy(), U0.cpu().numpy()) <= 1e-13
    U2, _, r2 = ctx.solve_gamma(dg, g0 * 1.001, x0=gw0.clone(), **kw)
    U3, _, r3 = ctx.solve_gamma(dg, g0 * 1.001, **kw)
    say(f"  cold iters {r3.iters} warm iters {r2.iters}")
    assert r2.status == 0 and r2.iters < r3.iters
    assert rel(U2.cpu().numpy(), U3.cpu().numpy()) <= 1e-11


def test_wall_matrix_entrywise(ww, ctx):
    say("case wall_matrix ragged")
    cfg = _cfg("ragged")
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    W = ctx.debug_matrix(dg, ww.MAT_WALL, ww.FP64).cpu().numpy()
    Wr = O.wall_matrix(O.OGeom.from_synth(cfg["geom"])).numpy()
    assert np.abs(W - Wr).max() <= 1e-13


@pytest.mark.parametrize("n", [8, 64, 250, 1024])
@pytest.mark.parametrize("op", ["D", "D2", "H", "ABSD"])
def test_spectral(ww, ctx, n, op):
    say(f"case spectral {op} {n}")
    f = np.random.default_rng(n).standard_normal(n)
    code = {"D": ww.OP_D, "D2": ww.OP_D2, "H": ww.OP_H, "ABSD": ww.OP_ABSD}[op]
    out = ctx.spectral(torch.as_tensor(f, device=DEV), code).cpu().numpy()
    ref = O.spectral(torch.as_tensor(f), op).numpy()
    scale = {"D": n, "D2": n * n, "H": 1, "ABSD": n}[op]
    assert np.abs(out - ref).max() <= 1e-12 * scale * np.abs(f).max()


def test_manufactured_flow_on_gpu(ww, ctx):
    say("case manufactured 256/256/128")
    geom, phi, U_exact, ck = manufactured_case(256, 256, 128)
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    U, _, psi, rep = ctx.solve_phi(dg, torch.as_tensor(phi, device=DEV), tol=1e-13)
    assert rel(U.cpu().numpy(), U_exact) <= 1e-12
    assert np.abs(psi - ck).max() <= 1e-12


def test_errors_are_reported(ww, ctx):
    say("case errors")
    cfg = make_config(1)
    geom = cfg["geom"]
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    # NaN in the node data
    bad = ww.DeviceGeometry.from_synth(geom, DEV)
    bad.x[5] = float("nan")
    U = torch.full((geom.M[0],), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(ww.WWBIError) as e:
        ctx.solve_phi(bad, phi, U=U)
    assert e.value.status == ww.EINVAL_NONFINITE
    assert bool((U == 7.0).all())            # outputs untouched on invalid input
    # NaN in the potential
    phibad = phi.clone()
    phibad[3] = float("inf")
    with pytest.raises(ww.WWBIError) as e:
        ctx.solve_phi(dg, phibad)
    assert e.value.status == ww.EINVAL_NONFINITE
    # counter-clockwise obstacle
    from synth.geometry import ellipse
    import copy
    g2 = copy.deepcopy(geom)
    g2.curves[2] = ellipse(128, np.pi, -0.5, 0.3, 0.15, 0.0, clockwise=False)
    with pytest.raises(ww.WWBIError) as e:
        ctx.solve_phi(ww.DeviceGeometry.from_synth(g2, DEV), phi)
    assert e.value.status == ww.EINVAL_ORIENTATION
    # odd node count
    odd = ww.DeviceGeometry(geom.M[:1] + [geom.M[1] - 1] + geom.M[2:], dg.x[:-1], dg.y[:-1],
                            dg.dx[:-1], dg.dy[:-1], dg.ddx[:-1], dg.ddy[:-1], geom.zc, geom.a, 1.0,
                            device=DEV)
    with pytest.raises(ww.WWBIError) as e:
        ctx.solve_phi(odd, phi)
    assert e.value.status == ww.EINVAL_SIZE
    # iteration budget too small: warning status with the best iterate
    U, om, _, rep = ctx.solve_phi(dg, phi, max_iter=1, restart=1, check=False)
    assert rep.status == ww.NOT_CONVERGED and rep.iters == 1
    assert np.isfinite(U.cpu().numpy()).all()
    # dropping the rank-one correction makes A singular: GMRES must not report success
    U, om, _, rep = ctx.solve_phi(dg, phi, flags=ww.FLAG_NO_CORRECTION, restart=20, max_iter=200,
                                  check=False)
    assert rep.status in (ww.STAGNATED, ww.NOT_CONVERGED)


def test_deterministic(ww, ctx):
    say("case determinism c1")
    cfg = make_config(1)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    a = ctx.solve_phi(dg, phi, precision=ww.FP32_REFINED)[0].cpu().numpy()
    b = ctx.solve_phi(dg, phi, precision=ww.FP32_REFINED)[0].cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("h", [1.0, 3.0])
def test_flat_strip_closed_form(ww, ctx, prec, h):
    """No obstacles, flat bottom at depth h, phi~ = cos(k alpha): the device U
    is the finite-depth Dirichlet-Neumann operator k tanh(k h) cos(k alpha)
    (Sec. 3 with N = 1), on both precision paths and both matvec modes; the
    ragged surface/bottom sizes give tiles with tails."""
    say(f"case flat strip h={h} {prec}")
    from manufactured import flat_strip
    geom = flat_strip(200, 136, h, 1.0)
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    al = 2 * np.pi * np.arange(200) / 200
    kw = dict(tol=1e-13 if prec == "fp64" else 1e-14,
              precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED)
    for k in (1, 3, 7):
        phi = torch.as_tensor(np.cos(k * al), device=DEV)
        for mode in (ww.MATVEC_STORED, ww.MATVEC_ON_THE_FLY):
            U, _, _, rep = ctx.solve_phi(dg, phi, matvec=mode, **kw)
            err = np.abs(U.cpu().numpy() - k * np.tanh(k * h) * np.cos(k * al)).max()
            assert rep.status == 0 and err <= (1e-12 if prec == "fp64" else 1e-11) * k, (k, err)


def test_node_height_range(ww, ctx):
    """Far pairs use E = e^{i zeta} with FP32 intermediate steps, so nodes must
    keep |y| <= 30: a bottom at depth 29 solves (U = k tanh(29 k) cos(k alpha),
    both precisions), one at depth 31 is rejected with the outputs untouched."""
    say("case node height range")
    from manufactured import flat_strip
    al = 2 * np.pi * np.arange(64) / 64
    phi = torch.as_tensor(np.cos(3 * al), device=DEV)
    dg = ww.DeviceGeometry.from_synth(flat_strip(64, 48, 29.0, 0.0), DEV)
    for prec, tol in ((ww.FP64, 1e-13), (ww.FP32_REFINED, 1e-14)):
        U, _, _, rep = ctx.solve_phi(dg, phi, precision=prec, tol=tol)
        assert rep.status == 0
        assert np.abs(U.cpu().numpy() - 3 * np.tanh(87.0) * np.cos(3 * al)).max() <= 1e-11
    deep = ww.DeviceGeometry.from_synth(flat_strip(64, 48, 31.0, 0.0), DEV)
    U = torch.full((64,), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(ww.WWBIError) as e:
        ctx.solve_phi(deep, phi, U=U)
    assert e.value.status == ww.EINVAL_RANGE
    assert bool((U == 7.0).all())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_right_hand_side(ww, ctx, prec):
    """b = 0 (flat strip, phi~ = 0, V1 = 0, no obstacles): omega = 0 and U = 0
    exactly, on both precision paths (the cold start writes x without a fill)."""
    say(f"case zero rhs {prec}")
    from manufactured import flat_strip
    geom = flat_strip(64, 64, 1.0, 0.0)
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    phi = torch.zeros(64, dtype=torch.float64, device=DEV)
    U, om, _, rep = ctx.solve_phi(dg, phi, tol=1e-13 if prec == "fp64" else 1e-14,
                                  precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED)
    assert rep.status == 0
    assert float(om.abs().max()) == 0.0 and float(U.abs().max()) == 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_warm_start(ww, ctx, prec):
    """x0 = the converged omega: the solve stops at once with the same result;
    x0 = omega of a nearby state converges in fewer steps to the same answer."""
    say(f"case warm start {prec}")
    cfg = make_config(1)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    kw = dict(tol=1e-13 if prec == "fp64" else 1e-14,
              precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED)
    U0, om0, _, r0 = ctx.solve_phi(dg, phi, **kw)
    U1, om1, _, r1 = ctx.solve_phi(dg, phi, x0=om0.clone(), **kw)
    assert r1.iters == 0 and torch.equal(om1, om0)
    U2, om2, _, r2 = ctx.solve_phi(dg, phi * 1.001, x0=om0.clone(), **kw)
    U3, om3, _, r3 = ctx.solve_phi(dg, phi * 1.001, **kw)
    say(f"  cold iters {r3.iters} warm iters {r2.iters}")
    assert r2.iters < r3.iters
    assert float((U2 - U3).abs().max() / U3.abs().max()) <= 1e-11


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_poll_interval_does_not_change_results(ww, ctx, prec):
    """The host only learns where a GMRES cycle ends (from the state the ending
    kernel publishes); steps enqueued past the end do nothing.  So any polling
    interval gives the same steps and bitwise the same solution, also when the
    restart length cuts cycles short (several cycles per solve)."""
    say(f"case poll interval {prec}")
    cfg = make_config(1)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    for restart in (100, 7 if prec == "fp64" else 10):
        kw = dict(tol=1e-13 if prec == "fp64" else 1e-14, restart=restart, max_refine=30,
                  precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED)
        runs = [ctx.solve_phi(dg, phi, poll_every=p, **kw) for p in (1, 2, 3, 8, 50)]
        U0, om0, _, r0 = runs[0]
        assert r0.status == 0
        say(f"  restart {restart}: iters {r0.iters} cycles {r0.restarts}")
        for U, om, _, r in runs[1:]:
            assert r.status == 0 and r.iters == r0.iters and r.restarts == r0.restarts
            assert torch.equal(om, om0) and torch.equal(U, U0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_back_substitution_forms_agree(ww, ctx, prec):
    """A cycle's triangle is solved from LDS by one wave while it fits 60 KB
    (restart <= 123) and from global memory beyond.  Both forms take the same
    operations in the same order, so solves that end within their first
    cycle give bitwise the same result at restart 123, 124 and 256."""
    say(f"case back substitution forms {prec}")
    cfg = make_config(1)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    kw = dict(tol=1e-13 if prec == "fp64" else 1e-14,
              precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED)
    U0, om0, _, r0 = ctx.solve_phi(dg, phi, restart=123, **kw)
    assert r0.status == 0 and r0.iters < 123    # one cycle per (inner) solve
    for restart in (124, 256):
        U, om, _, r = ctx.solve_phi(dg, phi, restart=restart, **kw)
        say(f"  restart {restart}: iters {r.iters} (123: {r0.iters})")
        assert r.status == 0 and r.iters == r0.iters
        assert torch.equal(om, om0) and torch.equal(U, U0)


@pytest.mark.parametrize("gap", [0.3, 0.03, 0.01])
def test_underresolved_warning(ww, ctx, gap):
    """An ellipse `gap` below the flat surface (256/256/128 nodes): far away its
    omega is resolved and the solve reports OK; close to the surface both
    curves' omega keep energy near Nyquist and the solve reports
    WARN_UNDERRESOLVED (a RuntimeWarning from the binding), with the tail
    ratio of the oracle's FFT measure and the outputs still at parity.  The
    solve runs to the paper's 1e-15 (Sec. 7.4): U applies D to an omega with
    energy near Nyquist, which amplifies what a looser GMRES tolerance leaves
    in omega to about the 1e-11 bar."""
    say(f"case under-resolved gap {gap}")
    from synth.geometry import Geometry, ellipse, fourier_surface, graph_bottom
    b = 0.15
    geom = Geometry([fourier_surface(256, 0.0, []), graph_bottom(256, -1.0),
                     ellipse(128, np.pi, -gap - b, 0.3, b, 0.0)],
                    np.array([np.pi - (gap + b) * 1j]), np.array([0.5]), 1.0)
    phi = 0.1 * np.cos(np.arange(256) * 2 * np.pi / 256)
    ref = O.solve_phi(O.OGeom.from_synth(geom), torch.as_tensor(phi))
    t_ref = oracle_tail(geom, ref["omega"].numpy())
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    with pytest.warns(RuntimeWarning) if gap < 0.1 else contextlib.nullcontext():
        U, om, _, rep = ctx.solve_phi(dg, torch.as_tensor(phi, device=DEV), tol=1e-15)
    eU = rel(U.cpu().numpy(), ref["U"].numpy())
    say(f"  tail ratio {rep.tail_ratio:.2e} oracle {t_ref:.2e} status {rep.status}  U {eU:.2e}")
    check_tail_status(ww, rep, 1e-15, t_ref)
    assert (rep.status == ww.WARN_UNDERRESOLVED) == (gap < 0.1)
    assert eU <= 1e-11


@pytest.mark.parametrize("name", ["tiny", "ragged", "c1"])
def test_T_matrix_entrywise(ww, ctx, name):
    """The normal-velocity map T of Sec. 3.4 (s U = u_mv + H gamma_0 / 2 +
    T gamma, gamma_0 = -D omega_0, gamma_j = D omega_j): the transposed G_00
    block over M_0 on the surface columns and the transposed K_j0 blocks over
    M_j on wall j, entrywise."""
    say(f"case T matrix {name}")
    cfg = _cfg(name)
    geom = cfg["geom"]
    g = O.OGeom.from_synth(geom)
    cols = [O.G_block(g, 0, 0).T / geom.M[0]]
    cols += [O.K_block(g, j, 0).T / geom.M[j] for j in range(1, geom.nb)]
    Tr = torch.cat(cols, dim=1).numpy()
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    T = ctx.debug_matrix(dg, ww.MAT_T, ww.FP64).cpu().numpy()
    assert T.shape == Tr.shape
    assert np.abs(T - Tr).max() <= 1e-13, np.abs(T - Tr).max()
    # T v for a seeded v against the oracle's product
    v = np.random.default_rng(3).standard_normal(geom.Mtot)
    assert rel(T @ v, Tr @ v) <= 1e-13


def test_report_residual_history(ww, ctx):
    """report.resid_hist: the true residual at every cycle start of an FP64
    solve (restart 7: several cycles, decreasing, the last the reported
    rel_resid) and the FP64 residual after every refinement step."""
    say("case report residual history")
    cfg = make_config(1)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    _, _, _, rep = ctx.solve_phi(dg, phi, tol=1e-13, restart=7)
    h = rep.history()
    say(f"  fp64 restarts {rep.restarts}: {['%.1e' % v for v in h]}")
    assert rep.status == 0 and len(h) == min(32, rep.restarts + 1)
    assert h[0] == 1.0 and h[-1] == rep.rel_resid and h[-1] <= 1e-13
    assert all(b < a for a, b in zip(h, h[1:]))
    _, _, _, rep = ctx.solve_phi(dg, phi, tol=1e-14, precision=ww.FP32_REFINED)
    h = rep.history()
    say(f"  refined steps {rep.refine_steps}: {['%.1e' % v for v in h]}")
    assert rep.status == 0 and len(h) == rep.refine_steps
    assert h[-1] == rep.rel_resid and h[-1] <= 1e-14
    assert all(b < a for a, b in zip(h, h[1:]))
