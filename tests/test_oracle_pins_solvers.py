"""Pins of the oracle's restarted GMRES, its chunked U map and its
tangent-linear model: the pieces that give the large cell (M = 40960) an
oracle reference where a dense solve with autograd is out of reach.

* the refined dense solve (LU plus one step of iterative refinement with an
  extended-precision residual) against the solution in 40-digit arithmetic,
  on a system ill-conditioned enough that LU alone is visibly off, and the refined residual of a seeded cell at
  the extended precision's level;
* GMRES against dense LU (a library routine) on a random well-conditioned
  nonsymmetric system and on the seeded cells of 640 and 4608 unknowns, and
  against the manufactured flow's closed-form U (Sec. 3.4);
* the chunked U map against the unchunked one;
* the tangent-linear derivative of J = sum w U^2 against Richardson-
  extrapolated central differences of the oracle's own forward solve (an
  independent check: only the forward map is shared), and against the
  reverse-mode autograd gradient of the same J.
"""
import numpy as np
import pytest
import torch

import oracle as O
from manufactured import manufactured_case
from synth import make_config, tiny_config


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def _solve_mp(A, b):
    """The solution of A x = b in 40-digit decimal arithmetic (mpmath's LU)."""
    import mpmath
    mpmath.mp.dps = 40
    x = mpmath.lu_solve(mpmath.matrix(A.tolist()), mpmath.matrix(b.tolist()))
    return np.array([float(v) for v in x])


def test_dense_solve_reaches_the_extended_precision_solution():
    """A = Q1 diag(s) Q2^T with singular values from 1 to 1e-5 (n = 60): LU
    alone is off by about cond * eps (9e-13); one refinement step with the
    residual in extended precision reaches the solution of the same FP64
    system computed in 40-digit arithmetic, to a few units of rounding."""
    rng = np.random.default_rng(21)
    n = 60
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q1 * np.logspace(0, -5, n)) @ Q2.T
    b = rng.standard_normal(n)
    ref = _solve_mp(A, b)
    lu = torch.linalg.solve(torch.as_tensor(A), torch.as_tensor(b)).numpy()
    x = O.dense_solve(torch.as_tensor(A), torch.as_tensor(b)).numpy()
    assert _rel(lu, ref) > 1e-13          # the case is one LU alone does not settle
    assert _rel(x, ref) < 1.5e-15
    # several right-hand sides at once, and the autograd path
    B = np.stack([b, rng.standard_normal(n)], axis=1)
    X = O.dense_solve(torch.as_tensor(A), torch.as_tensor(B)).numpy()
    assert _rel(X[:, 0], ref) < 1.5e-15
    At = torch.as_tensor(A).requires_grad_(True)
    xg = O.dense_solve(At, torch.as_tensor(b))
    assert _rel(xg.detach().numpy(), ref) < 1.5e-15
    (gA,) = torch.autograd.grad(xg.sum(), At)
    # d(sum x)/dA = -A^{-T} 1 x^T
    lam = np.linalg.solve(A.T, np.ones(n))
    assert _rel(gA.numpy(), -np.outer(lam, ref)) < 1e-8


def test_dense_solve_residual_on_seeded_cell():
    """Config 1 (640 unknowns): the refined omega leaves a residual, formed in
    extended precision, within a few units of rounding of |A| |omega|."""
    cfg = make_config(1)
    og = O.OGeom.from_synth(cfg["geom"])
    r = O.solve_phi(og, torch.as_tensor(cfg["phi"]))
    res = O.residual_ext(r["A"], r["b"], r["omega"]).numpy()
    scale = (np.abs(r["A"].numpy()) @ np.abs(r["omega"].numpy())).max()
    assert np.abs(res).max() <= 4e-16 * scale


def test_gmres_random_system_matches_lu():
    """A = 2 I + N(0, 1)/(4 sqrt n), n = 300, restart shorter than n: the
    restarted solve reaches the LU solution; its cycle history decreases."""
    rng = np.random.default_rng(11)
    n = 300
    A = torch.as_tensor(2.0 * np.eye(n) + rng.standard_normal((n, n)) / (4 * np.sqrt(n)))
    b = torch.as_tensor(rng.standard_normal(n))
    x, hist, steps = O.gmres(lambda v: A @ v, b, tol=1e-14, restart=15)
    ref = torch.linalg.solve(A, b)
    assert _rel(x, ref) < 1e-13
    assert hist[-1] <= 1e-14 and len(hist) > 2
    assert all(h1 < h0 for h0, h1 in zip(hist, hist[1:]))
    # a warm start at the solution returns at once
    x2, hist2, steps2 = O.gmres(lambda v: A @ v, b, tol=1e-13, restart=15, x0=ref)
    assert steps2 == 0 and hist2[0] <= 1e-13


@pytest.mark.parametrize("c", [1, 2])
def test_gmres_matches_lu_on_seeded_cells(c):
    """The velocity-potential system of the seeded cells (640 and 4608
    unknowns): GMRES to 1e-14 against dense LU, omega to 1e-12 and U to 1e-11."""
    cfg = make_config(c)
    og = O.OGeom.from_synth(cfg["geom"])
    ref = O.solve_phi(og, torch.as_tensor(cfg["phi"]))
    A = ref["A"]
    x, hist, steps = O.gmres(lambda v: A @ v, ref["b"], tol=1e-14, restart=60)
    assert hist[-1] <= 1e-14
    assert _rel(x, ref["omega"]) < 1e-12
    U = O.dphi_dn_from_omega_chunked(og, O.split(og, x), chunk=97)
    assert _rel(U, ref["U"]) < 1e-11


def test_gmres_manufactured_closed_form():
    """The manufactured periodic flow (exact U in closed form, Sec. 3.4):
    GMRES on the row-blocked matrix plus the chunked U map reach it as the
    dense path does."""
    geom, phi, U_exact, ck = manufactured_case(128, 128, 64)
    og = O.OGeom.from_synth(geom)
    A = O.assemble_A_blocked(og, chunk=50)
    b = O.rhs(og, torch.as_tensor(phi))
    x, hist, _ = O.gmres(lambda v: A @ v, b, tol=1e-14, restart=40)
    parts = O.split(og, x)
    U = O.dphi_dn_from_omega_chunked(og, parts, chunk=33).numpy()
    assert _rel(U, U_exact) < 1e-9
    psi = np.array([float(p.mean()) for p in parts[2:]])
    assert np.abs(psi - np.asarray(ck)).max() < 1e-10


def test_blocked_assembly_and_products():
    """Row-blocked assembly equals the full one to the last bit of the
    vectorised tan, A_times_blocked equals A x, and the chunked U map equals
    the unchunked one (same sums, grouped)."""
    cfg = make_config(1)
    og = O.OGeom.from_synth(cfg["geom"])
    A = O.assemble_A(og)
    Ab = O.assemble_A_blocked(og, chunk=77)
    assert float((A - Ab).abs().max()) <= 1e-18
    x = torch.as_tensor(np.random.default_rng(2).standard_normal(A.shape[0]))
    assert _rel(O.A_times_blocked(og, x, chunk=61), A @ x) < 1e-14
    om = O.split(og, torch.linalg.solve(A, O.rhs(og, torch.as_tensor(cfg["phi"]))))
    assert _rel(O.dphi_dn_from_omega_chunked(og, om, chunk=29), O.dphi_dn_from_omega(og, om)) < 1e-13


def _smooth_dirs(M, rng, n):
    al = 2 * np.pi * np.arange(M) / M
    k = np.arange(1, 9)
    ang = np.outer(al, k)

    def f():
        return (np.exp(-k / 3) * (rng.standard_normal(8) * np.cos(ang)
                                  + rng.standard_normal(8) * np.sin(ang))).sum(1)
    return [(f(), f(), f()) for _ in range(n)]


@pytest.mark.parametrize("name", ["tiny", "c1"])
def test_tangent_linear_model(name):
    """dJ along three smooth directions: Richardson-extrapolated central
    differences of the forward solve (h = 2e-4 and 1e-4, error O(h^4)) agree
    to 1e-9 relative; the reverse-mode gradient of the same J to 1e-12."""
    cfg = tiny_config() if name == "tiny" else make_config(1)
    geom = cfg["geom"]
    og = O.OGeom.from_synth(geom)
    M0 = geom.M[0]
    z0 = geom.curves[0].z
    al = 2 * np.pi * np.arange(M0) / M0
    xt, yt, ph = z0.real - al, z0.imag, np.asarray(cfg["phi"])
    rng = np.random.default_rng(3)
    w = rng.uniform(0, 1, M0)
    dirs = _smooth_dirs(M0, rng, 3)
    z, d, e = O.surface_from_periodic(torch.as_tensor(xt), torch.as_tensor(yt))
    A = O.assemble_A(og.with_surface(z, d, e))
    J, U, om, dJ, dU = O.tangent_J(og, xt, yt, ph, w, dirs, lambda r: torch.linalg.solve(A, r),
                                   chunk=90)
    Jr, gx, gy, gp, Ur = O.J_and_grad(og, xt, yt, ph, w)
    assert abs(J - Jr) <= 1e-14 * abs(Jr)

    def J_at(dx, dy, dp, s):
        z, d, e = O.surface_from_periodic(torch.as_tensor(xt + s * dx), torch.as_tensor(yt + s * dy))
        Us = O.solve_phi(og.with_surface(z, d, e), torch.as_tensor(ph + s * dp))["U"].numpy()
        return float((w * Us * Us).sum())

    for i, (dx, dy, dp) in enumerate(dirs):
        rev = float((gx.numpy() * dx).sum() + (gy.numpy() * dy).sum() + (gp.numpy() * dp).sum())
        cd = lambda h: (J_at(dx, dy, dp, h) - J_at(dx, dy, dp, -h)) / (2 * h)
        d1, d2 = cd(2e-4), cd(1e-4)
        rich = (4 * d2 - d1) / 3
        assert abs(dJ[i] - rich) <= 1e-9 * abs(rich), (i, dJ[i], rich)
        assert abs(dJ[i] - rev) <= 1e-12 * abs(rev), (i, dJ[i], rev)


def _smooth_dirs_nodes(M, rng, n):
    """Directions of the surface node data from degree-8 trig fields with their
    exact derivatives: (dx, dy, dx', dy', dx'', dy'', dphi)."""
    al = 2 * np.pi * np.arange(M) / M
    k = np.arange(1, 9)
    ang = np.outer(al, k)
    out = []
    for _ in range(n):
        comps = []
        for _c in range(3):
            a, b = rng.standard_normal(8), rng.standard_normal(8)
            wk = np.exp(-k / 3)
            f = (wk * (a * np.cos(ang) + b * np.sin(ang))).sum(1)
            f1 = (wk * k * (-a * np.sin(ang) + b * np.cos(ang))).sum(1)
            f2 = (wk * k * k * (-a * np.cos(ang) - b * np.sin(ang))).sum(1)
            comps.append((f, f1, f2))
        (x, x1, x2), (y, y1, y2), (p, _, _) = comps
        out.append((x, y, x1, y1, x2, y2, p))
    return out


def test_tangent_linear_model_on_node_data():
    """tangent_J_nodes (derivatives along the node data, directions with exact
    derivatives, surface as given) against tangent_J (derivatives along the
    periodic displacements, spectral derivatives) on the config-1 cell, whose
    surface is a trig polynomial of degree 16 so that both describe the same
    curve and the same directions to rounding; and against Richardson-
    extrapolated central differences of the forward solve on the node data."""
    cfg = make_config(1)
    geom = cfg["geom"]
    og = O.OGeom.from_synth(geom)
    M0 = geom.M[0]
    z0 = geom.curves[0].z
    al = 2 * np.pi * np.arange(M0) / M0
    xt, yt, ph = z0.real - al, z0.imag, np.asarray(cfg["phi"])
    rng = np.random.default_rng(5)
    w = rng.uniform(0, 1, M0)
    dn = _smooth_dirs_nodes(M0, rng, 2)
    A = O.assemble_A(og)
    solve = lambda r: torch.linalg.solve(A, r)
    J, U, om, dJ, _ = O.tangent_J_nodes(og, ph, w, dn, solve, chunk=111)
    Jp, _, _, dJp, _ = O.tangent_J(og, xt, yt, ph, w, [(d[0], d[1], d[6]) for d in dn], solve,
                                   chunk=111)
    assert abs(J - Jp) <= 1e-13 * abs(J)
    for a, b in zip(dJ, dJp):
        assert abs(a - b) <= 1e-11 * abs(b), (a, b)

    def J_at(d, s):
        gs = og.with_surface(torch.as_tensor(z0 + s * (d[0] + 1j * d[1])),
                             torch.as_tensor(geom.curves[0].d + s * (d[2] + 1j * d[3])),
                             torch.as_tensor(geom.curves[0].e + s * (d[4] + 1j * d[5])))
        Us = O.solve_phi(gs, torch.as_tensor(ph + s * d[6]))["U"].numpy()
        return float((w * Us * Us).sum())

    for i, d in enumerate(dn):
        cd = lambda h: (J_at(d, h) - J_at(d, -h)) / (2 * h)
        rich = (4 * cd(1e-4) - cd(2e-4)) / 3
        assert abs(dJ[i] - rich) <= 1e-9 * abs(rich), (i, dJ[i], rich)


def test_gradient_on_node_data():
    """J_and_grad_nodes (reverse mode along the node data) against J_and_grad
    (reverse mode along the periodic displacements) through the chain rule of
    the spectral surface, g_xt = g_x - D g_x' + D2 g_x'' (D antisymmetric, D2
    symmetric), and against the forward-mode tangent_J_nodes along two
    directions: the same J, reached through different code."""
    cfg = make_config(1)
    geom = cfg["geom"]
    og = O.OGeom.from_synth(geom)
    M0 = geom.M[0]
    z0 = geom.curves[0].z
    al = 2 * np.pi * np.arange(M0) / M0
    xt, yt, ph = z0.real - al, z0.imag, np.asarray(cfg["phi"])
    rng = np.random.default_rng(6)
    w = rng.uniform(0, 1, M0)
    J, gr, U = O.J_and_grad_nodes(og, ph, w)
    Jp, gx, gy, gp, _ = O.J_and_grad(og, xt, yt, ph, w)
    assert abs(J - Jp) <= 1e-13 * abs(J)
    cx = gr[0] - O.spectral(gr[2], "D") + O.spectral(gr[4], "D2")
    cy = gr[1] - O.spectral(gr[3], "D") + O.spectral(gr[5], "D2")
    for a, b in ((cx, gx), (cy, gy), (gr[6], gp)):
        assert _rel(a.numpy(), b.numpy()) < 1e-11
    dn = _smooth_dirs_nodes(M0, rng, 2)
    A = O.assemble_A(og)
    _, _, _, dJ, _ = O.tangent_J_nodes(og, ph, w, dn, lambda r: torch.linalg.solve(A, r))
    for i, d in enumerate(dn):
        rev = sum(float((g.numpy() * np.asarray(v)).sum()) for g, v in zip(gr, d))
        assert abs(rev - dJ[i]) <= 1e-12 * abs(dJ[i]), (i, rev, dJ[i])
