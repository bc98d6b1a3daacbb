"""Pins of the oracle's restarted GMRES, its chunked U map and its
tangent-linear model: the pieces that give the large cell (M = 40960) an
oracle reference where a dense solve with autograd is out of reach.

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
