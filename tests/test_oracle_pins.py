"""Pins of the FP64 CPU oracle to values the paper and the mathematics fix.

Each pin is chosen so that a plausible slip in the oracle (a wrong sign on a
G block, a dropped E_m correction, a transposed kernel block in U, a wrong
Hilbert or Nyquist convention, a wrong diagonal limit) fails at least one
of them.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
from manufactured import (CASE_FLOW, Flow, exact_dphi_ds, flat_strip, manufactured_case,
                          manufactured_inputs)
from synth import make_config, paper_problem, ragged_config, tiny_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_energy():
    out = {}
    with open(os.path.join(GOLDEN, "energy_problems_1_3.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                n, e = line.split()
                out[int(n)] = float(e)
    return out


@pytest.mark.parametrize("problem", [1, 2, 3])
def test_energy_matches_printed_E0(problem):
    """E(0) of problems 1-3 (Sec. 7.3 table; geometry Sec. 7.1) to the 5 printed decimals."""
    ref = _golden_energy()[problem]
    cfg = paper_problem(problem)
    g = O.OGeom.from_synth(cfg["geom"])
    phi = torch.as_tensor(cfg["phi"])
    r = O.solve_phi(g, phi)
    E = O.energy(g, phi, r["omega"], cfg["tau"], cfg["g"])
    assert abs(E - ref) <= 6e-6, (E, ref)


def test_energy_resolution_independent():
    """The same E(0) at doubled resolution (the discretization is converged)."""
    cfg1, cfg2 = paper_problem(3), paper_problem(3, 512, 192, 256)
    Es = []
    for cfg in (cfg1, cfg2):
        g = O.OGeom.from_synth(cfg["geom"])
        phi = torch.as_tensor(cfg["phi"])
        Es.append(O.energy(g, phi, O.solve_phi(g, phi)["omega"], 0.1))
    assert abs(Es[0] - Es[1]) < 1e-9


@pytest.mark.parametrize("h", [1.0, 3.0])
@pytest.mark.parametrize("k", [1, 3, 7])
@pytest.mark.parametrize("V1", [0.0, 1.0])
def test_flat_strip_dno(h, k, V1):
    """No obstacles, flat bottom at depth h: U = k tanh(k h) cos(k alpha)."""
    geom = flat_strip(64, 64, h, V1)
    al = 2 * np.pi * np.arange(64) / 64
    g = O.OGeom.from_synth(geom)
    U = O.solve_phi(g, torch.as_tensor(np.cos(k * al)))["U"].numpy()
    assert np.abs(U - k * np.tanh(k * h) * np.cos(k * al)).max() < 1e-12


def test_tangential_velocity_manufactured():
    """dphi/ds on the surface, the bottom and the obstacle (Sec. 5.1 formulas)
    against Re{Phi'(zeta) zeta'}/|zeta'| of the manufactured flow, converging
    spectrally; the same formula on the walls of a flow with no obstacles."""
    errs = []
    for M0, M1, M2 in [(64, 64, 32), (128, 128, 64), (256, 256, 128)]:
        geom, phi, _, _ = manufactured_case(M0, M1, M2)
        g = O.OGeom.from_synth(geom)
        r = O.solve_phi(g, torch.as_tensor(phi))
        ds = torch.cat(O.dphi_ds_from_omega(g, O.split(g, r["omega"]))).numpy()
        ex = exact_dphi_ds(geom, CASE_FLOW)
        errs.append(np.abs(ds - ex).max() / np.abs(ex).max())
    assert errs[-1] < 1e-10, errs
    assert errs[0] > 10 * errs[-1], errs


@pytest.mark.parametrize("k", [1, 4])
def test_tangential_velocity_flat_strip(k):
    """Flat strip of depth h, phi~ = cos(k alpha): phi = cosh(k(y+h))/cosh(kh) cos(kx),
    so dphi/ds = -k sin(k alpha) on the surface and -k sin(k alpha)/cosh(kh) on
    the bottom (whose tangent points in +x)."""
    h = 1.5
    geom = flat_strip(64, 64, h)
    al = 2 * np.pi * np.arange(64) / 64
    g = O.OGeom.from_synth(geom)
    r = O.solve_phi(g, torch.as_tensor(np.cos(k * al)))
    ds = O.dphi_ds_from_omega(g, O.split(g, r["omega"]))
    assert np.abs(ds[0].numpy() + k * np.sin(k * al)).max() < 1e-12
    assert np.abs(ds[1].numpy() + k * np.sin(k * al) / np.cosh(k * h)).max() < 1e-12


def _gamma_of_state(g, phi):
    parts = O.split(g, O.solve_phi(g, phi)["omega"])
    return torch.cat([-O.spectral(parts[0], "D")] + [O.spectral(p, "D") for p in parts[1:]])


@pytest.mark.parametrize("tau,vamp", [(0.1, 0.1), (0.0, -0.3)])
def test_gamma_t_matches_time_derivative(tau, vamp):
    """The Sec. 4.2 system for gamma_t against the time derivative of the
    velocity-potential solution: move the surface by zeta_t = (V + iU) zeta'/s
    and phi~ by its Sec. 3.5 equation, re-solve at t +- dt and difference
    gamma = (-D omega_0, D omega_j) centrally (config 1, M = 640)."""
    cfg = make_config(1)
    g = O.OGeom.from_synth(cfg["geom"])
    phi = torch.as_tensor(cfg["phi"])
    M0 = g.M[0]
    al = 2 * np.pi * torch.arange(M0, dtype=torch.float64) / M0
    V = vamp * torch.sin(al) + 0.03 * torch.cos(2 * al)
    gt = O.solve_gamma_t(g, phi, V, tau)["gamma_t"]
    zt, phit = O.surface_velocity_state(g, phi, V, tau)
    xt, yt = g.z[0].real - al, g.z[0].imag
    dt = 1e-4
    gams = []
    for sg in (1.0, -1.0):
        z, d, e = O.surface_from_periodic(xt + sg * dt * zt.real, yt + sg * dt * zt.imag)
        gams.append(_gamma_of_state(g.with_surface(z, d, e), phi + sg * dt * phit))
    fd = (gams[0] - gams[1]) / (2 * dt)
    off = np.cumsum([0] + g.M)
    for k in range(g.nb):
        a, b = gt[off[k]:off[k + 1]], fd[off[k]:off[k + 1]]
        assert float((a - b).abs().max() / a.abs().max()) < 1e-6, k


def test_manufactured_flow_converges_spectrally():
    """Exact U and psi|_k of a manufactured periodic flow, with spectral convergence."""
    errs = []
    for M0, M1, M2 in [(32, 32, 16), (64, 64, 32), (128, 128, 64), (256, 256, 128)]:
        geom, phi, U, ck = manufactured_case(M0, M1, M2)
        g = O.OGeom.from_synth(geom)
        r = O.solve_phi(g, torch.as_tensor(phi))
        errs.append(np.abs(r["U"].numpy() - U).max() / np.abs(U).max())
        if M0 >= 128:
            assert np.abs(r["psi_k"].numpy() - ck).max() < 1e-13
    assert errs[0] > 100 * errs[1] > 100 * 100 * errs[2] * 0.1
    assert errs[2] < 1e-12 and errs[3] < 1e-12


def test_mv_term_alone():
    """w_j = z_j and F = 0: b = 0 so omega = 0 and U = Re{Phi_mv' i zeta'}/s."""
    cfg = make_config(1)
    geom = cfg["geom"]
    flow = Flow(1.0, geom.a, geom.zc)
    phi, pw, U, _ = manufactured_inputs(geom, flow, [0.0])
    geom.psi_wall = pw
    g = O.OGeom.from_synth(geom)
    r = O.solve_phi(g, torch.as_tensor(phi))
    assert r["omega"].abs().max() < 1e-13
    assert np.abs(r["U"].numpy() - U).max() < 1e-13


def _indicator(g, m):
    return torch.cat([torch.full((g.M[k],), 1.0 if k == m else 0.0, dtype=torch.float64)
                      for k in range(g.nb)])


@pytest.mark.parametrize("which", ["c1", "ragged"])
def test_null_vectors(which):
    """A 1_0 = -1_0/2; A 1_1 = 1/2 on every wall and 0 on the surface; A 1_m = -1_m (m >= 2)."""
    geom = make_config(1)["geom"] if which == "c1" else ragged_config()["geom"]
    g = O.OGeom.from_synth(geom)
    A = O.assemble_A(g)
    walls = 1.0 - _indicator(g, 0)
    tol = 1e-12 if which == "c1" else 1e-10    # identities hold to spectral accuracy
    assert (A @ _indicator(g, 0) + 0.5 * _indicator(g, 0)).abs().max() < tol
    assert (A @ _indicator(g, 1) - 0.5 * walls).abs().max() < tol
    for m in range(2, g.nb):
        assert (A @ _indicator(g, m) + _indicator(g, m)).abs().max() < tol


@pytest.mark.parametrize("which", ["c1", "ragged"])
def test_zero_net_flux(which):
    """Incompressibility: sum_m U_m s_m = 0 over one period."""
    cfg = make_config(1) if which == "c1" else ragged_config()
    g = O.OGeom.from_synth(cfg["geom"])
    U = O.solve_phi(g, torch.as_tensor(cfg["phi"]))["U"]
    assert abs(float((U * g.d[0].abs()).sum())) < 1e-12 * g.M[0]


@pytest.mark.parametrize("which", ["c1", "ragged"])
def test_velocity_potential_equals_vortex_sheet(which):
    """U from gamma_0 = -omega_0' (Sec. 4.1) equals U of Sec. 3.4; gamma_j = omega_j'."""
    cfg = make_config(1) if which == "c1" else ragged_config()
    g = O.OGeom.from_synth(cfg["geom"])
    r = O.solve_phi(g, torch.as_tensor(cfg["phi"]))
    parts = O.split(g, r["omega"])
    rv = O.solve_gamma(g, -O.spectral(parts[0], "D"))
    assert (rv["U"] - r["U"]).abs().max() < 1e-12
    gw = torch.cat([O.spectral(p, "D") for p in parts[1:]])
    # gamma_j and omega_j' agree to the walls' resolution (coarse in the ragged cell)
    tol = 1e-10 if which == "c1" else 1e-6
    assert (rv["gamma_wall"] - gw).abs().max() < tol * max(1.0, float(gw.abs().max()))


def test_spectral_operators_on_trig_polynomials():
    M = 48
    al = torch.as_tensor(2 * np.pi * np.arange(M) / M)
    for k in (1, 5, 23):
        c, s = torch.cos(k * al), torch.sin(k * al)
        assert (O.spectral(c, "D") + k * s).abs().max() < 1e-12
        assert (O.spectral(s, "D2") + k * k * s).abs().max() < 1e-10
        assert (O.spectral(c, "H") - s).abs().max() < 1e-13
        assert (O.spectral(s, "H") + c).abs().max() < 1e-13
        assert (O.spectral(c, "ABSD") - k * c).abs().max() < 1e-12
    nyq = torch.cos(M // 2 * al)
    for op in ("D", "D2", "H", "ABSD"):
        assert O.spectral(nyq, op).abs().max() < 1e-12
    assert O.spectral(torch.ones(M, dtype=torch.float64), "H").abs().max() < 1e-14


def test_zero_data_gives_zero():
    cfg = make_config(1)
    geom = cfg["geom"]
    geom.V1, geom.a = 0.0, np.zeros_like(geom.a)
    g = O.OGeom.from_synth(geom)
    r = O.solve_phi(g, torch.zeros(geom.M[0], dtype=torch.float64))
    assert r["omega"].abs().max() == 0.0 and r["U"].abs().max() == 0.0


def test_linearity_in_data():
    cfg = make_config(1)
    g = O.OGeom.from_synth(cfg["geom"])
    phi = torch.as_tensor(cfg["phi"])
    r1 = O.solve_phi(g, phi)
    r2 = O.solve_phi(g, 2.0 * phi)
    g0 = O.OGeom.from_synth(cfg["geom"])
    g0.V1, g0.a = 0.0, torch.zeros_like(g0.a)
    rh = O.solve_phi(g0, phi)          # homogeneous part
    assert ((r2["omega"] - r1["omega"]) - rh["omega"]).abs().max() < 1e-12


def test_gradient_matches_central_differences():
    """Autograd gradient of J = sum w U^2 vs central differences of the oracle."""
    t = tiny_config()
    gw = O.OGeom.from_synth(t["geom"])
    al = gw.alpha[0]
    xt, yt = gw.z[0].real - al, gw.z[0].imag
    ph = torch.as_tensor(t["phi"])
    wts = torch.as_tensor(np.random.default_rng(3).uniform(0, 1, 32))
    _, gx, gy, gp, _ = O.J_and_grad(gw, xt, yt, ph, wts)
    rng = np.random.default_rng(5)
    for _ in range(3):
        v = [torch.as_tensor(np.cos(2 * al.numpy() + rng.uniform(0, 6)) * rng.standard_normal())
             for _c in range(3)]
        h = 1e-5
        Jp = O.J_and_grad(gw, xt + h * v[0], yt + h * v[1], ph + h * v[2], wts)[0]
        Jm = O.J_and_grad(gw, xt - h * v[0], yt - h * v[1], ph - h * v[2], wts)[0]
        fd = (Jp - Jm) / (2 * h)
        an = float((gx * v[0]).sum() + (gy * v[1]).sum() + (gp * v[2]).sum())
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)), (fd, an)


def test_sampled_rows_equal_full_matrix():
    cfg = ragged_config()
    g = O.OGeom.from_synth(cfg["geom"])
    A = O.assemble_A(g)
    rows = [0, 7, 249, 250, 375, 376, 441, 442, 499]
    assert (O.A_rows(g, rows) - A[rows]).abs().max() == 0.0


# ---------------------------------------------------------------------------
# one Runge-Kutta stage of the free-surface evolution (Sec. 2, 3.5, 5)
# ---------------------------------------------------------------------------

def _stage_setup():
    cfg = make_config(1)
    g = O.OGeom.from_synth(cfg["geom"])
    M0 = g.M[0]
    al = 2 * np.pi * torch.arange(M0, dtype=torch.float64) / M0
    return g, torch.as_tensor(cfg["phi"]), al


def test_hls_reconstruction_closes_the_curve():
    """P theta = 0 gives the flat surface; a general P theta gives a curve with
    |zeta'| = s_alpha, arg zeta' = theta, zeta' = 1 + D(zeta - alpha), xi(0) = 0
    and zero mean height (Sec. 2.2)."""
    _, _, al = _stage_setup()
    z, d, e, th, sa = O.hls_reconstruct(torch.zeros_like(al))
    assert float((z - al).abs().max()) < 1e-15 and abs(float(sa) - 1.0) < 1e-15
    Pt = 0.15 * torch.sin(al) + 0.05 * torch.cos(2 * al) - 0.04 * torch.sin(3 * al)
    z, d, e, th, sa = O.hls_reconstruct(Pt)
    assert float((d.abs() - sa).abs().max()) < 1e-14
    assert float((torch.angle(d) - th).abs().max()) < 1e-14
    dz = (1.0 + O.spectral(z.real - al, "D")) + 1j * O.spectral(z.imag, "D")
    assert float((dz - d).abs().max()) < 1e-12
    assert abs(float(z.real[0])) < 1e-15 and abs(float((z.imag * d.real).mean())) < 1e-15
    assert abs(complex(d.mean()) - 1.0) < 1e-14


@pytest.mark.parametrize("mode", ["graph", "hls"])
def test_stage_conserves_energy(mode):
    """Along the stage's time derivatives the energy of Sec. 5.2 is stationary:
    central differences over +-1e-4 give |dE/dt| below 1e-8, against
    derivatives of order one (a dropped or mis-signed term of the phi~
    equation, or a wrong V, moves it by orders of magnitude)."""
    g, phi, al = _stage_setup()
    tau = 0.1
    q = (0.1 * torch.cos(al) + 0.02 * torch.sin(2 * al) if mode == "graph"
         else 0.15 * torch.sin(al) + 0.05 * torch.cos(2 * al))
    qt, pt, _ = O.stage_rhs(g, mode, q, phi, tau)

    def E(qq, pp):
        z, d, e = O.graph_surface(qq) if mode == "graph" else O.hls_reconstruct(qq)[:3]
        gg = g.with_surface(z, d, e)
        return O.energy(gg, pp, O.solve_phi(gg, pp)["omega"], tau, 1.0)

    dt = 1e-4
    dE = (E(q + dt * qt, phi + dt * pt) - E(q - dt * qt, phi - dt * pt)) / (2 * dt)
    assert float(qt.abs().max()) > 0.1 and float(pt.abs().max()) > 0.1
    assert abs(dE) < 1e-8, dE


def test_hls_kinematics():
    """The curve reconstructed from P theta +- dt (P theta)_t moves with
    (V + iU) zeta'/s_alpha (Sec. 2.2 and the HLS appendix): V keeps xi(0) = 0
    and the mean height fixed."""
    g, phi, al = _stage_setup()
    q = 0.15 * torch.sin(al) + 0.05 * torch.cos(2 * al)
    qt, _, ex = O.stage_rhs(g, "hls", q, phi, 0.1)
    dt = 1e-4
    zt = (O.hls_reconstruct(q + dt * qt)[0] - O.hls_reconstruct(q - dt * qt)[0]) / (2 * dt)
    ref = (ex["V"] + 1j * ex["U"]) * ex["d"] / ex["d"].abs()
    assert float((zt - ref).abs().max()) < 1e-8


def test_rk4_converges_at_fourth_order():
    """The classical RK4 tableau through rk_step (filter off): halving h
    divides the error at T = 0.02 by about 16."""
    g, phi, al = _stage_setup()
    q0 = 0.1 * torch.cos(al) + 0.02 * torch.sin(2 * al)
    A = [[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1, 0]]
    b = [1 / 6, 1 / 3, 1 / 3, 1 / 6]

    def run(h, nsteps):
        q, p = q0.clone(), phi.clone()
        for _ in range(nsteps):
            q, p = O.rk_step(g, "graph", A, b, h, q, p, 0.1, filt=False)
        return q, p

    qr, pr = run(0.02 / 16, 16)
    errs = []
    for k in (2, 4):
        q, p = run(0.02 / k, k)
        errs.append(max(float((q - qr).abs().max()), float((p - pr).abs().max())))
    assert 10.0 < errs[0] / errs[1] < 24.0, errs


def test_filter_symbol():
    """exp(-36 (|k|/kmax)^36): mode kmax/2 is damped by 36 * 2^-36 (5.2e-10),
    the top mode below Nyquist is cut to exp(-36 ((M/2-1)/(M/2))^36) (Sec. 5)."""
    M = 64
    al = 2 * np.pi * torch.arange(M, dtype=torch.float64) / M
    f = torch.cos(16 * al)
    want = np.exp(-36.0 * 0.5 ** 36)
    assert float((O.spectral(f, "FILTER") - want * f).abs().max()) < 1e-13
    f = torch.cos(31 * al)
    want = np.exp(-36.0 * (31 / 32) ** 36)
    assert float((O.spectral(f, "FILTER") - want * f).abs().max()) < 1e-13


# ---------------------------------------------------------------------------
# values inside the fluid (Sec. 5.1, Helsing-Ojala appendix)
# ---------------------------------------------------------------------------

def _inward_points(g, dists=(1e-1, 1e-2, 1e-4, 1e-7), stride=7):
    """Points pushed into the fluid from every stride-th node: along -i zeta'/s
    below the surface, along +i zeta'/s off the bottom and the clockwise obstacles."""
    pts = []
    for k in range(g.nb):
        nrm = (-1j if k == 0 else 1j) * g.d[k] / torch.abs(g.d[k])
        for dist in dists:
            pts.append(g.z[k][::stride] + dist * nrm[::stride])
    return torch.cat(pts)


def test_helsing_ojala_analytic_function():
    """e^{-iz} + 0.15 cot((z - p)/2) with p inside the obstacle, from its boundary
    values, at points down to 1e-7 from every boundary: spectrally accurate (1e-14);
    the same sum with the surface taken along its parameter fails."""
    geom, _, _, _ = manufactured_case(256, 256, 128)
    g = O.OGeom.from_synth(geom)
    z = _inward_points(g)
    f = lambda w: torch.exp(-1j * w) + 0.15 / torch.tan(0.5 * (w - (np.pi - 0.5j)))
    val = O.helsing_ojala(g, [f(zz) for zz in g.z], z)
    assert float((val - f(z)).abs().max() / f(z).abs().max()) < 1e-14
    flipped = O.OGeom([g.z[0].flip(0)] + g.z[1:], [-g.d[0].flip(0)] + g.d[1:],
                      [g.e[0].flip(0)] + g.e[1:], g.zc, g.a, g.V1)
    bad = O.helsing_ojala(flipped, [f(zz) for zz in flipped.z], z)
    assert float((bad - f(z)).abs().max() / f(z).abs().max()) > 1e-3


def test_boundary_and_interior_velocity_manufactured():
    """Phi' = u - iv of the manufactured flow: on all boundaries from the
    solve's densities (dphi/ds and dphi/dn of every boundary) and inside the
    fluid by the Helsing-Ojala rule, down to 1e-7 from the boundary."""
    geom, phi, _, _ = manufactured_case(256, 256, 128)
    g = O.OGeom.from_synth(geom)
    om = O.split(g, O.solve_phi(g, torch.as_tensor(phi))["omega"])
    bd = O.boundary_dPhi(g, om)
    for k, c in enumerate(geom.curves):
        ex = torch.as_tensor(CASE_FLOW.dPhi(c.z))
        assert float((bd[k] - ex).abs().max()) < 1e-10, k
    z = _inward_points(g)
    exz = torch.as_tensor(CASE_FLOW.dPhi(z.numpy()))
    assert float((O.helsing_ojala(g, bd, z) - exz).abs().max() / exz.abs().max()) < 1e-11


def test_walls_are_streamlines():
    """For the physical problem (psi_wall = 0) dphi/dn vanishes on every wall up
    to the discretization error, and equals U on the surface."""
    cfg = make_config(1)
    g = O.OGeom.from_synth(cfg["geom"])
    r = O.solve_phi(g, torch.as_tensor(cfg["phi"]))
    dn = O.dphi_dn_all(g, O.split(g, r["omega"]))
    assert float((dn[0] - r["U"]).abs().max()) < 1e-14
    for v in dn[1:]:
        assert float(v.abs().max()) < 1e-10


def test_plemelj_boundary_values_consistent():
    """For an arbitrary density omega, the Helsing-Ojala rule applied to the
    Plemelj boundary values of sum_k Phi_k (Re and Im on every boundary)
    reproduces the directly summed Cauchy integrals at points away from the
    boundaries: a wrong sign or kernel in any of the eight formulas fails."""
    cfg = make_config(1)
    g = O.OGeom.from_synth(cfg["geom"])
    rng = np.random.default_rng(3)
    om = [torch.as_tensor(0.2 * np.cos(np.arange(m) * 2 * np.pi / m * rng.integers(1, 4))
                          + 0.1 * rng.standard_normal()) for m in g.M]
    xs = torch.linspace(0.3, 2 * np.pi - 0.3, 9, dtype=torch.float64)
    z = torch.cat([xs - 0.25j, xs - 0.8j])
    z = z[((z.real - np.pi) / 0.3) ** 2 + ((z.imag + 0.5) / 0.15) ** 2 > 2.0]
    direct = O.layer_potential_direct(g, om, z)
    ho = O.helsing_ojala(g, O.boundary_Phi(g, om), z)
    assert float((direct - ho).abs().max() / direct.abs().max()) < 1e-12


@pytest.mark.parametrize("V1", [0.0, 0.7])
def test_pressure_hydrostatic_and_uniform_current(V1):
    """Flat surface over a flat bottom, phi~ = 0: at rest and in a uniform
    current V1 the pressure is hydrostatic, p = -g y (steady Bernoulli)."""
    geom = flat_strip(64, 64, 1.0, V1)
    g = O.OGeom.from_synth(geom)
    z = torch.tensor([1.0 - 0.3j, 2.0 - 0.6j, 4.0 - 0.95j], dtype=torch.complex128)
    p = O.pressure(g, torch.zeros(64, dtype=torch.float64), 0.1, 1.0, z)
    assert float((p + z.imag).abs().max()) < 1e-14


def test_pressure_surface_limit():
    """Approaching the free surface the pressure tends to -tau kappa
    (Laplace-Young), the Dirichlet data of the auxiliary problem."""
    cfg = make_config(1)
    g = O.OGeom.from_synth(cfg["geom"])
    d = g.d[0][::16]
    z = g.z[0][::16] + 1e-9 * (-1j) * d / d.abs()
    p = O.pressure(g, torch.as_tensor(cfg["phi"]), 0.1, 1.0, z)
    kappa = ((g.e[0] / g.d[0]).imag / g.d[0].abs())[::16]
    assert float((p + 0.1 * kappa).abs().max()) < 1e-7


def test_spectral_tail_closed_forms():
    """The resolution measure (Sec. 7.1's Fourier-tail test): the root of the
    energy fraction in the modes |k| >= 3M/8.  Single modes below and in the
    band give 0 and 1; a Nyquist mode carries one coefficient of size M
    against two of M/2 for the others; and the Poisson kernel
    1/(1 - 2 rho cos a + rho^2), whose coefficients are rho^|k| / (1 - rho^2),
    gives a geometric tail sum (sampled, mode k also collects its aliases:
    (rho^|k| + rho^(M - |k|)) / (1 - rho^M), up to the common factor)."""
    M = 64
    a = torch.arange(M, dtype=torch.float64) * (2 * np.pi / M)
    assert O.spectral_tail(torch.cos(5 * a)) < 1e-14
    assert O.spectral_tail(torch.cos(23 * a)) < 1e-14          # 23 < 24 = 3M/8
    assert abs(O.spectral_tail(torch.sin(24 * a)) - 1.0) < 1e-14
    x, y = 0.6, 1.7
    r = O.spectral_tail(x * torch.cos(3 * a) + y * torch.cos(30 * a))
    assert abs(r - y / np.hypot(x, y)) < 1e-14
    r = O.spectral_tail(x * torch.cos(3 * a) + y * torch.cos(32 * a))   # Nyquist
    assert abs(r - y / np.sqrt(x * x / 2 + y * y)) < 1e-14
    M = 256
    a = torch.arange(M, dtype=torch.float64) * (2 * np.pi / M)
    rho = 0.9
    f = 1.0 / (1.0 - 2 * rho * torch.cos(a) + rho * rho)
    k = np.abs(np.arange(-M // 2 + 1, M // 2 + 1))
    e = ((rho ** k + rho ** (M - k)) / (1 - rho ** M)) ** 2
    expect = np.sqrt(e[k >= 96].sum() / e.sum())
    assert abs(O.spectral_tail(f) / expect - 1.0) < 1e-9
