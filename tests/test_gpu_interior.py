"""Velocity on the boundaries and inside the fluid (Sec. 4.1, 5.1 and the
Helsing-Ojala rule) on the device, against the oracle and closed forms."""
import numpy as np
import pytest
import torch

import oracle as O
from manufactured import CASE_FLOW, manufactured_case
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


def _inward_points(g, dists=(1e-1, 1e-2, 1e-4, 1e-7), stride=7):
    pts = []
    for k in range(g.nb):
        nrm = (-1j if k == 0 else 1j) * g.d[k] / torch.abs(g.d[k])
        for dist in dists:
            pts.append(g.z[k][::stride] + dist * nrm[::stride])
    return torch.cat(pts)


def test_interior_eval_analytic(ww, ctx):
    """An analytic periodic function at points down to 1e-7 from every
    boundary, plus points exactly on nodes."""
    say("case interior eval analytic")
    geom, _, _, _ = manufactured_case(256, 256, 128)
    g = O.OGeom.from_synth(geom)
    z = torch.cat([_inward_points(g), g.z[0][:5], g.z[2][3:6]])
    f = lambda w: torch.exp(-1j * w) + 0.15 / torch.tan(0.5 * (w - (np.pi - 0.5j)))
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    fb = torch.cat([f(zz) for zz in g.z]).to(DEV)
    val = ctx.interior_eval(dg, fb, z.to(DEV)).cpu()
    err = float((val - f(z)).abs().max() / f(z).abs().max())
    ref = O.helsing_ojala(g, [f(zz) for zz in g.z], z)
    par = float((val - ref).abs().max() / ref.abs().max())
    say(f"  err vs closed form {err:.1e}  vs oracle {par:.1e}")
    assert err <= 1e-13 and par <= 1e-13


@pytest.mark.parametrize("name", ["manufactured", "c1", "ragged"])
def test_boundary_and_interior_velocity(ww, ctx, name):
    say(f"case velocity {name}")
    if name == "manufactured":
        geom, phi, _, _ = manufactured_case(256, 256, 128)
    else:
        cfg = make_config(1) if name == "c1" else ragged_config()
        geom, phi = cfg["geom"], cfg["phi"]
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    _, omega, _, _ = ctx.solve_phi(dg, torch.as_tensor(phi, device=DEV), tol=1e-13)
    g = O.OGeom.from_synth(geom)
    om = O.split(g, omega.cpu())
    bd = torch.cat(O.boundary_dPhi(g, om))
    u, v = ctx.boundary_velocity(dg, omega)
    fb = torch.complex(u.cpu(), -v.cpu())
    eb = float((fb - bd).abs().max() / bd.abs().max())
    z = _inward_points(g)
    ui, vi = ctx.interior_velocity(dg, omega, z.to(DEV))
    fi = torch.complex(ui.cpu(), -vi.cpu())
    ref = O.helsing_ojala(g, O.boundary_dPhi(g, om), z)
    ei = float((fi - ref).abs().max() / ref.abs().max())
    say(f"  boundary parity {eb:.1e}  interior parity {ei:.1e}")
    assert eb <= 1e-11 and ei <= 1e-11
    if name == "manufactured":
        ex = torch.as_tensor(CASE_FLOW.dPhi(z.numpy()))
        ee = float((fi - ex).abs().max() / ex.abs().max())
        say(f"  interior vs closed form {ee:.1e}")
        assert ee <= 1e-10


@pytest.mark.parametrize("name,prec", [("c1", "fp64"), ("ragged", "fp64"), ("c1", "fp32")])
def test_pressure_matches_oracle(ww, ctx, name, prec):
    """Pressure at points inside the fluid, down to 1e-7 from the boundaries."""
    say(f"case pressure {name} {prec}")
    cfg = make_config(1) if name == "c1" else ragged_config()
    geom, phi = cfg["geom"], cfg["phi"]
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    g = O.OGeom.from_synth(geom)
    z = _inward_points(g, dists=(1e-1, 1e-3, 1e-7), stride=11)
    p, rep = ctx.pressure(dg, torch.as_tensor(phi, device=DEV), z.to(DEV), tau=0.1,
                          tol=1e-13 if prec == "fp64" else 1e-14,
                          precision=ww.FP64 if prec == "fp64" else ww.FP32_REFINED)
    ref = O.pressure(g, torch.as_tensor(phi), 0.1, 1.0, z)
    err = float((p.cpu() - ref).abs().max() / ref.abs().max())
    say(f"  err {err:.1e}  iters {rep.iters}")
    assert err <= (1e-11 if prec == "fp64" else 1e-10)


@pytest.mark.parametrize("V1", [0.0, 0.7])
def test_pressure_hydrostatic(ww, ctx, V1):
    say(f"case pressure hydrostatic V1={V1}")
    from manufactured import flat_strip
    geom = flat_strip(64, 64, 1.0, V1)
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    z = torch.tensor([1.0 - 0.3j, 2.0 - 0.6j, 4.0 - 0.95j], dtype=torch.complex128)
    p, _ = ctx.pressure(dg, torch.zeros(64, dtype=torch.float64, device=DEV), z.to(DEV), tau=0.1)
    assert float((p.cpu() + z.imag).abs().max()) <= 1e-13


def test_interior_point_checks(ww, ctx):
    """Interior points are checked before any work: a non-finite coordinate
    gives EINVAL_NONFINITE, |y| > 30 gives EINVAL_RANGE, on all three entries;
    valid points afterwards still evaluate."""
    say("case interior point checks")
    cfg = make_config(1)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    _, omega, _, _ = ctx.solve_phi(dg, phi, tol=1e-13)
    good = torch.tensor([1.0 - 0.3j, 2.0 - 0.7j], dtype=torch.complex128, device=DEV)
    f = torch.zeros(dg.n, dtype=torch.complex128, device=DEV)
    for bad, status in ((torch.tensor([1.0 - 0.3j, complex(float("nan"), -0.5)]), ww.EINVAL_NONFINITE),
                        (torch.tensor([1.0 - 0.3j, 2.0 - 31.0j]), ww.EINVAL_RANGE)):
        z = bad.to(torch.complex128).to(DEV)
        with pytest.raises(ww.WWBIError) as e:
            ctx.interior_eval(dg, f, z)
        assert e.value.status == status
        with pytest.raises(ww.WWBIError) as e:
            ctx.interior_velocity(dg, omega, z)
        assert e.value.status == status
        with pytest.raises(ww.WWBIError) as e:
            ctx.pressure(dg, phi, z, tol=1e-13)
        assert e.value.status == status
    u, v = ctx.interior_velocity(dg, omega, good)
    assert torch.isfinite(u).all() and torch.isfinite(v).all()
