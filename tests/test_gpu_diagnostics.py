"""Tangential velocity on every boundary and the energy (Sec. 5.1 and 5.2)
from the densities of a velocity-potential solve, against the oracle, the
manufactured flow's closed form and the paper's printed E(0)."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from manufactured import CASE_FLOW, exact_dphi_ds, manufactured_case
from synth import make_config, paper_problem, ragged_config, tiny_config

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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
    if name == "tiny":
        return tiny_config()
    if name == "ragged":
        return ragged_config()
    return make_config(int(name[1]))


@pytest.mark.parametrize("name", ["tiny", "ragged", "c1", "c2"])
def test_tangential_and_energy_match_oracle(ww, ctx, name):
    say(f"case tangential/energy vs oracle {name}")
    cfg = _cfg(name)
    geom = cfg["geom"]
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    _, omega, _, _ = ctx.solve_phi(dg, phi, tol=1e-13)
    ds, E, _ = ctx.tangential_energy(dg, omega, phi, tau=0.1, grav=1.0)
    og = O.OGeom.from_synth(geom)
    om = omega.cpu()
    ref = torch.cat(O.dphi_ds_from_omega(og, O.split(og, om))).numpy()
    err = np.abs(ds.cpu().numpy() - ref).max() / np.abs(ref).max()
    Er = O.energy(og, torch.as_tensor(cfg["phi"]), om, 0.1, 1.0)
    say(f"  dphi/ds err {err:.2e}  E {E:.15f} oracle {Er:.15f}")
    assert err <= 1e-12
    assert abs(E - Er) <= 1e-13 * max(1.0, abs(Er))


def test_tangential_manufactured(ww, ctx):
    """dphi/ds on the surface, bottom and obstacle of the manufactured flow."""
    say("case tangential manufactured 256/256/128")
    geom, phi, _, _ = manufactured_case(256, 256, 128)
    dg = ww.DeviceGeometry.from_synth(geom, DEV)
    _, omega, _, _ = ctx.solve_phi(dg, torch.as_tensor(phi, device=DEV), tol=1e-14)
    ds, _, _ = ctx.tangential_energy(dg, omega, want_energy=False)
    ex = exact_dphi_ds(geom, CASE_FLOW)
    err = np.abs(ds.cpu().numpy() - ex).max() / np.abs(ex).max()
    say(f"  err vs closed form {err:.2e}")
    assert err <= 1e-10


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
def test_energy_matches_printed_E0(ww, ctx, problem):
    """E(0) of problems 1-3 (Sec. 7.3 table) computed entirely on the device."""
    say(f"case energy problem {problem}")
    ref = _golden_energy()[problem]
    cfg = paper_problem(problem)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    phi = torch.as_tensor(cfg["phi"], device=DEV)
    _, omega, _, _ = ctx.solve_phi(dg, phi, tol=1e-13)
    _, E, _ = ctx.tangential_energy(dg, omega, phi, tau=cfg["tau"], grav=cfg["g"],
                                    want_dphids=False)
    say(f"  E {E:.7f} printed {ref}")
    assert abs(E - ref) <= 6e-6


def test_tangential_energy_errors(ww, ctx):
    say("case tangential/energy errors")
    cfg = make_config(1)
    dg = ww.DeviceGeometry.from_synth(cfg["geom"], DEV)
    omega = torch.zeros(dg.n, dtype=torch.float64, device=DEV)
    with pytest.raises(ww.WWBIError) as e:
        ctx.tangential_energy(dg, omega, None, want_dphids=False, want_energy=True)
    assert e.value.status == ww.EINVAL_NULL
    with pytest.raises(ww.WWBIError) as e:
        ctx.tangential_energy(dg, omega, want_dphids=False, want_energy=False)
    assert e.value.status == ww.EINVAL_NULL
