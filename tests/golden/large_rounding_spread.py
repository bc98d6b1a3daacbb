"""Rounding floor of U on the large cell (M = 40960), recorded beside the
oracle's reference in tests/golden/large_M40960.json.

U applies D and |d| to omega (Sec. 3.4), which amplify its highest modes by
up to M_0/2, and divides by |zeta'|; on this near-overturning surface that
turns rounding-level noise in omega into a visible error in U.  Two oracle-only
measurements bound what an FP64 implementation can be asked to match:

* omega rounding: U from the stored reference omega against U from omega with
  every entry perturbed by one relative unit of rounding (2^-53 times a
  seeded standard normal), three seeds;
* entry rounding: the matrix of the collocated system (Sec. 3.3) with every
  entry perturbed by one relative unit of rounding (one seed), solved by the
  oracle's GMRES to 1e-15 and mapped to U, against the stored reference U --
  what any implementation whose entries are correct to an ulp may differ by.

Run from the repository root:  python tests/golden/large_rounding_spread.py
(a few minutes on 8 cores; peaks near 15 GB of host memory).
"""
import json
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import make_config  # noqa: E402


def rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def main():
    cfg = make_config(5)
    og = O.OGeom.from_synth(cfg["geom"])
    gd = np.load(os.path.join(HERE, "large_M40960.npz"))
    om = torch.as_tensor(gd["omega"])
    U0 = O.dphi_dn_from_omega_chunked(og, O.split(og, om))
    spreads = []
    for seed in (1, 2, 3):
        xi = torch.as_tensor(np.random.default_rng(seed).standard_normal(om.shape[0]))
        U1 = O.dphi_dn_from_omega_chunked(og, O.split(og, om * (1.0 + 2.0 ** -53 * xi)))
        spreads.append(rel(U1, U0))
        print(f"omega rounding, seed {seed}: {spreads[-1]:.3e}", flush=True)

    A = O.assemble_A_blocked(og, chunk=512)
    rng = np.random.default_rng(7)
    for r0 in range(0, A.shape[0], 512):
        blk = A[r0:r0 + 512]
        blk *= 1.0 + 2.0 ** -53 * torch.as_tensor(rng.standard_normal(tuple(blk.shape)))
    b = O.rhs(og, torch.as_tensor(np.asarray(cfg["phi"])))
    x, hist, steps = O.gmres(lambda v: A @ v, b, tol=1e-15, restart=120, max_iter=1200)
    del A
    Ue = O.dphi_dn_from_omega_chunked(og, O.split(og, x))
    ent = {"U": rel(Ue, torch.as_tensor(gd["U"])), "omega": rel(x, om),
           "gmres_steps": steps, "cycle_start_resid": hist, "seed": 7}
    print(f"entry rounding: {ent}", flush=True)

    path = os.path.join(HERE, "large_M40960.json")
    meta = json.load(open(path))
    meta["U_rounding_spread"] = {
        "omega_rounding": {"seeds": [1, 2, 3], "rel_change_U": spreads},
        "entry_rounding": ent,
        "command": "python tests/golden/large_rounding_spread.py"}
    with open(path, "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
