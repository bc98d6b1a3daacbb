"""Rounding floor of gamma_t (Sec. 4.2) on the config-2 cell (M = 4608,
surface 2048), recorded in tests/golden/gamma_t_spread.json.

gamma_t applies d/dalpha twice to the velocity-potential solution (gamma_0 =
-D omega_0, then D of the right-hand side's bracket), so rounding upstream
reaches it amplified by up to about (M_0/2)^2.  This script measures, with the
oracle alone, how far gamma_t moves when every kernel entry it uses moves by
one relative unit of rounding (2^-53 times a seeded standard normal): the
K and G blocks of Table 1 from which the velocity-potential matrix (Sec.
3.3), the gamma_t operator (Sec. 4.2) and the maps of its right-hand side
(U, the tangential velocity, the F operators) are all built, and every
output of the spectral operators D and H.  Three seeds, at the state and
tangential velocity the GPU tests use (V = 0.1 sin(alpha) + 0.03 cos(2
alpha), tau = 0.1).  An implementation that forms each entry and each
spectral derivative to about an ulp may differ from the oracle by that much.

A second measure perturbs only omega, the velocity-potential solution the
right-hand side is built from, by one relative unit of rounding per entry
(three seeds): the rounding every FP64 solve leaves in omega, which the two
derivatives amplify by up to about (M_0/2)^2.

A third measure swaps the solver: both systems solved by the oracle's
restarted GMRES to 1e-15 (the paper's solver and tolerance, Sec. 7.4) instead
of the refined dense solve (LU plus one extended-precision refinement step,
which reaches the FP64 system's solution to its last bits).  GMRES stops at
its tolerance, and the truncation error it leaves in omega is what the two
derivatives amplify; that spread separates a correct GMRES-based FP64
implementation from the oracle.

Run from the repository root:  python tests/golden/gamma_t_spread.py
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
import oracle.bim as B  # noqa: E402
from synth import make_config  # noqa: E402


def perturbed(fn, rng):
    def wrapped(*a, **k):
        M = fn(*a, **k)
        return M * (1.0 + 2.0 ** -53 * torch.as_tensor(rng.standard_normal(tuple(M.shape))))
    return wrapped


def main():
    out = {}
    for c in (1, 2):
        cfg = make_config(c)
        og = O.OGeom.from_synth(cfg["geom"])
        M0 = cfg["geom"].M[0]
        al = 2 * np.pi * np.arange(M0) / M0
        V = torch.as_tensor(0.1 * np.sin(al) + 0.03 * np.cos(2 * al))
        phi = torch.as_tensor(cfg["phi"])
        ref = O.solve_gamma_t(og, phi, V, 0.1)["gamma_t"]
        spreads = []
        orig = (B.K_block, B.G_block, B.spectral)
        for seed in (1, 2, 3):
            rng = np.random.default_rng(seed)
            B.K_block, B.G_block, B.spectral = (perturbed(f, rng) for f in orig)
            try:
                gt = O.solve_gamma_t(og, phi, V, 0.1)["gamma_t"]
            finally:
                B.K_block, B.G_block, B.spectral = orig
            spreads.append(float((gt - ref).abs().max() / ref.abs().max()))
            print(f"config {c} seed {seed}: {spreads[-1]:.3e}", flush=True)
        # omega (and U from it) perturbed by one unit of rounding per entry
        orig_solve = B.solve_phi
        om_spread = []
        for seed in (1, 2, 3):
            rng = np.random.default_rng(100 + seed)

            def solve_phi_pert(g, ph):
                r = orig_solve(g, ph)
                om = r["omega"] * (1.0 + 2.0 ** -53 * torch.as_tensor(
                    rng.standard_normal(r["omega"].shape[0])))
                return {**r, "omega": om, "U": B.dphi_dn_from_omega(g, B.split(g, om))}

            B.solve_phi = solve_phi_pert
            try:
                gt = O.solve_gamma_t(og, phi, V, 0.1)["gamma_t"]
            finally:
                B.solve_phi = orig_solve
            om_spread.append(float((gt - ref).abs().max() / ref.abs().max()))
            print(f"config {c} omega rounding seed {seed}: {om_spread[-1]:.3e}", flush=True)
        # the same gamma_t with both solves by GMRES to 1e-15

        def solve_phi_gmres(g, ph):
            A = B.assemble_A(g)
            b = B.rhs(g, ph)
            om, _, _ = B.gmres(lambda v: A @ v, b, tol=1e-15, restart=100)
            parts = B.split(g, om)
            return {"omega": om, "U": B.dphi_dn_from_omega(g, parts), "A": A, "b": b}

        B.solve_phi = solve_phi_gmres
        try:
            r = B.gamma_t_rhs(og, phi, V, 0.1)
        finally:
            B.solve_phi = orig_solve
        Bm = B.gamma_t_matrix(og)
        gt, _, _ = B.gmres(lambda v: Bm @ v, r["b"], tol=1e-15, restart=100)
        solver = float((gt - ref).abs().max() / ref.abs().max())
        print(f"config {c} GMRES vs refined dense solve: {solver:.3e}", flush=True)
        out[f"c{c}"] = {"M0": M0, "rel_change": spreads, "omega_rounding": om_spread,
                         "gmres_vs_lu": solver}
    out["command"] = "python tests/golden/gamma_t_spread.py"
    with open(os.path.join(HERE, "gamma_t_spread.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
