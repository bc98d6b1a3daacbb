"""Write the oracle's reference for the large cell (M = 40960: surface 16384,
bottom 8192, eight ellipses of 2048; seeded inputs of synth.make_config(5),
stage 0): tests/golden/large_M40960.npz and large_M40960.json.

Only oracle/ and synth/ are used.  The FP64 matrix of the collocated system
(Sec. 3.3) is assembled row block by row block (13.4 GB) and solved twice:

* by the oracle's restarted GMRES (unpreconditioned, CGS2, restart 120) to a
  relative true residual of 1e-15 -- the stored reference omega, U, psi|_k;
* by dense LU of the same matrix -- a second oracle solution whose distance
  to the first is recorded as the oracle-vs-oracle spread per output.

It then evaluates J = sum w U^2 (weights of synth.large_adjoint_draws) and
its derivatives along the 4 seeded directions by the tangent-linear model
on the surface's node data (tangent_J_nodes, with the LU factors as the
solver): each direction moves (x~, y, phi) and, with their exact
derivatives, (x', y', x'', y''), so no spectral derivative of the surface or
of the directions enters (at 16384 surface nodes the rounding of a spectral
second derivative alone reaches 1e-9).

Run from the repository root:  python tests/golden/make_large_golden.py
(about 40 minutes on 8 cores; peaks near 35 GB of host memory).
"""
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import large_adjoint_draws, make_config  # noqa: E402


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def main():
    t_all = time.time()
    cfg = make_config(5)
    geom = cfg["geom"]
    og = O.OGeom.from_synth(geom)
    phi = torch.as_tensor(np.asarray(cfg["phi"]))
    n, M0 = geom.Mtot, geom.M[0]
    meta = {"cell": f"synth.make_config(5) stage 0: M={n} (surface {M0}, bottom {geom.M[1]}, "
                    f"{geom.nb - 2} ellipses of {geom.M[2]})",
            "threads": torch.get_num_threads(), "command": "python tests/golden/make_large_golden.py"}

    t = time.time()
    A = O.assemble_A_blocked(og, chunk=512)
    meta["t_assemble_s"] = time.time() - t
    log(f"assembled {n}x{n} in {meta['t_assemble_s']:.0f} s")
    b = O.rhs(og, phi)

    t = time.time()
    x, hist, steps = O.gmres(lambda v: A @ v, b, tol=1e-15, restart=120, max_iter=1200)
    meta["t_gmres_s"] = time.time() - t
    meta["gmres"] = {"tol": 1e-15, "restart": 120, "steps": steps, "cycle_start_resid": hist}
    log(f"gmres {steps} steps in {meta['t_gmres_s']:.0f} s, history {hist}")
    res = float(torch.linalg.vector_norm(b - A @ x) / torch.linalg.vector_norm(b))
    meta["gmres"]["final_rel_resid"] = res

    t = time.time()
    lu, piv = torch.linalg.lu_factor(A)
    meta["t_lu_factor_s"] = time.time() - t
    log(f"LU factor in {meta['t_lu_factor_s']:.0f} s")

    def lu_solve(r):
        return torch.linalg.lu_solve(lu, piv, r[:, None])[:, 0]

    x_lu = lu_solve(b)
    meta["lu_rel_resid"] = float(torch.linalg.vector_norm(b - A @ x_lu) / torch.linalg.vector_norm(b))
    del A

    t = time.time()
    parts = O.split(og, x)
    U = O.dphi_dn_from_omega_chunked(og, parts)
    meta["t_U_s"] = time.time() - t
    U_lu = O.dphi_dn_from_omega_chunked(og, O.split(og, x_lu))
    psi = torch.stack([p.mean() for p in parts[2:]])
    psi_lu = torch.stack([p.mean() for p in O.split(og, x_lu)[2:]])
    meta["spread_gmres_vs_lu"] = {"omega": rel(x, x_lu), "U": rel(U, U_lu), "psi_k": rel(psi, psi_lu)}
    log(f"spread GMRES vs LU {meta['spread_gmres_vs_lu']}")

    adj = large_adjoint_draws(M0)
    dirs = []
    for d, dd in zip(adj["directions"], adj["derivatives"]):
        # (x, y, x', y', x'', y'', phi): x~ and y move with their derivatives
        dirs.append((d[0], d[1], dd[0][0], dd[1][0], dd[0][1], dd[1][1], d[2]))
    t = time.time()
    J, U_t, _, dJ, _ = O.tangent_J_nodes(og, np.asarray(cfg["phi"]), adj["weights"], dirs,
                                         lu_solve, omega=x, chunk=512)
    meta["t_tangent_s"] = time.time() - t
    meta["U_tangent_vs_U"] = rel(U_t, U)
    log(f"J {J:.17g} dJ {dJ} in {meta['t_tangent_s']:.0f} s")

    np.savez_compressed(os.path.join(HERE, "large_M40960.npz"), U=U.numpy(), omega=x.numpy(),
                        psi_k=psi.numpy(), J=np.array(J), dJ=np.array(dJ))
    meta["t_total_s"] = time.time() - t_all
    with open(os.path.join(HERE, "large_M40960.json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(f"done in {meta['t_total_s']:.0f} s")


if __name__ == "__main__":
    main()
