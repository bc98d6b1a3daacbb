"""Write the oracle's tangent-linear derivatives of U on the adjoint cell
(config 4: synth.make_config(4), M = 4608: surface 2048, bottom 1024, three
ellipses of 512) along 8 seeded directions of the surface's node data (x, y,
x', y', x'', y'') and phi~, walls fixed: tests/golden/tangent_c4.npz and
tangent_c4.json.

Each direction's seven components are independent smooth fields (Fourier
modes 0..8 with seeded normal coefficients decaying as 1/(1 + k), scaled to
a largest entry of 1); the tangent-linear model is defined for any such node
data.  They are stored with the result, so a test reads its inputs from
here.

Only oracle/ and synth/ are used: forward-mode autodiff through the oracle's
assembly and U map around its refined dense solve (oracle.tangent_J_nodes,
Sec. 3.2-3.4 differentiated), with J = sum w U^2 for the config's weights.

Run from the repository root:  python tests/golden/make_tangent_golden.py
(under a minute on 8 cores).
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
from synth import make_config  # noqa: E402

ND = 8


def smooth(rng, M, kmax=8):
    a = 2 * np.pi * np.arange(M) / M
    f = np.zeros(M)
    for k in range(kmax + 1):
        f += (rng.standard_normal() * np.cos(k * a) + rng.standard_normal() * np.sin(k * a)) / (1 + k)
    return f / np.abs(f).max()


def main():
    cfg = make_config(4)
    geom = cfg["geom"]
    M0 = geom.M[0]
    og = O.OGeom.from_synth(geom)
    rng = np.random.default_rng(4608)
    dirs = np.array([[smooth(rng, M0) for _ in range(7)] for _ in range(ND)])   # (ND, 7, M0)
    t = time.time()
    A = O.assemble_A(og)
    J, U, om, dJ, dU = O.tangent_J_nodes(og, np.asarray(cfg["phi"]), cfg["weights"],
                                         [tuple(d) for d in dirs], lambda r: O.dense_solve(A, r))
    np.savez_compressed(os.path.join(HERE, "tangent_c4.npz"), dirs=dirs,
                        dU=np.array([d.numpy() for d in dU]), dJ=np.array(dJ), U=U.numpy(),
                        J=np.array(J))
    meta = {"cell": "synth.make_config(4): M=4608 (surface 2048, bottom 1024, 3 ellipses of 512)",
            "directions": ND, "seed": 4608, "J": J, "dJ": dJ,
            "threads": torch.get_num_threads(), "t_s": time.time() - t,
            "command": "python tests/golden/make_tangent_golden.py"}
    with open(os.path.join(HERE, "tangent_c4.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta, indent=1))


if __name__ == "__main__":
    main()
