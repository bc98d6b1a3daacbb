"""Write the oracle's gradient of J = sum w U^2 on the adjoint cell (config 4:
synth.make_config(4), M = 4608: surface 2048, bottom 1024, three ellipses of
512; weights w_m ~ U[0, 1] from the config's draws) with respect to the
surface's node data (x, y, x', y', x'', y'') and phi~, walls fixed:
tests/golden/adjoint_c4.npz and adjoint_c4.json.

Only oracle/ and synth/ are used: reverse-mode autograd through the dense
FP64 solve (oracle.J_and_grad_nodes, Sec. 3.2-3.4).

Run from the repository root:  python tests/golden/make_adjoint_golden.py
(a few minutes on 8 cores; peaks near 20 GB of host memory).
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


def main():
    cfg = make_config(4)
    og = O.OGeom.from_synth(cfg["geom"])
    t = time.time()
    J, grads, U = O.J_and_grad_nodes(og, np.asarray(cfg["phi"]), cfg["weights"])
    names = ["x", "y", "dx", "dy", "ddx", "ddy", "phi"]
    np.savez_compressed(os.path.join(HERE, "adjoint_c4.npz"), J=np.array(J), U=U.numpy(),
                        **{f"g_{k}": g.numpy() for k, g in zip(names, grads)})
    meta = {"cell": "synth.make_config(4): M=4608 (surface 2048, bottom 1024, 3 ellipses of 512)",
            "J": J, "threads": torch.get_num_threads(), "t_s": time.time() - t,
            "command": "python tests/golden/make_adjoint_golden.py"}
    with open(os.path.join(HERE, "adjoint_c4.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(f"J {J:.17g} in {meta['t_s']:.0f} s", flush=True)


if __name__ == "__main__":
    main()
