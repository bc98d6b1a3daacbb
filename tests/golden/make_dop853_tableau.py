"""Write tests/golden/dop853_tableau.json: the explicit 12-stage Runge-Kutta
tableau (A, b, c) of Dormand and Prince's eighth-order method DOP853, as
published by Hairer, Norsett and Wanner (Solving Ordinary Differential
Equations I, 2nd ed., Springer 1993, Sec. II.10, and their DOP853 code).

The numbers are taken once from SciPy's transcription of that code (a
private module, read here at generation time only); the tests and the bench
read the JSON file, and tests/test_dop853_tableau.py pins it by its order of
convergence.

Run from the repository root:  python tests/golden/make_dop853_tableau.py
"""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    from scipy.integrate._ivp import dop853_coefficients as d
    n = d.N_STAGES
    A = np.array(d.A[:n, :n], dtype=np.float64)
    b = np.array(d.B[:n], dtype=np.float64)
    c = np.array(d.C[:n], dtype=np.float64)
    out = {"method": "DOP853 (Dormand-Prince 8(5,3)), the 12 stages of the 8th-order solution",
           "source": "Hairer, Norsett, Wanner, Solving ODEs I (2nd ed., 1993), Sec. II.10",
           "stages": n, "A": A.tolist(), "b": b.tolist(), "c": c.tolist(),
           "command": "python tests/golden/make_dop853_tableau.py"}
    with open(os.path.join(HERE, "dop853_tableau.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
