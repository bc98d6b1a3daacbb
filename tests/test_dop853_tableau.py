"""The DOP853 tableau the RK-step tests and the bench run (tests/golden/
dop853_tableau.json; Hairer, Norsett and Wanner, Sec. II.10): explicit,
consistent (c_i = sum_j a_ij, sum b = 1, the quadrature conditions
sum b c^(k-1) = 1/k through k = 8), and of order eight on a nonlinear
system, which checks every order condition at once: halving the step cuts
the global error by about 2^8."""
import json
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dop853_tableau.json")


def _tableau():
    d = json.load(open(PATH))
    return np.array(d["A"]), np.array(d["b"]), np.array(d["c"])


def test_tableau_is_explicit_and_consistent():
    A, b, c = _tableau()
    assert A.shape == (12, 12) and np.all(np.triu(A) == 0.0)
    assert np.abs(A.sum(axis=1) - c).max() < 1e-14
    for k in range(1, 9):
        assert abs(b @ c ** (k - 1) - 1.0 / k) < 1e-14, k


def _integrate(A, b, c, f, y0, T, N):
    h, y, t = T / N, np.array(y0, dtype=float), 0.0
    s = len(b)
    for _ in range(N):
        K = np.zeros((s, y.size))
        for i in range(s):
            K[i] = f(t + c[i] * h, y + h * (A[i, :i] @ K[:i]))
        y = y + h * (b @ K)
        t += h
    return y


def test_order_eight_on_a_nonlinear_system():
    """Van der Pol with mu = 1/2 over one unit of time: the error against a
    32-times finer solution of the same method shrinks about 2^8-fold when
    4 steps become 8 (2.9e-13 at 8 steps, well above rounding)."""
    A, b, c = _tableau()
    f = lambda t, y: np.array([y[1], -y[0] + 0.5 * (1.0 - y[0] ** 2) * y[1]])
    ref = _integrate(A, b, c, f, [2.0, 0.0], 1.0, 256)
    errs = [np.abs(_integrate(A, b, c, f, [2.0, 0.0], 1.0, N) - ref).max() for N in (4, 8)]
    order = np.log2(errs[0] / errs[1])
    assert 7.5 < order < 8.7, (errs, order)
