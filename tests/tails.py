"""Expected status of a velocity-potential solve under the Fourier-tail
resolution check (the paper's grid test, Sec. 7.1): WARN_UNDERRESOLVED when
the largest per-boundary tail ratio of omega exceeds max(1e-12, 10 tol)."""
import numpy as np
import torch

import oracle as O


def oracle_tail(geom, omega) -> float:
    """Largest tail ratio over the boundaries of an omega (oracle or GPU): the
    root of boundary k's tail energy over M_k^2 times the largest mean square of
    omega on any boundary (on the boundary carrying that mean square, the
    energy fraction of its own tail)."""
    w = torch.as_tensor(np.asarray(omega, dtype=np.float64))
    parts = torch.split(w, list(geom.M))
    total = [len(v) * float((v * v).sum()) for v in parts]       # FFT energy (Parseval)
    smax = max(t / len(v) ** 2 for t, v in zip(total, parts))
    if smax == 0.0:
        return 0.0
    return max(float(np.sqrt(O.spectral_tail(v) ** 2 * t / (smax * len(v) ** 2))) if t > 0 else 0.0
               for t, v in zip(total, parts))


def check_tail_status(ww, rep, tol, ref_tail):
    """rep.tail_ratio agrees with the oracle's measure where the tail stands
    above the rounding of omega, and the status follows the threshold."""
    thr = max(1e-12, 10 * tol)
    if ref_tail > 1e-10:
        assert abs(rep.tail_ratio / ref_tail - 1.0) <= 1e-4, (rep.tail_ratio, ref_tail)
    else:
        assert rep.tail_ratio <= 1e-10, rep.tail_ratio
    if ref_tail > 10 * thr:
        assert rep.status == ww.WARN_UNDERRESOLVED
    elif ref_tail < 0.1 * thr:
        assert rep.status == ww.OK
    expect = ww.WARN_UNDERRESOLVED if rep.tail_ratio > thr else ww.OK
    assert rep.status == expect, (rep.status, rep.tail_ratio, thr)
