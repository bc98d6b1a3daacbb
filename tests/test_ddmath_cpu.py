"""The double-double E = e^{i zeta} = e^{-y}(cos x + i sin x) of the node
preparation, built for the host from the same header the kernels include,
against 60-digit decimal arithmetic (pi by Machin's formula, sin and cos by
their Taylor series after reduction by 2 pi, exp from the decimal module).

The kernel entries form E_q - E_p from both parts, so the trailing part must
carry E to about 1e-30 relative: then the difference of two nodes 1e-6 apart
still has a relative error near 1e-24 from E alone.
"""
import ctypes
import os
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "dd_expi_host.hip")
HDR = os.path.join(ROOT, "paper_2108_01786_amd", "csrc", "ddmath.h")
LIB = os.path.join(ROOT, "_build", "libdd_expi_host.so")

getcontext().prec = 60


def _pi():
    def atan_inv(n):
        x = Decimal(1) / n
        x2, t, s, k = x * x, x, Decimal(0), 0
        while True:
            term = t / (2 * k + 1)
            if term < Decimal(10) ** -58:
                return s
            s += term if k % 2 == 0 else -term
            t *= x2
            k += 1
    return 4 * (4 * atan_inv(5) - atan_inv(239))


PI = _pi()


def _sincos(x: Decimal):
    x = x - (2 * PI) * (x / (2 * PI)).to_integral_value()
    s, c, t, n = Decimal(0), Decimal(0), Decimal(1), 0
    while True:                 # t = x^n / n!
        if abs(t) < Decimal(10) ** -58 and n > 2:
            return s, c
        if n % 4 == 0:
            c += t
        elif n % 4 == 1:
            s += t
        elif n % 4 == 2:
            c -= t
        else:
            s -= t
        n += 1
        t = t * x / n


@pytest.fixture(scope="module")
def lib():
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    stale = (not os.path.exists(LIB)
             or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(HDR)))
    if stale:
        subprocess.run(["/opt/rocm/bin/hipcc", "--cuda-host-only", "-x", "hip", "-O2",
                        "-std=c++17", "-shared", "-fPIC", SRC, "-o", LIB], check=True)
    h = ctypes.CDLL(LIB)
    h.dd_expi_host.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    return h


def _dd(lib, x, y):
    out = (ctypes.c_double * 4)()
    lib.dd_expi_host(x, y, out)
    return out[0], out[1], out[2], out[3]


def test_dd_expi_against_decimal(lib):
    rng = np.random.default_rng(3)
    xs = list(rng.uniform(-10.0, 20.0, 60)) + [0.0, 1e-9, np.pi / 2, -np.pi, 2 * np.pi, 7.85398,
                                              3.92699, 1e5 + 0.3]
    ys = list(rng.uniform(-30.0, 30.0, 60)) + [0.0, -1e-12, 0.5, 30.0, -30.0, 1.0, -3.0, 0.2]
    worst = 0.0
    for x, y in zip(xs, ys):
        rh, rl, ih, il = _dd(lib, float(x), float(y))
        s, c = _sincos(Decimal(float(x)))
        m = (-Decimal(float(y))).exp()
        er, ei = m * c, m * s
        err = max(abs(Decimal(rh) + Decimal(rl) - er), abs(Decimal(ih) + Decimal(il) - ei))
        rel = float(err / m)
        worst = max(worst, rel)
        # the leading parts alone are the correctly rounded FP64 values up to an ulp
        assert abs(rh - float(er)) <= 2.3e-16 * float(m) and abs(ih - float(ei)) <= 2.3e-16 * float(m)
    assert worst < 1e-30, worst


def test_dd_difference_of_nearby_nodes(lib):
    """(E_q - E_p) formed from both parts, as the kernel entries form it,
    against the decimal difference for nodes 1e-7 to 1e-2 apart."""
    rng = np.random.default_rng(4)
    for _ in range(40):
        x, y = rng.uniform(0, 2 * np.pi), rng.uniform(-1.5, 1.5)
        d = 10.0 ** rng.uniform(-7, -2)
        th = rng.uniform(0, 2 * np.pi)
        xq, yq = x + d * np.cos(th), y + d * np.sin(th)
        p, q = _dd(lib, x, y), _dd(lib, xq, yq)
        dr = (q[0] - p[0]) + (q[1] - p[1])
        di = (q[2] - p[2]) + (q[3] - p[3])
        sp, cp = _sincos(Decimal(x))
        sq, cq = _sincos(Decimal(float(xq)))
        mp, mq = (-Decimal(y)).exp(), (-Decimal(float(yq))).exp()
        er, ei = mq * cq - mp * cp, mq * sq - mp * sp
        mag = (er * er + ei * ei).sqrt()
        err = float(max(abs(Decimal(dr) - er), abs(Decimal(di) - ei)) / mag)
        assert err < 4e-16, (d, err)
