"""Seeded workloads.

Each config is drawn from ``numpy.random.default_rng(178600 + c)`` with the
draws taken in the order the boundaries are listed (surface, bottom,
obstacles, circulations, surface potential).  Ellipse draws that come closer
than the stated clearance to any other boundary (including the +-2pi images)
are redrawn from the same stream.

The paper's own test problems (Sec. 7.1, ellipse table and the three
choices of V1, a_j) are provided by ``paper_problem`` at t = 0: flat free
surface, zero surface potential, flat bottom y = -3.  The printed ellipse
parameterization has no centre and runs counter-clockwise; the curves here
are centred at (x_j, y_j) and run clockwise, as the orientation contract of
Sec. 2 requires.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .geometry import (Curve, Geometry, ellipse, fourier_surface, graph_bottom,
                       grid, trig_potential)

CONFIG_NAMES = {
    1: "fp64-cpu-sized M=640",
    2: "fp64-gpu M=4608",
    3: "refined-fp32 M=10240",
    4: "adjoint M=4608",
    5: "large M=40960",
}

_CLEAR_RES = 512   # resolution at which candidate ellipses are checked


def _clearance(a: Curve, b: Curve) -> float:
    za = a.z if a.M <= 2048 else a.z[:: a.M // 2048]
    zb = b.z if b.M <= 2048 else b.z[:: b.M // 2048]
    best = np.inf
    for s in (-2 * np.pi, 0.0, 2 * np.pi):
        best = min(best, float(np.abs(za[:, None] - (zb[None, :] + s)).min()))
    return best


def _phi_law(rng, M0: int) -> np.ndarray:
    A = 0.1 * rng.standard_normal(3)
    B = 0.1 * rng.standard_normal(3)
    return trig_potential(M0, A, B), (A, B)


def _draw_ellipses(rng, n, fixed: List[Curve], M_ell: int, cx_jit, cy_rng, ab_rng,
                   delta: float) -> Tuple[List[Curve], List[complex], list]:
    out, centres, params = [], [], []
    for jj in range(n):
        for attempt in range(1000):
            cx = 2 * np.pi * (jj + 0.5) / n + rng.uniform(-cx_jit, cx_jit)
            cy = rng.uniform(*cy_rng)
            q = rng.uniform(*ab_rng)
            b = rng.uniform(*ab_rng)
            th = rng.uniform(0.0, np.pi)
            cand = ellipse(_CLEAR_RES, cx, cy, q, b, th)
            others = [c for c in fixed] + [ellipse(_CLEAR_RES, *p) for p in params]
            if all(_clearance(cand, o) >= delta for o in others):
                break
        else:
            raise RuntimeError("could not place ellipse with the requested clearance")
        params.append((cx, cy, q, b, th))
        centres.append(cx + 1j * cy)
        out.append(ellipse(M_ell, cx, cy, q, b, th))
    return out, centres, params


def _config1_draws(rng):
    g = rng.standard_normal(15)
    h = rng.standard_normal(15)
    ks = np.arange(2, 17)
    coeffs = 0.01 * np.exp(-ks / 4.0) * (g + 1j * h)
    A = 0.1 * rng.standard_normal(3)
    B = 0.1 * rng.standard_normal(3)
    return coeffs, A, B


def make_config(c: int) -> Dict:
    """Return {'geom': Geometry, 'phi': surface potential, ...} for config c."""
    rng = np.random.default_rng(178600 + c)
    if c == 1:
        coeffs, A, B = _config1_draws(rng)
        surf = fourier_surface(256, 0.1, coeffs)
        bot = graph_bottom(256, -1.0)
        ell = ellipse(128, np.pi, -0.5, 0.3, 0.15, 0.0)
        geom = Geometry([surf, bot, ell], np.array([np.pi - 0.5j]), np.array([0.5]), 1.0,
                        meta={"config": 1})
        return {"geom": geom, "phi": trig_potential(256, A, B), "tol": 1e-13}
    if c in (2, 4):
        rng = np.random.default_rng(178602)
        g = rng.standard_normal(15)
        h = rng.standard_normal(15)
        ks = np.arange(2, 17)
        coeffs = 0.015 * np.exp(-ks / 4.0) * (g + 1j * h)
        surf = fourier_surface(2048, 0.15, coeffs)
        bot = graph_bottom(1024, -1.0, [(1, 0.1)])
        fixed = [fourier_surface(_CLEAR_RES, 0.15, coeffs), graph_bottom(_CLEAR_RES, -1.0, [(1, 0.1)])]
        ells, centres, params = _draw_ellipses(rng, 3, fixed, 512, 0.3, (-0.8, -0.3), (0.1, 0.3), 0.1)
        a = rng.uniform(-1.0, 1.0, 3)
        phi, _ = _phi_law(rng, 2048)
        geom = Geometry([surf, bot] + ells, np.array(centres), a, 1.0,
                        meta={"config": c, "ellipses": params})
        out = {"geom": geom, "phi": phi, "tol": 1e-13}
        if c == 4:
            out.update(_adjoint_draws(2048))
        return out
    if c == 3:
        rng1 = np.random.default_rng(178601)
        coeffs, A, B = _config1_draws(rng1)
        surf = fourier_surface(4096, 0.1, coeffs)
        bot = graph_bottom(2048, -1.0)
        ells = [ellipse(1024, (2 * m + 1) * np.pi / 4, -0.5, 0.3, 0.15, 0.0) for m in range(4)]
        centres = np.array([(2 * m + 1) * np.pi / 4 - 0.5j for m in range(4)])
        geom = Geometry([surf, bot] + ells, centres, np.full(4, 0.5), 1.0, meta={"config": 3})
        return {"geom": geom, "phi": trig_potential(4096, A, B), "tol": 1e-12}
    if c == 5:
        return _config5(rng)
    raise ValueError(f"unknown config {c}")


def _smooth_field(rng, M: int, K: int, decay: float) -> np.ndarray:
    al = grid(M)
    ks = np.arange(1, K + 1)
    cc = rng.standard_normal(K)
    ss = rng.standard_normal(K)
    w = np.exp(-ks / decay)
    f = (w[None, :] * (cc[None, :] * np.cos(np.outer(al, ks)) + ss[None, :] * np.sin(np.outer(al, ks)))).sum(1)
    return f


def _smooth_field3(rng, M: int, K: int, decay: float):
    """The field of _smooth_field (same draws) with its exact first and second
    alpha-derivatives."""
    al = grid(M)
    ks = np.arange(1, K + 1)
    cc = rng.standard_normal(K)
    ss = rng.standard_normal(K)
    w = np.exp(-ks / decay)
    c, s = np.cos(np.outer(al, ks)), np.sin(np.outer(al, ks))
    f = (w * (cc * c + ss * s)).sum(1)
    f1 = (w * ks * (-cc * s + ss * c)).sum(1)
    f2 = (w * ks * ks * (-cc * c - ss * s)).sum(1)
    return f, f1, f2


def _adjoint_draws(M0: int) -> Dict:
    """Weights w_m ~ U[0,1] and 32 smooth directions (x~, y, phi), max-norm 1."""
    rng = np.random.default_rng(178604)
    w = rng.uniform(0.0, 1.0, M0)
    dirs = []
    for _ in range(32):
        comps = []
        for _c in range(3):
            f = _smooth_field(rng, M0, 16, 4.0)
            comps.append(f / np.abs(f).max())
        dirs.append(np.stack(comps))
    return {"weights": w, "directions": np.stack(dirs), "fd_h": 1e-6}


def large_adjoint_draws(M0: int = 16384) -> Dict:
    """Weights and directions of J = sum w U^2 on the large cell: w_m ~ U[0, 1]
    from seed 178605, and 4 directions (x~, y, phi), each component
    sum_{k=1..32} e^{-k/8}(N cos k alpha + N sin k alpha) scaled to max-norm 1,
    from seed 178615.  `derivatives` holds, per direction and component, the
    exact first and second alpha-derivatives (same scale), so that a
    direction of the surface nodes (zeta, zeta', zeta'') needs no numerical
    differentiation."""
    w = np.random.default_rng(178605).uniform(0.0, 1.0, M0)
    rng = np.random.default_rng(178615)
    dirs, ders = [], []
    for _ in range(4):
        comps, cd = [], []
        for _c in range(3):
            f, f1, f2 = _smooth_field3(rng, M0, 32, 8.0)
            sc = np.abs(f).max()
            comps.append(f / sc)
            cd.append(np.stack([f1 / sc, f2 / sc]))
        dirs.append(np.stack(comps))
        ders.append(np.stack(cd))
    return {"weights": w, "directions": np.stack(dirs), "derivatives": np.stack(ders)}


def _config5(rng) -> Dict:
    g = rng.standard_normal(31)
    h = rng.standard_normal(31)
    ks = np.arange(2, 33)
    base = np.exp(-ks / 8.0) * (g + 1j * h)
    # xi' = 1 - sum_k k Re(c_k e^{ik alpha}); choose sigma so that min xi' = 0.15
    al = grid(1 << 16)
    xip = (ks[None, :] * (base[None, :] * np.exp(1j * np.outer(al, ks))).real).sum(1)
    sigma = 0.85 / xip.max()
    coeffs = sigma * base
    surf = fourier_surface(16384, 0.2, coeffs)
    bot_terms = [(1, 0.15), (3, 0.05)]
    bot = graph_bottom(8192, -1.0, bot_terms)
    fixed = [fourier_surface(_CLEAR_RES * 4, 0.2, coeffs), graph_bottom(_CLEAR_RES, -1.0, bot_terms)]
    ells, centres, params = _draw_ellipses(rng, 8, fixed, 2048, 0.1, (-0.75, -0.45), (0.08, 0.2), 0.08)
    a = rng.uniform(-1.0, 1.0, 8)
    phi, _ = _phi_law(rng, 16384)
    # smooth per-stage displacement fields of degree <= 32 for (x~, y, phi)
    disp = np.stack([_smooth_field(rng, 16384, 32, 8.0) for _ in range(3)])
    geom = Geometry([surf, bot] + ells, np.array(centres), a, 1.0,
                    meta={"config": 5, "sigma": sigma, "ellipses": params})
    return {"geom": geom, "phi": phi, "tol": 1e-12, "stage_disp": disp, "surface_coeffs": coeffs}


def paper_problem(n: int, M0: int = 256, M1: int = 96, Mj: int = 128) -> Dict:
    """Problems 1-3 of Sec. 7.1 at t = 0 (flat surface, phi = 0, bottom y = -3)."""
    table = [(np.pi, -1.00, 0.5, 0.5, 0.0), (4.0, -1.75, 0.6, 0.4, 1.0), (2.3, -1.60, 0.7, 0.3, -0.5)]
    a2 = {1: -1.0, 2: 0.0, 3: 1.0}[n]
    surf = fourier_surface(M0, 0.0, [])
    bot = graph_bottom(M1, -3.0)
    ells = [ellipse(Mj, *p) for p in table]
    centres = np.array([p[0] + 1j * p[1] for p in table])
    geom = Geometry([surf, bot] + ells, centres, np.array([a2, 0.0, 0.0]), 1.0,
                    meta={"problem": n})
    return {"geom": geom, "phi": np.zeros(M0), "tau": 0.1, "g": 1.0}


def tiny_config(M0: int = 32, M1: int = 32, M2: int = 16) -> Dict:
    """A coarse single-obstacle cell for gradient checks."""
    rng = np.random.default_rng(178610)
    coeffs = 0.01 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
    surf = fourier_surface(M0, 0.1, coeffs)
    bot = graph_bottom(M1, -1.0)
    ell = ellipse(M2, np.pi, -0.5, 0.3, 0.15, 0.0)
    phi = trig_potential(M0, 0.1 * rng.standard_normal(2), 0.1 * rng.standard_normal(2))
    geom = Geometry([surf, bot, ell], np.array([np.pi - 0.5j]), np.array([0.5]), 1.0,
                    meta={"config": "tiny", "surface_coeffs": coeffs})
    return {"geom": geom, "phi": phi, "surface_coeffs": coeffs}


def ragged_config() -> Dict:
    """Sizes that are not multiples of any tile (M = 250 + 126 + 66 + 58 = 500)."""
    rng = np.random.default_rng(178611)
    g = rng.standard_normal(6)
    h = rng.standard_normal(6)
    coeffs = 0.012 * np.exp(-np.arange(2, 8) / 4.0) * (g + 1j * h)
    surf = fourier_surface(250, 0.12, coeffs)
    bot = graph_bottom(126, -1.0, [(1, 0.08)])
    e2 = ellipse(66, 2.0, -0.55, 0.25, 0.12, 0.4)
    e3 = ellipse(58, 4.6, -0.6, 0.2, 0.15, 2.0)
    phi, _ = _phi_law(rng, 250)
    geom = Geometry([surf, bot, e2, e3], np.array([2.0 - 0.55j, 4.6 - 0.6j]),
                    np.array([0.7, -0.4]), 1.0, meta={"config": "ragged"})
    return {"geom": geom, "phi": phi, "tol": 1e-13}
