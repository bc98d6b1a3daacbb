"""Closed-form boundary curves sampled on uniform grids (FP64, numpy).

Every boundary k is sampled at alpha_{k,m} = 2*pi*m/M_k, m = 0..M_k-1
(Sec. 3.3, numerical discretization).  Curves are described by their complex
position zeta = xi + i*eta and the exact first and second alpha-derivatives,
so that no numerical differentiation enters the inputs.

Orientation contract (Sec. 2): the free surface and the bottom run left to
right with zeta(alpha + 2*pi) = zeta(alpha) + 2*pi; obstacles are closed
curves traversed clockwise so that the fluid lies on their left.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np


def grid(M: int) -> np.ndarray:
    """Uniform periodic grid alpha_m = 2*pi*m/M."""
    return 2.0 * np.pi * np.arange(M, dtype=np.float64) / M


@dataclass
class Curve:
    """One sampled boundary: position and its first two alpha-derivatives."""
    z: np.ndarray   # complex128, zeta(alpha_m)
    d: np.ndarray   # complex128, zeta'(alpha_m)
    e: np.ndarray   # complex128, zeta''(alpha_m)

    @property
    def M(self) -> int:
        return int(self.z.shape[0])


def fourier_surface(M: int, a1: float, coeffs: Sequence[complex], k0: int = 2) -> Curve:
    """zeta(alpha) = alpha + i*(a1*cos(alpha) + sum_k c_k e^{i k alpha}), k = k0, k0+1, ...

    The complex coefficients make the curve a general (non-graph)
    parameterization: xi = alpha - sum Im(c_k e^{ik alpha}),
    eta = a1 cos(alpha) + sum Re(c_k e^{ik alpha}).
    """
    al = grid(M)
    z = al + 1j * a1 * np.cos(al)
    d = 1.0 - 1j * a1 * np.sin(al)
    e = -1j * a1 * np.cos(al)
    for n, c in enumerate(coeffs):
        k = k0 + n
        ph = c * np.exp(1j * k * al)
        z = z + 1j * ph
        d = d + 1j * (1j * k) * ph
        e = e + 1j * (1j * k) ** 2 * ph
    return Curve(z.astype(np.complex128), d.astype(np.complex128), e.astype(np.complex128))


def graph_bottom(M: int, h0: float, cos_terms: Sequence[Tuple[int, float]] = ()) -> Curve:
    """zeta(alpha) = alpha + i*(h0 + sum_j b_j cos(k_j alpha)), run left to right."""
    al = grid(M)
    eta = np.full(M, h0, dtype=np.float64)
    deta = np.zeros(M)
    ddeta = np.zeros(M)
    for k, b in cos_terms:
        eta = eta + b * np.cos(k * al)
        deta = deta - b * k * np.sin(k * al)
        ddeta = ddeta - b * k * k * np.cos(k * al)
    z = al + 1j * eta
    d = 1.0 + 1j * deta
    e = 1j * ddeta
    return Curve(z, d, e)


def ellipse(M: int, cx: float, cy: float, q: float, b: float, theta: float,
            clockwise: bool = True) -> Curve:
    """zeta(alpha) = c + e^{i theta} (q cos(alpha) - i b sin(alpha)) (clockwise).

    With clockwise=False the sign of the sin term flips, giving the
    counter-clockwise curve (used only to exercise input validation).
    """
    al = grid(M)
    sgn = -1.0 if clockwise else 1.0
    rot = np.exp(1j * theta)
    c = cx + 1j * cy
    z = c + rot * (q * np.cos(al) + sgn * 1j * b * np.sin(al))
    d = rot * (-q * np.sin(al) + sgn * 1j * b * np.cos(al))
    e = rot * (-q * np.cos(al) - sgn * 1j * b * np.sin(al))
    return Curve(z, d, e)


def clustered_flat_surface(M: int, x0: float, beta: float, h: float = 0.0) -> Curve:
    """zeta(alpha) = alpha + beta sin(alpha - x0) ... reparameterised flat line
    y = h whose nodes cluster around x = x0: xi(alpha) = alpha - beta sin(alpha - x0)
    with 0 <= beta < 1, so xi' = 1 - beta cos(alpha - x0) is smallest (1 - beta)
    at alpha = x0 and the curve still runs left to right (Sec. 2 allows any
    parameterisation of the surface)."""
    al = grid(M)
    s, c = np.sin(al - x0), np.cos(al - x0)
    z = al - beta * s + 1j * h
    d = (1.0 - beta * c) + 0j
    e = beta * s + 0j
    return Curve(z.astype(np.complex128), d.astype(np.complex128), e.astype(np.complex128))


def clustered_ellipse(M: int, cx: float, cy: float, q: float, b: float, theta_c: float,
                      gamma: float) -> Curve:
    """The clockwise ellipse c + q cos(t) - i b sin(t) with its parameter t(alpha)
    = alpha - gamma sin(alpha - theta_c), 0 <= gamma < 1: nodes cluster around
    t = theta_c (t' = 1 - gamma cos(alpha - theta_c))."""
    al = grid(M)
    t = al - gamma * np.sin(al - theta_c)
    t1 = 1.0 - gamma * np.cos(al - theta_c)
    t2 = gamma * np.sin(al - theta_c)
    w = q * np.cos(t) - 1j * b * np.sin(t)
    w1 = -q * np.sin(t) - 1j * b * np.cos(t)      # d/dt
    w2 = -q * np.cos(t) + 1j * b * np.sin(t)      # d2/dt2
    z = (cx + 1j * cy) + w
    d = w1 * t1
    e = w2 * t1 * t1 + w1 * t2
    return Curve(z.astype(np.complex128), d.astype(np.complex128), e.astype(np.complex128))


def trig_potential(M: int, A: Sequence[float], B: Sequence[float]) -> np.ndarray:
    """phi(alpha) = sum_{k>=1} A_k cos(k alpha) + B_k sin(k alpha)."""
    al = grid(M)
    out = np.zeros(M)
    for k, (ak, bk) in enumerate(zip(A, B), start=1):
        out = out + ak * np.cos(k * al) + bk * np.sin(k * al)
    return out


@dataclass
class Geometry:
    """All boundaries of one periodic cell plus the multi-valued flow data.

    Boundary 0 is the free surface, 1 the bottom, 2..N the obstacles.  Node
    arrays are concatenated boundary by boundary.  ``zc[j-2]`` is the point
    z_j inside obstacle j and ``a[j-2]`` its circulation parameter a_j; V1 is
    the background-flow strength (Sec. 3, decomposition of Phi).
    ``psi_wall`` optionally prescribes stream-function data on the walls
    (nodes of boundaries 1..N, concatenated); None means zero.
    """
    curves: List[Curve]
    zc: np.ndarray                      # complex128, (N-1,)
    a: np.ndarray                       # float64, (N-1,)
    V1: float = 1.0
    psi_wall: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> List[int]:
        return [c.M for c in self.curves]

    @property
    def nb(self) -> int:
        return len(self.curves)

    @property
    def Mtot(self) -> int:
        return int(sum(self.M))

    def cat(self, attr: str) -> np.ndarray:
        return np.concatenate([getattr(c, attr) for c in self.curves])

    def arrays(self) -> dict:
        """FP64 structure-of-arrays view: x, y, dx, dy, ddx, ddy (concatenated)."""
        z, d, e = self.cat("z"), self.cat("d"), self.cat("e")
        return {
            "x": np.ascontiguousarray(z.real), "y": np.ascontiguousarray(z.imag),
            "dx": np.ascontiguousarray(d.real), "dy": np.ascontiguousarray(d.imag),
            "ddx": np.ascontiguousarray(e.real), "ddy": np.ascontiguousarray(e.imag),
        }

    def min_clearance(self) -> float:
        """Smallest node distance between different boundaries (with +-2pi images)."""
        best = np.inf
        for i in range(self.nb):
            for j in range(i + 1, self.nb):
                zi, zj = self.curves[i].z, self.curves[j].z
                for s in (-2 * np.pi, 0.0, 2 * np.pi):
                    dmin = np.abs(zi[:, None] - (zj[None, :] + s)).min()
                    best = min(best, dmin)
        return float(best)
