"""Closed-form flows used as pins (test helpers; independent of oracle and GPU code).

Manufactured periodic flow.  Pick
    Phi_exact(z) = V1 z + sum_j a_j Phi_cyl(z - w_j) + F(z),
with w_j any point inside obstacle j and F single-valued, 2pi-periodic and
holomorphic on the closed fluid cell.  With the solver's own points z_j the
difference Phi_exact - Phi_mv is single-valued in the fluid, so the layer
potentials can represent it.  Feeding
    phi~ = Re(Phi_exact - Phi_mv) on the surface,
    g_k  = Im Phi_exact - c_k on wall k (c_1 = 0)
must give U = Re{Phi_exact'(zeta) i zeta'}/|zeta'|, psi|_k = c_k and, on every
boundary, dphi/ds = Re{Phi_exact'(zeta) zeta'}/|zeta'|.

Flat strip of depth h with no obstacles: phi~ = cos(k alpha) on y = 0 gives
U = k tanh(k h) cos(k alpha) (the finite-depth Dirichlet-Neumann operator).
"""
from __future__ import annotations

import numpy as np

from synth.geometry import Geometry, ellipse, fourier_surface, graph_bottom, grid


def phi_cyl(z):
    """-i Log(1 - e^{iz}), principal branch (continuous where Im z > 0)."""
    return -1j * np.log(1.0 - np.exp(1j * z))


def dphi_cyl(z):
    return 0.5 - 0.5j / np.tan(0.5 * z)


class Flow:
    def __init__(self, V1, a, w, c_cot=0.0, p_cot=None, c_exp=0.0, c_low=0.0, q_low=None):
        self.V1, self.a, self.w = V1, np.asarray(a, float), np.asarray(w, complex)
        self.c_cot, self.p_cot = c_cot, p_cot
        self.c_exp = c_exp
        self.c_low, self.q_low = c_low, q_low

    def F(self, z):
        out = np.zeros_like(z, dtype=complex)
        if self.c_cot:
            out += self.c_cot * 0.5 / np.tan(0.5 * (z - self.p_cot))
        if self.c_exp:
            out += self.c_exp * np.exp(-1j * z)
        if self.c_low:
            out += self.c_low * phi_cyl(z - self.q_low)
        return out

    def dF(self, z):
        out = np.zeros_like(z, dtype=complex)
        if self.c_cot:
            out += -self.c_cot * 0.25 / np.sin(0.5 * (z - self.p_cot)) ** 2
        if self.c_exp:
            out += -1j * self.c_exp * np.exp(-1j * z)
        if self.c_low:
            out += self.c_low * dphi_cyl(z - self.q_low)
        return out

    def psi(self, z):
        """Im Phi_exact: single valued (Im Phi_cyl = -ln|1 - e^{iz}|)."""
        out = self.V1 * z.imag + self.F(z).imag
        for aj, wj in zip(self.a, self.w):
            out = out - aj * np.log(np.abs(1.0 - np.exp(1j * (z - wj))))
        return out

    def dPhi(self, z):
        out = self.V1 + self.dF(z)
        for aj, wj in zip(self.a, self.w):
            out = out + aj * dphi_cyl(z - wj)
        return out


def manufactured_inputs(geom: Geometry, flow: Flow, consts):
    """Return (phi~, psi_wall, U_exact, psi_k_exact) for the solver's geometry."""
    z0 = geom.curves[0].z
    d0 = geom.curves[0].d
    # phi~ = Re(Phi_exact - Phi_mv): the V1 z terms cancel; the log terms pair up
    diff = flow.F(z0)
    for aj, wj, zj in zip(geom.a, flow.w, geom.zc):
        diff = diff + aj * (phi_cyl(z0 - wj) - phi_cyl(z0 - zj))
    phi = diff.real
    walls = []
    for k, c in enumerate(geom.curves[1:], start=1):
        ck = 0.0 if k == 1 else consts[k - 2]
        walls.append(flow.psi(c.z) - ck)
    U = (flow.dPhi(z0) * 1j * d0).real / np.abs(d0)
    return phi, np.concatenate(walls), U, np.asarray(consts, float)


def exact_dphi_ds(geom: Geometry, flow: Flow):
    """dphi/ds = Re{Phi_exact'(zeta) zeta'}/|zeta'| on every boundary, concatenated."""
    return np.concatenate([(flow.dPhi(c.z) * c.d).real / np.abs(c.d) for c in geom.curves])


CASE_FLOW = Flow(1.0, [0.5], [np.pi + 0.06 - 0.47j], c_cot=0.07, p_cot=np.pi - 0.05 - 0.52j,
                 c_exp=0.03, c_low=0.2, q_low=0.4 - 1.6j)


def manufactured_case(M0=256, M1=256, M2=128, with_psi_wall=True):
    """Config-1-like cell with an off-centre vortex, a cot pole inside the
    ellipse, e^{-iz} and a log-sin source below the bottom (flow CASE_FLOW)."""
    rng = np.random.default_rng(7)
    coeffs = 0.01 * np.exp(-np.arange(2, 8) / 4.0) * (rng.standard_normal(6) + 1j * rng.standard_normal(6))
    surf = fourier_surface(M0, 0.1, coeffs)
    bot = graph_bottom(M1, -1.0, [(1, 0.05)])
    ell = ellipse(M2, np.pi, -0.5, 0.3, 0.15, 0.3)
    geom = Geometry([surf, bot, ell], np.array([np.pi - 0.5j]), np.array([0.5]), 1.0)
    phi, pw, U, ck = manufactured_inputs(geom, CASE_FLOW, [0.37])
    if with_psi_wall:
        geom.psi_wall = pw
    return geom, phi, U, ck


def flat_strip(M0, M1, h, V1=0.0):
    surf = fourier_surface(M0, 0.0, [])
    bot = graph_bottom(M1, -h)
    return Geometry([surf, bot], np.zeros(0, complex), np.zeros(0), V1)
