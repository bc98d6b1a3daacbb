"""Plain FP64 CPU oracle of the velocity-potential and vortex-sheet solves.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path must
never import this module.

Every function restates one passage of Ambrose, Camassa, Marzuola,
McLaughlin, Robinson and Wilkening, "Numerical algorithms for water waves
with background flow over obstacles and topography" (arXiv 2108.01786):

* kernels K_kj and G_kj with their diagonal limits ........ Sec. 3.2, Table 1
* block operator, rank-(N-1) correction, right-hand side ... Sec. 3.2 (B, A, Aw=b)
* collocation / trapezoid discretization ................... Sec. 3.3
* multi-valued potential Phi_mv and its derivative ......... Sec. 3, 3.1
* normal velocity U (velocity-potential method) ............ Sec. 3.4
* tangential velocity on every boundary .................... Sec. 5.1
* vortex-sheet wall system and U from gamma ................ Sec. 4.1
* energy E ................................................. Sec. 5.2
* gamma_t system (time derivative of the sheet strengths) .. Sec. 4.2
* one Runge-Kutta stage: graph and HLS surfaces, V, filter . Sec. 2, 3.5, 5
* velocity and pressure inside the fluid (Helsing-Ojala) .... Sec. 5.1, appendix
* spectral derivative and Hilbert transform (FFT symbols) .. Sec. 3.4
* restarted GMRES on the stored matrix ...................... Sec. 7.4 (solver)
* dense LU with one extended-precision refinement step ...... Sec. 7.4 (tolerance)
* tangent-linear model of J = sum w U^2 ..................... Sec. 3.2-3.4 differentiated
  (along surface displacements, or along the surface's node data)

Conventions the paper leaves open and that are fixed here: the Nyquist
coefficient of D, H and |d| is set to zero; the point z_j inside obstacle j
is supplied with the geometry; the stream-function constant on the bottom is
zero.  Matrix blocks are written with targets alpha_km along rows and
sources alpha_jl along columns; the diagonal of a same-boundary block is the
analytic limit, never the (singular) kernel value.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

F64 = torch.float64
C128 = torch.complex128


class OGeom:
    """Per-boundary complex samples z = zeta, d = zeta', e = zeta'' (FP64)."""

    def __init__(self, z: List[torch.Tensor], d: List[torch.Tensor], e: List[torch.Tensor],
                 zc: torch.Tensor, a: torch.Tensor, V1: float,
                 psi_wall: Optional[List[torch.Tensor]] = None):
        self.z, self.d, self.e = z, d, e
        self.M = [int(t.shape[0]) for t in z]
        self.nb = len(z)
        self.alpha = [2.0 * math.pi * torch.arange(m, dtype=F64) / m for m in self.M]
        self.zc = zc.to(C128)
        self.a = a.to(F64)
        self.V1 = float(V1)
        self.psi_wall = psi_wall

    @classmethod
    def from_synth(cls, geom) -> "OGeom":
        t = lambda v: torch.as_tensor(v, dtype=C128)
        z = [t(c.z) for c in geom.curves]
        d = [t(c.d) for c in geom.curves]
        e = [t(c.e) for c in geom.curves]
        pw = None
        if geom.psi_wall is not None:
            pw, off = [], 0
            for m in geom.M[1:]:
                pw.append(torch.as_tensor(geom.psi_wall[off:off + m], dtype=F64))
                off += m
        return cls(z, d, e, torch.as_tensor(geom.zc), torch.as_tensor(geom.a), geom.V1, pw)

    def with_surface(self, z0, d0, e0) -> "OGeom":
        """Same walls, new free surface (used for the gradient of J)."""
        return OGeom([z0] + self.z[1:], [d0] + self.d[1:], [e0] + self.e[1:],
                     self.zc, self.a, self.V1, self.psi_wall)


# ---------------------------------------------------------------------------
# kernels (Sec. 3.2, Table 1)
# ---------------------------------------------------------------------------

def half_cot(w: torch.Tensor) -> torch.Tensor:
    """(1/2) cot(w/2): the periodized Cauchy kernel (Mittag-Leffler sum, Sec. 3)."""
    return 0.5 / torch.tan(0.5 * w)


def _source_pairs(g: OGeom, k: int, j: int, rows: Optional[torch.Tensor]):
    """zeta_j'(b)/2 cot((zeta_j(b) - zeta_k(a))/2) for a = alpha_km (m in rows), b = alpha_jl.

    Returns (S, regulariser, diag) where for k == j the regulariser is
    (1/2)cot((b - a)/2) and diag marks the pairs m == l.  On diag the
    arguments are replaced by a harmless value; callers overwrite those
    entries with the analytic limit.
    """
    if rows is None:
        rows = torch.arange(g.M[k])
    zt = g.z[k][rows]
    at = g.alpha[k][rows]
    diff = g.z[j][None, :] - zt[:, None]
    reg, diag = None, None
    if k == j:
        diag = rows[:, None] == torch.arange(g.M[j])[None, :]
        diff = torch.where(diag, torch.ones_like(diff), diff)
        da = g.alpha[j][None, :] - at[:, None]
        reg = half_cot(torch.where(diag, torch.ones_like(da), da))
    S = g.d[j][None, :] * half_cot(diff)
    return S, reg, diag, rows


def self_limit(g: OGeom, k: int) -> torch.Tensor:
    """zeta''/(2 zeta'): the limit of the regularised self kernel (Sec. 3.2)."""
    return g.e[k] / (2.0 * g.d[k])


def K_block(g: OGeom, k: int, j: int, rows=None) -> torch.Tensor:
    """K_kj(alpha_km, alpha_jl) = Im{zeta_j'(b)/2 cot((zeta_j(b) - zeta_k(a))/2)}."""
    S, _, diag, rows = _source_pairs(g, k, j, rows)
    K = S.imag
    if diag is not None:
        lim = self_limit(g, k).imag[rows]
        K = torch.where(diag, lim[:, None].expand_as(K), K)
    return K


def G_block(g: OGeom, k: int, j: int, rows=None) -> torch.Tensor:
    """G_kj(alpha_km, alpha_jl) = Re{zeta_j'/2 cot(...) - delta_kj (1/2)cot((b - a)/2)}."""
    S, reg, diag, rows = _source_pairs(g, k, j, rows)
    G = S.real
    if diag is not None:
        G = G - reg
        lim = self_limit(g, k).real[rows]
        G = torch.where(diag, lim[:, None].expand_as(G), G)
    return G


# ---------------------------------------------------------------------------
# the linear system (Sec. 3.2 and 3.3)
# ---------------------------------------------------------------------------

def A_block(g: OGeom, k: int, j: int, rows=None) -> torch.Tensor:
    """Block (k, j) of the collocated, rank-corrected operator A.

    Row blocks: k = 0 gives phi~ on the surface, k >= 1 gives psi~ on wall k.
    (0,0): -I/2 + K_00/M_0;  (0,j): G_0j/M_j;  (k,0): -G_k0/M_0;
    (k,j): delta_kj I/2 + K_kj/M_j - delta_kj [k >= 2] E_k, E_k = e e^T / M_k.
    """
    if rows is None:
        rows = torch.arange(g.M[k])
    Mj = g.M[j]
    eye = (rows[:, None] == torch.arange(Mj)[None, :]).to(F64) if k == j else None
    if k == 0 and j == 0:
        return K_block(g, 0, 0, rows) / Mj - 0.5 * eye
    if k == 0:
        return G_block(g, 0, j, rows) / Mj
    if j == 0:
        return -G_block(g, k, 0, rows) / Mj
    B = K_block(g, k, j, rows) / Mj
    if k == j:
        B = B + 0.5 * eye
        if k >= 2:
            B = B - torch.full_like(B, 1.0 / Mj)
    return B


def _local_rows(g: OGeom, rows: torch.Tensor):
    off = [0]
    for m in g.M:
        off.append(off[-1] + m)
    out = []
    for k in range(g.nb):
        sel = (rows >= off[k]) & (rows < off[k + 1])
        if bool(sel.any()):
            out.append((k, torch.nonzero(sel).flatten(), rows[sel] - off[k]))
    return out


def A_rows(g: OGeom, rows: Sequence[int]) -> torch.Tensor:
    """Selected rows (global node indices) of A, e.g. for sampled checks at large M."""
    rows = torch.as_tensor(rows, dtype=torch.long)
    out = torch.zeros(rows.shape[0], sum(g.M), dtype=F64)
    for k, pos, loc in _local_rows(g, rows):
        out[pos] = torch.cat([A_block(g, k, j, loc) for j in range(g.nb)], dim=1)
    return out


def assemble_A(g: OGeom) -> torch.Tensor:
    """The whole M x M matrix of the collocated system (Sec. 3.3)."""
    return torch.cat([torch.cat([A_block(g, k, j) for j in range(g.nb)], dim=1)
                      for k in range(g.nb)], dim=0)


# ---------------------------------------------------------------------------
# multi-valued part of the potential (Sec. 3 and 3.1)
# ---------------------------------------------------------------------------

def dPhi_mv(g: OGeom, z: torch.Tensor) -> torch.Tensor:
    """Phi_mv'(z) = V1 + sum_j a_j (1/2 - (i/2) cot((z - z_j)/2))."""
    out = torch.full_like(z, g.V1)
    for aj, zj in zip(g.a, g.zc):
        out = out + aj * (0.5 - 1j * half_cot(z - zj))
    return out


def psi_mv(g: OGeom, z: torch.Tensor) -> torch.Tensor:
    """Im Phi_mv(z) = V1 Im z - sum_j a_j ln|1 - e^{i(z - z_j)}|."""
    out = g.V1 * z.imag
    for aj, zj in zip(g.a, g.zc):
        out = out - aj * torch.log(torch.abs(1.0 - torch.exp(1j * (z - zj))))
    return out


def u_mv(g: OGeom, z: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """s_alpha dphi_mv/dn = Re{Phi_mv'(zeta) i zeta'}  (Sec. 3.4, first line)."""
    return (dPhi_mv(g, z) * 1j * d).real


def rhs(g: OGeom, phi: torch.Tensor) -> torch.Tensor:
    """b_0 = phi~; b_k = psi_wall_k - psi_mv(zeta_k) for k >= 1 (psi_wall = 0 by default)."""
    parts = [phi.to(F64)]
    for k in range(1, g.nb):
        bk = -psi_mv(g, g.z[k])
        if g.psi_wall is not None:
            bk = bk + g.psi_wall[k - 1]
        parts.append(bk)
    return torch.cat(parts)


# ---------------------------------------------------------------------------
# spectral operators (Sec. 3.4)
# ---------------------------------------------------------------------------

def spectral(f: torch.Tensor, op: str) -> torch.Tensor:
    """FFT-symbol operators on a uniform periodic grid: D (ik), D2 (-k^2),
    H (-i sgn k), ABSD (|k|), INT (1/(ik), the zero-mean antiderivative) and
    FILTER (the 36th-order filter).  The Nyquist coefficient is zeroed."""
    M = f.shape[-1]
    k = torch.fft.fftfreq(M, d=1.0 / M).to(F64)
    nyq = (k == -M / 2)
    if op == "D":
        sym = 1j * k
    elif op == "D2":
        sym = -(k * k) + 0j
    elif op == "H":
        sym = -1j * torch.sign(k)
    elif op == "ABSD":
        sym = torch.abs(k) + 0j
    elif op == "INT":
        # zero-mean periodic antiderivative: 1/(ik) for k != 0, 0 at k = 0
        sym = torch.where(k == 0, torch.zeros_like(k), 1.0 / torch.where(k == 0, torch.ones_like(k), k)) / 1j
    elif op == "FILTER":
        # the 36th-order filter of Sec. 5: exp(-36 (|k| / kmax)^36), kmax = M/2
        sym = torch.exp(-36.0 * (torch.abs(k) / (M / 2)) ** 36) + 0j
    else:
        raise ValueError(op)
    sym = torch.where(nyq, torch.zeros_like(sym), sym)
    return torch.fft.ifft(sym * torch.fft.fft(f.to(C128))).real


def split(g: OGeom, v: torch.Tensor) -> List[torch.Tensor]:
    return list(torch.split(v, g.M))


def spectral_tail(f: torch.Tensor) -> float:
    """Resolution measure of one periodic sample vector (the Fourier-tail test
    the paper applies before refining its grids, Sec. 7.1: the mode amplitudes
    must decay before k reaches M/2): the square root of the fraction of the
    spectral energy held by the modes |k| >= 3M/8, from the full FFT."""
    M = f.shape[-1]
    c = torch.fft.fft(f.to(C128))
    k = torch.fft.fftfreq(M, d=1.0 / M).abs()
    e = c.abs() ** 2
    tail = e[k >= -(-3 * M // 8)].sum()
    return float(torch.sqrt(tail / e.sum())) if float(e.sum()) > 0 else 0.0


# ---------------------------------------------------------------------------
# velocity-potential method (Sec. 3.2 - 3.4)
# ---------------------------------------------------------------------------

def dphi_dn_from_omega(g: OGeom, omega: List[torch.Tensor]) -> torch.Tensor:
    """U on the free surface from the densities (Sec. 3.4):

    s U = Re{Phi_mv' i zeta'} - H(omega_0')/2 - (1/M_0) sum_l G_00(b_l, a) omega_0'(b_l)
          + sum_{j>=1} (1/M_j) sum_l K_j0(b_l, a) omega_j'(b_l).
    The integration variable sits in the first slot of G_00 and K_j0, so
    these are the transposes of the blocks G_00 and K_j0.
    """
    dw = [spectral(w, "D") for w in omega]
    s0 = torch.abs(g.d[0])
    acc = u_mv(g, g.z[0], g.d[0])
    acc = acc - 0.5 * spectral(dw[0], "H")
    acc = acc - (G_block(g, 0, 0).T @ dw[0]) / g.M[0]
    for j in range(1, g.nb):
        acc = acc + (K_block(g, j, 0).T @ dw[j]) / g.M[j]
    return acc / s0


def dphi_ds_from_omega(g: OGeom, omega: List[torch.Tensor]) -> List[torch.Tensor]:
    """Tangential derivative dphi/ds on every boundary (Sec. 5.1, the formulas
    for s dphi/ds_k that accompany the normal ones of Sec. 4.1), with
    gamma_0 = -omega_0' and gamma_j = omega_j':

    s dphi/ds_k = Re{Phi_mv'(zeta_k) zeta_k'} + [k = 0] gamma_0 / 2
                  + (1/M_0) sum_l K_0k(b_l, a) gamma_0(b_l)
                  + sum_{j>=1} ( -[k = j] H(gamma_j)/2 - (1/M_j) sum_l G_jk(b_l, a) gamma_j(b_l) ).
    The free surface is taken on its fluid (lower) side, where the jump term
    of gamma_0 enters with a plus sign.  The integration variable sits in
    the first slot of K_0k and G_jk, so the blocks enter transposed.
    """
    gam = [-spectral(omega[0], "D")] + [spectral(w, "D") for w in omega[1:]]
    out = []
    for k in range(g.nb):
        acc = (dPhi_mv(g, g.z[k]) * g.d[k]).real
        if k == 0:
            acc = acc + 0.5 * gam[0]
        acc = acc + (K_block(g, 0, k).T @ gam[0]) / g.M[0]
        for j in range(1, g.nb):
            if j == k:
                acc = acc - 0.5 * spectral(gam[j], "H")
            acc = acc - (G_block(g, j, k).T @ gam[j]) / g.M[j]
        out.append(acc / torch.abs(g.d[k]))
    return out


def residual_ext(A: torch.Tensor, b: torch.Tensor, x: torch.Tensor, chunk: int = 1024):
    """b - A x formed in extended precision (numpy longdouble: a 64-bit
    significand on x86) and rounded once to FP64, a chunk of rows at a time."""
    xl = x.numpy().astype(np.longdouble)
    r = np.empty(tuple(b.shape), dtype=np.float64)
    for r0 in range(0, A.shape[0], chunk):
        Al = A[r0:r0 + chunk].numpy().astype(np.longdouble)
        r[r0:r0 + chunk] = (b[r0:r0 + chunk].numpy().astype(np.longdouble) - Al @ xl)
    return torch.as_tensor(r)


def dense_solve(A: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """A x = b by dense LU followed by one step of iterative refinement whose
    residual is formed in extended precision (residual_ext).

    The paper runs its solver to a relative residual of 1e-15 (Sec. 7.4).  An
    FP64 LU alone stops near 1e-13 on these systems, with a forward error of
    about that size that depends on how the LAPACK in use orders its sums:
    harmless for omega itself, but two spectral derivatives (the gamma_t
    system, Sec. 4.2) amplify it by up to (M_0/2)^2.  One refinement step takes
    x to the exact solution of the FP64 system up to its last bits (the LU
    factors contract the error by their own backward error, about 1e-14 here),
    independently of the LAPACK.  Autograd differentiates the LU solve; the
    correction is a constant for it (the derivative of the solution map is the
    same in exact arithmetic)."""
    Ad = A.detach()
    vec = b.dim() == 1
    if A.requires_grad or b.requires_grad:
        x = torch.linalg.solve(A, b)
        LU, piv = torch.linalg.lu_factor(Ad)
    else:
        LU, piv = torch.linalg.lu_factor(Ad)
        x = torch.linalg.lu_solve(LU, piv, b[:, None] if vec else b)
        x = x[:, 0] if vec else x
    r = residual_ext(Ad, b.detach(), x.detach())
    d = torch.linalg.lu_solve(LU, piv, r[:, None] if vec else r)
    return x + (d[:, 0] if vec else d)


def solve_phi(g: OGeom, phi: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Solve A omega = b (dense_solve); return omega, psi|_k (k >= 2) and U."""
    A = assemble_A(g)
    b = rhs(g, phi)
    omega = dense_solve(A, b)
    parts = split(g, omega)
    psi_k = torch.stack([p.mean() for p in parts[2:]]) if g.nb > 2 else torch.zeros(0, dtype=F64)
    U = dphi_dn_from_omega(g, parts)
    return {"omega": omega, "psi_k": psi_k, "U": U, "A": A, "b": b}


# ---------------------------------------------------------------------------
# vortex-sheet method (Sec. 4.1)
# ---------------------------------------------------------------------------

def wall_matrix(g: OGeom) -> torch.Tensor:
    """Row block k, column block j (k, j >= 1): -delta_kj I/2 + K_jk^dagger,
    (K_jk^dagger)_{ml} = K_jk(alpha_jl, alpha_km)/M_j."""
    rows = []
    for k in range(1, g.nb):
        blocks = []
        for j in range(1, g.nb):
            B = K_block(g, j, k).T / g.M[j]
            if j == k:
                B = B - 0.5 * torch.eye(g.M[k], dtype=F64)
            blocks.append(B)
        rows.append(torch.cat(blocks, dim=1))
    return torch.cat(rows, dim=0)


def solve_gamma(g: OGeom, gamma0: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Given gamma_0 on the surface, solve the wall system for gamma_1..gamma_N
    (zero normal velocity on every wall) and return U (Sec. 4.1)."""
    gamma0 = gamma0.to(F64)
    rhs_w = []
    for k in range(1, g.nb):
        rk = -(G_block(g, 0, k).T @ gamma0) / g.M[0] - u_mv(g, g.z[k], g.d[k])
        rhs_w.append(rk)
    W = wall_matrix(g)
    gw = dense_solve(W, torch.cat(rhs_w))
    gparts = split(OGeom(g.z[1:], g.d[1:], g.e[1:], g.zc, g.a, g.V1), gw)
    s0 = torch.abs(g.d[0])
    acc = 0.5 * spectral(gamma0, "H") + (G_block(g, 0, 0).T @ gamma0) / g.M[0]
    for j in range(1, g.nb):
        acc = acc + (K_block(g, j, 0).T @ gparts[j - 1]) / g.M[j]
    acc = acc + u_mv(g, g.z[0], g.d[0])
    return {"U": acc / s0, "gamma_wall": gw, "W": W}


# ---------------------------------------------------------------------------
# time derivative of the vortex sheet strengths (Sec. 4.2)
# ---------------------------------------------------------------------------

def gamma_t_matrix(g: OGeom) -> torch.Tensor:
    """The collocated operator of the gamma_t system (Sec. 4.2, the gamma_0,t
    equation stacked on the wall equations), all blocks in the dagger form
    of Sec. 4.1 (integration variable in the first kernel slot, weight 1/M_j):
      row 0:  (I/2 + K_00^dagger) gamma_0,t - sum_j G_j0^dagger gamma_j,t
      row k:  G_0k^dagger gamma_0,t + (-I/2 + K_kk^dagger) gamma_k,t
              + sum_{j != k} K_jk^dagger gamma_j,t           (k >= 1)."""
    rows = []
    for k in range(g.nb):
        blocks = []
        for j in range(g.nb):
            if k == 0 and j == 0:
                B = K_block(g, 0, 0).T / g.M[0] + 0.5 * torch.eye(g.M[0], dtype=F64)
            elif k == 0:
                B = -G_block(g, j, 0).T / g.M[j]
            elif j == 0:
                B = G_block(g, 0, k).T / g.M[0]
            else:
                B = K_block(g, j, k).T / g.M[j]
                if j == k:
                    B = B - 0.5 * torch.eye(g.M[k], dtype=F64)
            blocks.append(B)
        rows.append(torch.cat(blocks, dim=1))
    return torch.cat(rows, dim=0)


def F_operators(g: OGeom, gamma0: torch.Tensor, U: torch.Tensor, V: torch.Tensor):
    """F_00 gamma_0 and F_k0 gamma_0 (k >= 1) in the regularised form that
    writes zeta_t = (V + i U) zeta' / s (Sec. 4.2):
      F_00 = -H(U gamma_0 / s)/2 + K_00(V gamma_0 / s) + G_00(U gamma_0 / s),
      F_k0 = G_k0(V gamma_0 / s) - K_k0(U gamma_0 / s),
    with K_kj f = (1/M_j) sum_l K_kj(a, b_l) f(b_l) (target in the first slot)."""
    s0 = torch.abs(g.d[0])
    fV = V * gamma0 / s0
    fU = U * gamma0 / s0
    out = [-0.5 * spectral(fU, "H") + (K_block(g, 0, 0) @ fV + G_block(g, 0, 0) @ fU) / g.M[0]]
    for k in range(1, g.nb):
        out.append((G_block(g, k, 0) @ fV - K_block(g, k, 0) @ fU) / g.M[0])
    return out


def gamma_t_rhs(g: OGeom, phi: torch.Tensor, V: torch.Tensor, tau: float,
                grav: float = 1.0) -> Dict[str, torch.Tensor]:
    """Right-hand side of the gamma_t system (Sec. 4.2) at the state (zeta, phi~).

    The velocity-potential solve gives omega, U and gamma = (-D omega_0,
    D omega_j); W is the Birkhoff-Rott velocity plus grad phi_mv on the
    surface, so that grad phi = W + gamma_0 t / (2 s) on the fluid side:
    W.t = dphi/ds - gamma_0 / (2 s), W.n = U.
      surface: d/dalpha( -W.W/2 + (V - W.t) gamma_0 / (2 s) - gamma_0^2 / (8 s^2)
                         + tau theta_alpha / s - g eta - F_00 gamma_0 ),
      wall k:  -d/dalpha( F_k0 gamma_0 )."""
    r = solve_phi(g, phi)
    parts = split(g, r["omega"])
    U = r["U"]
    gamma0 = -spectral(parts[0], "D")
    s0 = torch.abs(g.d[0])
    ds = dphi_ds_from_omega(g, parts)[0]
    Wt = ds - gamma0 / (2.0 * s0)
    WW = Wt * Wt + U * U
    theta_a = (g.e[0] / g.d[0]).imag
    F = F_operators(g, gamma0, U, V.to(F64))
    surf = (-0.5 * WW + (V - Wt) * gamma0 / (2.0 * s0) - gamma0 ** 2 / (8.0 * s0 ** 2)
            + tau * theta_a / s0 - grav * g.z[0].imag - F[0])
    b = [spectral(surf, "D")] + [-spectral(F[k], "D") for k in range(1, g.nb)]
    return {"b": torch.cat(b), "omega": r["omega"], "U": U, "gamma0": gamma0}


def solve_gamma_t(g: OGeom, phi: torch.Tensor, V: torch.Tensor, tau: float,
                  grav: float = 1.0) -> Dict[str, torch.Tensor]:
    """gamma_t = (gamma_0,t, gamma_1,t, ...) from the Sec. 4.2 system (dense_solve)."""
    r = gamma_t_rhs(g, phi, V, tau, grav)
    B = gamma_t_matrix(g)
    r["gamma_t"] = dense_solve(B, r["b"])
    r["B"] = B
    return r


def surface_velocity_state(g: OGeom, phi: torch.Tensor, V: torch.Tensor, tau: float,
                           grav: float = 1.0):
    """zeta_t = (V + i U) zeta'/s and the phi~ equation of Sec. 3.5 (C = 0):
    phi~_t = (phi~_alpha / s) V + (U - u_mv / s) U - |grad phi|^2 / 2 - g eta
             + tau theta_alpha / s, |grad phi|^2 = (phi_alpha / s)^2 + U^2."""
    r = solve_phi(g, phi)
    U = r["U"]
    z, d, e = g.z[0], g.d[0], g.e[0]
    s0 = torch.abs(d)
    zt = (V + 1j * U) * d / s0
    pa_t = spectral(phi.to(F64), "D")
    pa = pa_t + (dPhi_mv(g, z) * d).real
    dn_t = U - u_mv(g, z, d) / s0
    grad2 = (pa / s0) ** 2 + U ** 2
    phit = pa_t / s0 * V + dn_t * U - 0.5 * grad2 - grav * z.imag + tau * (e / d).imag / s0
    return zt, phit


# ---------------------------------------------------------------------------
# evolution of the free surface: one Runge-Kutta stage (Sec. 2, 3.5, 5)
# ---------------------------------------------------------------------------

def graph_surface(eta: torch.Tensor):
    """zeta = alpha + i eta with spectral zeta', zeta'' (Sec. 2.1, xi = alpha)."""
    M = eta.shape[0]
    al = 2.0 * math.pi * torch.arange(M, dtype=F64) / M
    z = al + 1j * eta
    d = 1.0 + 1j * spectral(eta, "D")
    e = 1j * spectral(eta, "D2")
    return z, d, e


def hls_reconstruct(Ptheta: torch.Tensor):
    """The curve from P theta (Sec. 2.2): C, S are the means of cos and sin of
    P theta, P_0 theta = arg(C - iS), s_alpha = (C^2 + S^2)^(-1/2),
    zeta' = s_alpha e^{i theta}; xi, eta are zero-mean antiderivatives shifted
    so that xi(0) = 0 and the mean height <eta> = P_0[eta xi'] = 0."""
    M = Ptheta.shape[0]
    al = 2.0 * math.pi * torch.arange(M, dtype=F64) / M
    C = torch.cos(Ptheta).mean()
    S = torch.sin(Ptheta).mean()
    theta = Ptheta + torch.atan2(-S, C)
    sa = 1.0 / torch.sqrt(C * C + S * S)
    d = sa * torch.exp(1j * theta)
    xa = spectral(d.real - 1.0, "INT")
    ya = spectral(d.imag, "INT")
    xi = al + xa - xa[0]
    eta = ya - (ya * d.real).mean()
    theta_a = spectral(Ptheta, "D")
    e = 1j * theta_a * d
    return xi + 1j * eta, d, e, theta, sa


def hls_V(theta_a: torch.Tensor, U: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """V = antiderivative of (theta_a U - mean), with V(0) = U(0) eta'(0)/xi'(0)
    so that xi(0) stays 0 (Sec. 5, the equation for V)."""
    f = theta_a * U
    V = spectral(f - f.mean(), "INT")
    return V - V[0] + U[0] * d[0].imag / d[0].real


def stage_rhs(g_walls: OGeom, mode: str, q: torch.Tensor, phi: torch.Tensor, tau: float,
              grav: float = 1.0):
    """Time derivatives of the surface variable q and of phi~ at one stage.

    mode "graph": q = eta with xi = alpha; V = eta_alpha U and
      eta_t = sqrt(1 + eta_alpha^2) U (Sec. 2.1).
    mode "hls": q = P theta; the curve is reconstructed (Sec. 2.2), V from its
      equation in Sec. 5 and (P theta)_t = P[(U_alpha + V theta_alpha) / s_alpha].
    phi~_t follows Sec. 3.5 with C(t) = 0 in both modes."""
    q = q.to(F64)
    if mode == "graph":
        z, d, e = graph_surface(q)
    else:
        z, d, e, theta, sa = hls_reconstruct(q)
    g = g_walls.with_surface(z, d, e)
    U = solve_phi(g, phi)["U"]
    if mode == "graph":
        ea = d.imag
        V = ea * U
        qt = torch.sqrt(1.0 + ea * ea) * U
    else:
        theta_a = spectral(q, "D")
        V = hls_V(theta_a, U, d)
        f = (spectral(U, "D") + V * theta_a) / sa
        qt = f - f.mean()
    _, phit = surface_velocity_state(g, phi, V, tau, grav)
    return qt, phit, {"z": z, "d": d, "e": e, "U": U, "V": V}


def rk_step(g_walls: OGeom, mode: str, A, b, h: float, q: torch.Tensor, phi: torch.Tensor,
            tau: float, grav: float = 1.0, filt: bool = True):
    """One explicit Runge-Kutta step with tableau (A, b), every stage by
    stage_rhs; the 36th-order filter (Sec. 5) is applied to q and phi~ at the
    end of the step when filt is set."""
    s = len(b)
    kq, kp = [], []
    for i in range(s):
        qi, pi = q.clone(), phi.clone()
        for j in range(i):
            if A[i][j] != 0.0:
                qi = qi + h * A[i][j] * kq[j]
                pi = pi + h * A[i][j] * kp[j]
        a1, a2, _ = stage_rhs(g_walls, mode, qi, pi, tau, grav)
        kq.append(a1)
        kp.append(a2)
    qn, pn = q.clone(), phi.clone()
    for i in range(s):
        if b[i] != 0.0:
            qn = qn + h * b[i] * kq[i]
            pn = pn + h * b[i] * kp[i]
    if filt:
        qn, pn = spectral(qn, "FILTER"), spectral(pn, "FILTER")
    return qn, pn


# ---------------------------------------------------------------------------
# values inside the fluid (Sec. 5.1 and the Helsing-Ojala appendix)
# ---------------------------------------------------------------------------

def dphi_dn_all(g: OGeom, omega: List[torch.Tensor]) -> List[torch.Tensor]:
    """Normal derivative dphi/dn on every boundary (Sec. 4.1, the formulas for
    s dphi/dn_k), gamma_0 = -omega_0', gamma_j = omega_j':
      s dphi/dn_k = Re{Phi_mv'(zeta_k) i zeta_k'} + [k = 0] H(gamma_0)/2
                    + (1/M_0) sum_l G_0k(b_l, a) gamma_0(b_l)
                    + sum_{j>=1} ( -[k = j] gamma_j/2 + (1/M_j) sum_l K_jk(b_l, a) gamma_j(b_l) ).
    On the surface this is U; on the walls it vanishes for the physical
    problem (psi constant there) up to the discretization error."""
    gam = [-spectral(omega[0], "D")] + [spectral(w, "D") for w in omega[1:]]
    out = []
    for k in range(g.nb):
        acc = u_mv(g, g.z[k], g.d[k])
        if k == 0:
            acc = acc + 0.5 * spectral(gam[0], "H")
        acc = acc + (G_block(g, 0, k).T @ gam[0]) / g.M[0]
        for j in range(1, g.nb):
            if j == k:
                acc = acc - 0.5 * gam[j]
            acc = acc + (K_block(g, j, k).T @ gam[j]) / g.M[j]
        out.append(acc / torch.abs(g.d[k]))
    return out


def boundary_dPhi(g: OGeom, omega: List[torch.Tensor]) -> List[torch.Tensor]:
    """Phi'(zeta) = u - i v = (dphi/ds - i dphi/dn) |zeta'| / zeta' on every
    boundary (Sec. 5.1)."""
    ds = dphi_ds_from_omega(g, omega)
    dn = dphi_dn_all(g, omega)
    return [(ds[k] - 1j * dn[k]) * torch.abs(g.d[k]) / g.d[k] for k in range(g.nb)]


def helsing_ojala(g: OGeom, fvals: List[torch.Tensor], z: torch.Tensor) -> torch.Tensor:
    """f(z) for z in the fluid from the boundary values of a periodic function
    analytic there (the Helsing-Ojala rule):
      f(z) = sum lam_km f_km / sum lam_km,
      lam_km = sigma_k / M_k * (1/2) cot((zeta_km - z)/2) zeta'_km.
    The trapezoid sums approximate contour integrals over the positively
    oriented boundary of the fluid, which runs along the free surface against
    its parameter (sigma_0 = -1) and along the bottom and the clockwise
    obstacles with it (sigma_k = +1).  A point on a node takes that node's value."""
    z = z.to(C128)
    num = torch.zeros_like(z)
    den = torch.zeros_like(z)
    hit = torch.full(z.shape, -1, dtype=torch.long)
    hitv = torch.zeros_like(z)
    for k in range(g.nb):
        sig = -1.0 if k == 0 else 1.0
        diff = g.z[k][None, :] - z[:, None]
        on = diff == 0
        lam = sig / g.M[k] * half_cot(torch.where(on, torch.ones_like(diff), diff)) * g.d[k][None, :]
        lam = torch.where(on, torch.zeros_like(lam), lam)
        num = num + (lam * fvals[k].to(C128)[None, :]).sum(1)
        den = den + lam.sum(1)
        rows = on.any(1)
        if bool(rows.any()):
            idx = on.float().argmax(1)
            hitv = torch.where(rows, fvals[k].to(C128)[idx], hitv)
            hit = torch.where(rows, torch.full_like(hit, k), hit)
    return torch.where(hit >= 0, hitv, num / den)


def layer_potential_direct(g: OGeom, omega: List[torch.Tensor], z: torch.Tensor) -> torch.Tensor:
    """The Cauchy integrals of Sec. 3 summed by the trapezoid rule at points z
    away from the boundaries: Phi_0 carries 1/(2 pi i), Phi_j (walls) 1/(2 pi)."""
    z = z.to(C128)
    out = torch.zeros_like(z)
    for k in range(g.nb):
        c = -1j if k == 0 else 1.0
        ker = half_cot(g.z[k][None, :] - z[:, None]) * g.d[k][None, :]
        out = out + c * (ker * omega[k].to(C128)[None, :]).sum(1) / g.M[k]
    return out


def boundary_Phi(g: OGeom, omega: List[torch.Tensor]) -> List[torch.Tensor]:
    """Fluid-side boundary values of the Cauchy integrals sum_k Phi_k (no
    multi-valued part), from the Plemelj formulas with the Table 1 kernels:
      surface: Re = -omega_0/2 + K_00 omega_0 + sum_j G_0j omega_j,
               Im = H(omega_0)/2 - G_00 omega_0 + sum_j K_0j omega_j;
      wall k:  Re = K_k0 omega_0 + sum_j G_kj omega_j - H(omega_k)/2,
               Im = -G_k0 omega_0 + omega_k/2 + sum_j K_kj omega_j,
    every block divided by its source count (the trapezoid weights)."""
    out = []
    for k in range(g.nb):
        if k == 0:
            re = -0.5 * omega[0] + (K_block(g, 0, 0) @ omega[0]) / g.M[0]
            im = 0.5 * spectral(omega[0], "H") - (G_block(g, 0, 0) @ omega[0]) / g.M[0]
            for j in range(1, g.nb):
                re = re + (G_block(g, 0, j) @ omega[j]) / g.M[j]
                im = im + (K_block(g, 0, j) @ omega[j]) / g.M[j]
        else:
            re = (K_block(g, k, 0) @ omega[0]) / g.M[0] - 0.5 * spectral(omega[k], "H")
            im = -(G_block(g, k, 0) @ omega[0]) / g.M[0] + 0.5 * omega[k]
            for j in range(1, g.nb):
                re = re + (G_block(g, k, j) @ omega[j]) / g.M[j]
                im = im + (K_block(g, k, j) @ omega[j]) / g.M[j]
        out.append(re + 1j * im)
    return out


def pressure(g: OGeom, phi: torch.Tensor, tau: float, grav: float, z: torch.Tensor):
    """p / rho = C - phi_t - |grad phi|^2 / 2 - g y inside the fluid (Sec. 5.1).
    phi_t - C is the harmonic function with the Dirichlet data
    tau kappa - |grad phi|^2 / 2 - g eta on the surface (Laplace-Young,
    p = -tau kappa there) and zero normal derivative on the walls: the same
    matrix A with b_0 = that data and b_k = 0, its Cauchy integrals carried
    inside by the Helsing-Ojala rule, as is u - i v."""
    r = solve_phi(g, phi)
    om = split(g, r["omega"])
    U = r["U"]
    ds = dphi_ds_from_omega(g, om)[0]
    s0 = torch.abs(g.d[0])
    kappa = (g.e[0] / g.d[0]).imag / s0
    data = tau * kappa - 0.5 * (ds * ds + U * U) - grav * g.z[0].imag
    b = torch.cat([data] + [torch.zeros(m, dtype=F64) for m in g.M[1:]])
    om_aux = split(g, dense_solve(r["A"], b))
    phit = helsing_ojala(g, boundary_Phi(g, om_aux), z).real
    w = helsing_ojala(g, boundary_dPhi(g, om), z)
    return -phit - 0.5 * (w.abs() ** 2) - grav * z.imag


# ---------------------------------------------------------------------------
# energy (Sec. 5.2)
# ---------------------------------------------------------------------------

def psi_on_surface(g: OGeom, omega: List[torch.Tensor]) -> torch.Tensor:
    """psi on the fluid side of the surface: psi_mv + Im of the Cauchy integrals.

    By the Plemelj formula the surface's own integral contributes
    H(omega_0)/2 - (1/M_0) sum_l G_00(a, b_l) omega_0(b_l); each wall j adds
    (1/M_j) sum_l K_0j(a, b_l) omega_j(b_l).
    """
    out = psi_mv(g, g.z[0]) + 0.5 * spectral(omega[0], "H")
    out = out - (G_block(g, 0, 0) @ omega[0]) / g.M[0]
    for j in range(1, g.nb):
        out = out + (K_block(g, 0, j) @ omega[j]) / g.M[j]
    return out


def energy(g: OGeom, phi: torch.Tensor, omega: torch.Tensor, tau: float, grav: float = 1.0) -> float:
    """E = <tau s + g eta^2 xi_a / 2 + psi|Gamma0 phi_a / 2> + sum_j a_j psi|_j / 2 (rho = 1)."""
    parts = split(g, omega)
    z0, d0 = g.z[0], g.d[0]
    s = torch.abs(d0)
    phi_a = spectral(phi.to(F64), "D") + (dPhi_mv(g, z0) * d0).real
    psiG = psi_on_surface(g, parts)
    E = (tau * s + 0.5 * grav * z0.imag ** 2 * d0.real + 0.5 * psiG * phi_a).mean()
    for j in range(2, g.nb):
        E = E + 0.5 * g.a[j - 2] * parts[j].mean()
    return float(E)


# ---------------------------------------------------------------------------
# surface parameterised by periodic displacements, and the gradient of J
# ---------------------------------------------------------------------------

def surface_from_periodic(xt: torch.Tensor, yt: torch.Tensor):
    """zeta = alpha + xt + i yt with spectral zeta', zeta'' (x = alpha + periodic part)."""
    M = xt.shape[0]
    al = 2.0 * math.pi * torch.arange(M, dtype=F64) / M
    z = (al + xt) + 1j * yt
    d = (1.0 + spectral(xt, "D")) + 1j * spectral(yt, "D")
    e = spectral(xt, "D2") + 1j * spectral(yt, "D2")
    return z, d, e


def J_and_grad(g_walls: OGeom, xt, yt, phi, weights):
    """J = sum_m w_m U_m^2 and its gradient w.r.t. (xt, yt, phi) by autograd."""
    xt = torch.as_tensor(xt, dtype=F64).clone().requires_grad_(True)
    yt = torch.as_tensor(yt, dtype=F64).clone().requires_grad_(True)
    ph = torch.as_tensor(phi, dtype=F64).clone().requires_grad_(True)
    w = torch.as_tensor(weights, dtype=F64)
    z0, d0, e0 = surface_from_periodic(xt, yt)
    g = g_walls.with_surface(z0, d0, e0)
    U = solve_phi(g, ph)["U"]
    J = (w * U * U).sum()
    gx, gy, gp = torch.autograd.grad(J, (xt, yt, ph))
    return float(J.detach()), gx.detach(), gy.detach(), gp.detach(), U.detach()


# ---------------------------------------------------------------------------
# large systems: row-blocked assembly, restarted GMRES, the U map summed over
# source chunks, and the tangent-linear model of the solve
# ---------------------------------------------------------------------------

def assemble_A_blocked(g: OGeom, chunk: int = 1024) -> torch.Tensor:
    """The matrix of assemble_A built chunk by chunk of rows (A_rows): every
    entry is the same elementwise expression (equal to assemble_A's up to the
    last bit of the vectorised tan), and the peak memory of the intermediates
    is bounded by the chunk."""
    n = sum(g.M)
    A = torch.empty(n, n, dtype=F64)
    for r0 in range(0, n, chunk):
        A[r0:r0 + chunk] = A_rows(g, range(r0, min(n, r0 + chunk)))
    return A


def gmres(matvec, b: torch.Tensor, tol: float = 1e-13, restart: int = 100,
          max_iter: int = 2000, x0: Optional[torch.Tensor] = None):
    """Restarted GMRES for A x = b, unpreconditioned, in the Euclidean norm
    (the paper's solver for the collocated system, Sec. 7.4; its unstated
    details follow the readings: start from x0, zero by default; the Arnoldi
    vectors are orthogonalised by classical Gram-Schmidt applied twice; the
    small least-squares problem is reduced by Givens rotations).

    Convergence is declared only on the true residual ||b - A x||_2 <=
    tol ||b||_2, formed at the start of every cycle; inside a cycle the
    rotated right-hand side only decides when the cycle ends.  Returns
    (x, relative true residual at every cycle start, Arnoldi steps)."""
    b = b.to(F64)
    n = b.shape[0]
    x = torch.zeros_like(b) if x0 is None else x0.to(F64).clone()
    bn = float(torch.linalg.vector_norm(b))
    hist: List[float] = []
    steps = 0
    if bn == 0.0:
        return torch.zeros_like(b), [0.0], 0
    while True:
        r = b - matvec(x) if (x0 is not None or steps > 0) else b.clone()
        beta = float(torch.linalg.vector_norm(r))
        hist.append(beta / bn)
        if beta <= tol * bn or steps >= max_iter:
            break
        if len(hist) > 1 and beta > 0.99 * hist[-2] * bn:
            break                       # the last cycle made no progress
        V = torch.zeros(restart + 1, n, dtype=F64)
        H = torch.zeros(restart + 1, restart, dtype=F64)
        cs = torch.zeros(restart, dtype=F64)
        sn = torch.zeros(restart, dtype=F64)
        gr = torch.zeros(restart + 1, dtype=F64)
        V[0] = r / beta
        gr[0] = beta
        k = 0
        for j in range(restart):
            w = matvec(V[j])
            for _ in range(2):          # classical Gram-Schmidt, twice
                h = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h
                H[:j + 1, j] += h
            hn = float(torch.linalg.vector_norm(w))
            H[j + 1, j] = hn
            if hn > 0.0:
                V[j + 1] = w / hn
            for i in range(j):          # earlier rotations on the new column
                a_, b_ = float(H[i, j]), float(H[i + 1, j])
                H[i, j] = cs[i] * a_ + sn[i] * b_
                H[i + 1, j] = -sn[i] * a_ + cs[i] * b_
            a_, b_ = float(H[j, j]), float(H[j + 1, j])
            rho = math.hypot(a_, b_)
            cs[j], sn[j] = a_ / rho, b_ / rho
            H[j, j], H[j + 1, j] = rho, 0.0
            gr[j + 1] = -sn[j] * gr[j]
            gr[j] = cs[j] * gr[j]
            k = j + 1
            steps += 1
            if abs(float(gr[k])) <= tol * bn or hn == 0.0 or steps >= max_iter:
                break
        y = torch.linalg.solve_triangular(H[:k, :k], gr[:k, None], upper=True)[:, 0]
        x = x + V[:k].T @ y
    return x, hist, steps


def dphi_dn_from_omega_chunked(g: OGeom, omega: List[torch.Tensor],
                               chunk: int = 2048) -> torch.Tensor:
    """dphi_dn_from_omega with the transposed blocks G_00^T and K_j0^T applied
    chunk by chunk of their rows (the sources): the same sums, grouped, so that
    the M_0 x M map never has to be held at once."""
    dw = [spectral(w, "D") for w in omega]
    s0 = torch.abs(g.d[0])
    acc = u_mv(g, g.z[0], g.d[0]) - 0.5 * spectral(dw[0], "H")
    for j in range(g.nb):
        sign = -1.0 if j == 0 else 1.0
        blk = G_block if j == 0 else K_block
        for r0 in range(0, g.M[j], chunk):
            rows = torch.arange(r0, min(g.M[j], r0 + chunk))
            acc = acc + sign * (blk(g, j, 0, rows).T @ dw[j][rows]) / g.M[j]
    return acc / s0


def A_times_blocked(g: OGeom, x: torch.Tensor, chunk: int = 1024) -> torch.Tensor:
    """A x with the rows of A formed chunk by chunk and never stored."""
    n = sum(g.M)
    return torch.cat([A_rows(g, range(r0, min(n, r0 + chunk))) @ x for r0 in range(0, n, chunk)])


def tangent_J(g_walls: OGeom, xt, yt, phi, weights, dirs, solve, omega=None,
              chunk: int = 1024):
    """Directional derivatives of J = sum_m w_m U_m^2 along directions
    (dxt, dyt, dphi) of the surface displacements and the surface potential,
    walls fixed: the tangent-linear model of the velocity-potential solve
    (Sec. 3.2-3.4 differentiated).  With A omega = b,
        d omega = A^{-1} (db - dA omega),   db = (dphi, 0, ..., 0),
        dU = (dU/dgeometry)[d] + (dU/domega)[d omega],
        dJ = sum_m 2 w_m U_m dU_m,
    where dA omega and both parts of dU are forward-mode derivatives of the
    assembly (row chunks of A times the fixed omega) and of the U map.
    solve(r) must return A^{-1} r for the matrix at (xt, yt); omega, when
    given, is the solution at the base state.  Returns (J, U, omega, [dJ_i],
    [dU_i])."""
    xt = torch.as_tensor(xt, dtype=F64)
    yt = torch.as_tensor(yt, dtype=F64)
    phi = torch.as_tensor(phi, dtype=F64)
    w = torch.as_tensor(weights, dtype=F64)

    def geom(a, b):
        z0, d0, e0 = surface_from_periodic(a, b)
        return g_walls.with_surface(z0, d0, e0)

    g0 = geom(xt, yt)
    if omega is None:
        omega = solve(rhs(g0, phi))
    n = omega.shape[0]

    def u_of(a, b, om):
        return dphi_dn_from_omega_chunked(geom(a, b), split(g_walls, om))

    U = u_of(xt, yt, omega)
    J = float((w * U * U).sum())
    dJ, dUs = [], []
    for d in dirs:
        dx, dy, dp = (torch.as_tensor(v, dtype=F64) for v in d)
        dAw = []
        for r0 in range(0, n, chunk):
            rows = range(r0, min(n, r0 + chunk))
            f = lambda a, b: A_rows(geom(a, b), rows) @ omega
            dAw.append(torch.func.jvp(f, (xt, yt), (dx, dy))[1])
        dAw = torch.cat(dAw)
        db = torch.cat([dp, torch.zeros(n - dp.shape[0], dtype=F64)])
        dom = solve(db - dAw)
        dU = torch.func.jvp(u_of, (xt, yt, omega), (dx, dy, dom))[1]
        dUs.append(dU)
        dJ.append(float((2.0 * w * U * dU).sum()))
    return J, U, omega, dJ, dUs


def tangent_J_nodes(g: OGeom, phi, weights, dirs, solve, omega=None, chunk: int = 1024):
    """Directional derivatives of J = sum_m w_m U_m^2 along directions of the
    surface's node data and potential, walls fixed: each direction gives the
    changes of (x, y, x', y', x'', y'') at the surface nodes and of phi~, so
    no derivative of the direction is taken numerically.  The same
    tangent-linear model as tangent_J (Sec. 3.2-3.4 differentiated):
        d omega = A^{-1} (db - dA omega),   db = (dphi, 0, ..., 0),
        dU = (dU/dnodes)[d] + (dU/domega)[d omega],  dJ = sum_m 2 w_m U_m dU_m,
    with dA omega and dU forward-mode derivatives of the assembly (row chunks
    of A times the fixed omega) and of the U map with respect to the six node
    arrays.  solve(r) returns A^{-1} r for the matrix of g; omega, when given,
    is the solution at g.  Returns (J, U, omega, [dJ_i], [dU_i])."""
    phi = torch.as_tensor(phi, dtype=F64)
    w = torch.as_tensor(weights, dtype=F64)
    base = (g.z[0].real, g.z[0].imag, g.d[0].real, g.d[0].imag, g.e[0].real, g.e[0].imag)

    def geom(x, y, dx, dy, ex, ey):
        return g.with_surface(x + 1j * y, dx + 1j * dy, ex + 1j * ey)

    if omega is None:
        omega = solve(rhs(g, phi))
    n = omega.shape[0]

    def u_of(x, y, dx, dy, ex, ey, om):
        return dphi_dn_from_omega_chunked(geom(x, y, dx, dy, ex, ey), split(g, om))

    U = u_of(*base, omega)
    J = float((w * U * U).sum())
    dJ, dUs = [], []
    for d in dirs:
        tang = tuple(torch.as_tensor(v, dtype=F64) for v in d[:6])
        dp = torch.as_tensor(d[6], dtype=F64)
        dAw = []
        for r0 in range(0, n, chunk):
            rows = range(r0, min(n, r0 + chunk))
            f = lambda *a: A_rows(geom(*a), rows) @ omega
            dAw.append(torch.func.jvp(f, base, tang)[1])
        dAw = torch.cat(dAw)
        db = torch.cat([dp, torch.zeros(n - dp.shape[0], dtype=F64)])
        dom = solve(db - dAw)
        dU = torch.func.jvp(u_of, base + (omega,), tang + (dom,))[1]
        dUs.append(dU)
        dJ.append(float((2.0 * w * U * dU).sum()))
    return J, U, omega, dJ, dUs


def J_and_grad_nodes(g: OGeom, phi, weights):
    """J = sum_m w_m U_m^2 and its gradient with respect to the surface's node
    data (x, y, x', y', x'', y'') and phi~ by autograd through the dense
    solve, walls fixed.  Returns (J, [g_x, g_y, g_x', g_y', g_x'', g_y'',
    g_phi], U)."""
    arrs = [v.clone().requires_grad_(True) for v in
            (g.z[0].real, g.z[0].imag, g.d[0].real, g.d[0].imag, g.e[0].real, g.e[0].imag)]
    ph = torch.as_tensor(phi, dtype=F64).clone().requires_grad_(True)
    w = torch.as_tensor(weights, dtype=F64)
    x, y, dx, dy, ex, ey = arrs
    gs = g.with_surface(x + 1j * y, dx + 1j * dy, ex + 1j * ey)
    U = solve_phi(gs, ph)["U"]
    J = (w * U * U).sum()
    grads = torch.autograd.grad(J, arrs + [ph])
    return float(J.detach()), [v.detach() for v in grads], U.detach()
