"""Oracle of the per-frequency non-singular boundary integral equation.

Test infrastructure only (see the package docstring).

Continuous statement (Sec. III, Eq. BRIEF with Eqs. Green_func, fEqn, gEqn):
for a collocation point x0 on S, with u(x) = P(x) - P(x0) g(x) - P'(x0) f(x),

    integral over S+S_inf of  u dG/dn  =  integral over S+S_inf of  (du/dn) G ,

G(x0,x) = exp(ik|x-x0|)/|x-x0|, and (Appendix A) f = sin(k n0.(x-x0))/k,
g = cos(k n0.(x-x0)).  The S_inf integrals are evaluated in closed form in
Appendix B and leave the term 4 pi P(x0) (the derivation there carries a sign
slip in the value printed for I1; direct evaluation gives I1 = +4 pi, which is
the value consistent with the stated "4 pi P(x0) on the left hand side").

Discretisation (nodal quadrature with weights w_j, collocation at the nodes,
normals n out of the body):

    4 pi phi_i + sum_{j!=i} w_j [psi_j - phi_i g'_ij - psi_i f'_ij] G_ij
               = sum_{j!=i} w_j [phi_j - phi_i g_ij  - psi_i f_ij ] H_ij

with d = x_j - x_i, r = |d|, G_ij = e^{ikr}/r, H_ij = dG/dn_j =
e^{ikr}(ikr-1)(d.n_j)/r^3, s = k n_i.d, g = cos s, f = sin(s)/k,
g' = -k sin(s) (n_i.n_j), f' = cos(s) (n_i.n_j).  The j = i term is omitted:
both brackets vanish there (u(x0) = 0 and du/dn(x0) = 0 by Eqs. fEqn, gEqn).
Collecting terms gives M_phi phi + M_psi psi = 0 with

    (M_phi)_ij = -w_j H_ij,   (M_phi)_ii = 4 pi - sum_{j!=i} w_j (g'_ij G_ij - g_ij H_ij)
    (M_psi)_ij =  w_j G_ij,   (M_psi)_ii =      - sum_{j!=i} w_j (f'_ij G_ij - f_ij H_ij).

Boundary conditions for the scattered field (Sec. IV A): sound-hard nodes know
psi = -dP_inc/dn and solve for phi; sound-soft nodes know phi = -P_inc and solve
for psi.  Column j of the system matrix A is column j of M_phi (hard) or M_psi
(soft); B holds the other columns; A x = -B y.  The paper solves this dense
system with a direct method (Sec. IV A); here LAPACK zgetrf/zgetrs.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .mesh import Surface

HARD = 0
SOFT = 1
FOUR_PI = 4.0 * np.pi


def pair_terms(x, nrm, k, rows):
    """G, H, g, f, g', f' for collocation nodes ``rows`` against every node j.

    Arrays are [len(rows), N]; the self entries (j == i) are set to zero.
    """
    rows = np.asarray(rows)
    xi = x[rows]
    ni = nrm[rows]
    d0 = x[None, :, 0] - xi[:, None, 0]
    d1 = x[None, :, 1] - xi[:, None, 1]
    d2 = x[None, :, 2] - xi[:, None, 2]
    self_mask = rows[:, None] == np.arange(x.shape[0])[None, :]
    r = np.sqrt((d0 * d0 + d1 * d1) + d2 * d2)
    r = np.where(self_mask, 1.0, r)
    E = np.exp(1j * k * r)
    G = E / r
    dn_j = (d0 * nrm[None, :, 0] + d1 * nrm[None, :, 1]) + d2 * nrm[None, :, 2]
    H = E * (1j * k * r - 1.0) * dn_j / (r * r * r)
    s = k * ((ni[:, 0:1] * d0 + ni[:, 1:2] * d1) + ni[:, 2:3] * d2)
    nn = (ni[:, 0:1] * nrm[None, :, 0] + ni[:, 1:2] * nrm[None, :, 1]) + ni[:, 2:3] * nrm[None, :, 2]
    g = np.cos(s)
    f = np.sin(s) / k
    gp = -k * np.sin(s) * nn
    fp = np.cos(s) * nn
    z = np.zeros_like(G)
    G = np.where(self_mask, z, G)
    H = np.where(self_mask, z, H)
    g = np.where(self_mask, 0.0, g)
    f = np.where(self_mask, 0.0, f)
    gp = np.where(self_mask, 0.0, gp)
    fp = np.where(self_mask, 0.0, fp)
    return G, H, g, f, gp, fp


def operator_matrices(surf: Surface, k: float, chunk: int = 512):
    """Dense M_phi, M_psi (N x N complex128) of the discrete equation above."""
    N = surf.n
    Mphi = np.empty((N, N), dtype=np.complex128)
    Mpsi = np.empty((N, N), dtype=np.complex128)
    w = surf.w
    for r0 in range(0, N, chunk):
        rows = np.arange(r0, min(N, r0 + chunk))
        G, H, g, f, gp, fp = pair_terms(surf.x, surf.nrm, k, rows)
        Mphi[rows] = -w[None, :] * H
        Mpsi[rows] = w[None, :] * G
        dphi = FOUR_PI - np.sum(w[None, :] * (gp * G - g * H), axis=1)
        dpsi = -np.sum(w[None, :] * (fp * G - f * H), axis=1)
        Mphi[rows, rows] = dphi
        Mpsi[rows, rows] = dpsi
    return Mphi, Mpsi


def incident_plane_wave(surf: Surface, k: float, direction=(0.0, 0.0, 1.0)):
    """P_inc = exp(ik dhat.x) and dP_inc/dn = ik (dhat.n) P_inc at the nodes."""
    dx = (surf.x[:, 0] * direction[0] + surf.x[:, 1] * direction[1]) + surf.x[:, 2] * direction[2]
    dn = (surf.nrm[:, 0] * direction[0] + surf.nrm[:, 1] * direction[1]) + surf.nrm[:, 2] * direction[2]
    p = np.exp(1j * k * dx)
    return p, 1j * k * dn * p


def known_data(surf: Surface, p_inc, dp_inc):
    """Known surface data of the scattered field: -dP_inc/dn on hard nodes,
    -P_inc on soft nodes (Sec. IV A)."""
    return np.where(surf.bc == HARD, -dp_inc, -p_inc)


def system(surf: Surface, k: float, y):
    """A, b of A x = -B y for the BC column selection described above."""
    Mphi, Mpsi = operator_matrices(surf, k)
    hard = surf.bc == HARD
    A = np.where(hard[None, :], Mphi, Mpsi)
    B = np.where(hard[None, :], Mpsi, Mphi)
    b = -(B @ y)
    return A, b


def split_unknowns(surf: Surface, xsol, y):
    """Full surface data (phi, psi) from the unknowns and the known data."""
    hard = surf.bc == HARD
    if xsol.ndim == 2:          # [N, n_rhs]
        hard = hard[:, None]
    phi = np.where(hard, xsol, y)
    psi = np.where(hard, y, xsol)
    return phi, psi


def solve(surf: Surface, k: float, y):
    """Direct dense solve of the discrete equation for one wavenumber.

    Returns (phi, psi, unknowns).  y may be [N] or [N, n_rhs]."""
    A, b = system(surf, k, y)
    lu = scipy.linalg.lu_factor(A)
    xs = scipy.linalg.lu_solve(lu, b)
    phi, psi = split_unknowns(surf, xs, y)
    return phi, psi, xs


def residual(surf: Surface, k: float, phi, psi):
    """R = M_phi phi + M_psi psi (zero for the exact discrete solution)."""
    Mphi, Mpsi = operator_matrices(surf, k)
    return Mphi @ phi + Mpsi @ psi


def scatter_plane_wave(surf: Surface, k: float):
    """Surface (phi, psi) of the field scattered from exp(ikz)."""
    p, dp = incident_plane_wave(surf, k)
    y = known_data(surf, p, dp)
    phi, psi, _ = solve(surf, k, y)
    return phi, psi
