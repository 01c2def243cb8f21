"""Oracle of the interior-point remedy for fictitious resonances.

Test infrastructure only (see the package docstring).

At wavenumbers where the interior of a scatterer has an eigenvalue, the
surface equation of Eq. BRIEF loses its uniqueness: its matrix becomes nearly
singular and the solution picks up a spurious interior mode (Sec. IV A avoids
those wavenumbers by choosing the pulse period).  The classical remedy
(combined Helmholtz integral equation, Schenck 1968) adds conditions at points
x_c strictly inside the bodies: for the radiating scattered field, Green's
second identity on the exterior domain gives, with normals out of the body,

    4 pi P(x) = integral over S of (P dG/dn - G dP/dn) dS     (x in the fluid)
            0 = integral over S of (P dG/dn - G dP/dn) dS     (x inside a body)

G = exp(ik|x' - x|)/|x' - x|, dG/dn the derivative at the surface point x'.
With the nodal quadrature of the surface equation (weights w_j) the interior
condition at x_c reads

    sum_j w_j (phi_j H_cj - psi_j G_cj) = 0,   d = x_j - x_c,
    G_cj = e^{ikr}/r,  H_cj = e^{ikr}(ikr - 1)(d.n_j)/r^3.

Split by the boundary conditions as for the surface equation (hard nodes:
unknown phi, soft nodes: unknown psi), each point gives one more row C x = d
with C_cj = w_j H_cj (hard j) or -w_j G_cj (soft j) and d = -(B_c y), B_c the
other columns.  The surface rows and the interior rows together are solved in
the least-squares sense (here LAPACK's least-squares solver on the stacked
system).  Away from resonances the interior rows hold up to the
discretisation error and the solution moves by that much; at a resonance they
remove the spurious mode.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import bie
from .mesh import Surface

HARD = bie.HARD


def interior_kernels(surf: Surface, k: float, xc):
    """w_j H_cj and w_j G_cj, [len(xc), N] complex128."""
    xc = np.asarray(xc, dtype=np.float64)
    d0 = surf.x[None, :, 0] - xc[:, None, 0]
    d1 = surf.x[None, :, 1] - xc[:, None, 1]
    d2 = surf.x[None, :, 2] - xc[:, None, 2]
    r = np.sqrt((d0 * d0 + d1 * d1) + d2 * d2)
    E = np.exp(1j * k * r)
    dn = (d0 * surf.nrm[None, :, 0] + d1 * surf.nrm[None, :, 1]) + d2 * surf.nrm[None, :, 2]
    H = E * (1j * k * r - 1.0) * dn / (r * r * r)
    G = E / r
    return surf.w[None, :] * H, surf.w[None, :] * G


def interior_rows(surf: Surface, k: float, xc, y):
    """C, d of the interior conditions C x = d for known data y ([N] or [N, n_rhs])."""
    wH, wG = interior_kernels(surf, k, xc)
    hard = surf.bc == HARD
    C = np.where(hard[None, :], wH, -wG)
    Bc = np.where(hard[None, :], -wG, wH)
    return C, -(Bc @ y)


def solve(surf: Surface, k: float, y, xc):
    """Least-squares solution of the surface rows and the interior rows for
    one wavenumber.  Returns (phi, psi, unknowns)."""
    A, b = bie.system(surf, k, y)
    C, d = interior_rows(surf, k, xc, y)
    xs = scipy.linalg.lstsq(np.vstack([A, C]), np.concatenate([b, d]))[0]
    phi, psi = bie.split_unknowns(surf, xs, y)
    return phi, psi, xs
