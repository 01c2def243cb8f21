"""Oracle of the surface-to-field step (Sec. III, Eq. BRIEFdmn).

Test infrastructure only (see the package docstring).

For an observation point x_p in the fluid, x0 is the surface point closest to
x_p; here the closest surface *node* i0 (ties go to the lowest index, squared
distance evaluated as (dx*dx + dy*dy) + dz*dz in FP64).  With
u_j = phi_j - phi_i0 g_j - psi_i0 f_j and u'_j = psi_j - phi_i0 g'_j - psi_i0 f'_j
(f, g of Appendix A centred at x_i0 with normal n_i0),

  4 pi P(x_p) = 4 pi phi_i0
              + sum_{j != i0} w_j [ u_j (H^p_j - H_i0j) - u'_j (G^p_j - G_i0j) ]

where G^p_j, H^p_j use d = x_j - x_p.  This is Eq. BRIEFdmn with its S_inf
integrals evaluated: they contribute 4 pi [phi_i0 (1 - g(x_p)) - psi_i0 f(x_p)],
which turns the constant term of the printed formula into 4 pi phi_i0 when the
integrals are taken over S alone (normals out of the body).  The j = i0 term is
exactly zero (u = u' = 0) and is skipped.

A point is inside a body when n_i0.(x_p - x_i0) < 0 (dot product evaluated as
(n0*d0 + n1*d1) + n2*d2); its field is defined as 0.
"""
from __future__ import annotations

import numpy as np

from .mesh import Surface

FOUR_PI = 4.0 * np.pi


def closest_node(x, xp):
    """i0[p] = argmin_j |x_p - x_j|^2, FP64, ties -> lowest j."""
    M = xp.shape[0]
    out = np.empty(M, dtype=np.int32)
    for p0 in range(0, M, 2048):
        q = xp[p0:p0 + 2048]
        d0 = q[:, None, 0] - x[None, :, 0]
        d1 = q[:, None, 1] - x[None, :, 1]
        d2 = q[:, None, 2] - x[None, :, 2]
        dist = (d0 * d0 + d1 * d1) + d2 * d2
        out[p0:p0 + 2048] = np.argmin(dist, axis=1)   # first minimum = lowest index
    return out


def inside_mask(x, nrm, xp, i0):
    d = xp - x[i0]
    nd = (nrm[i0, 0] * d[:, 0] + nrm[i0, 1] * d[:, 1]) + nrm[i0, 2] * d[:, 2]
    return (nd < 0.0).astype(np.uint8)


def field(surf: Surface, k: float, phi, psi, xp, i0=None):
    """Scattered field P at points xp for surface data (phi, psi) at wavenumber k.

    Returns (P [M] complex128, i0 [M] int32, inside [M] uint8)."""
    x, nrm, w = surf.x, surf.nrm, surf.w
    if i0 is None:
        i0 = closest_node(x, xp)
    inside = inside_mask(x, nrm, xp, i0)
    N = surf.n
    P = np.zeros(xp.shape[0], dtype=np.complex128)
    for p in range(xp.shape[0]):
        if inside[p]:
            continue
        a = int(i0[p])
        # kernel from the closest node x_a and from the field point x_p
        da = x - x[a]
        ra = np.sqrt((da[:, 0] * da[:, 0] + da[:, 1] * da[:, 1]) + da[:, 2] * da[:, 2])
        dp = x - xp[p]
        rp = np.sqrt((dp[:, 0] * dp[:, 0] + dp[:, 1] * dp[:, 1]) + dp[:, 2] * dp[:, 2])
        mask = np.arange(N) != a
        ra = np.where(mask, ra, 1.0)
        rp = np.where(mask, rp, 1.0)
        dna = (da[:, 0] * nrm[:, 0] + da[:, 1] * nrm[:, 1]) + da[:, 2] * nrm[:, 2]
        dnp = (dp[:, 0] * nrm[:, 0] + dp[:, 1] * nrm[:, 1]) + dp[:, 2] * nrm[:, 2]
        Ea = np.exp(1j * k * ra)
        Ep = np.exp(1j * k * rp)
        Ga = Ea / ra
        Gp = Ep / rp
        Ha = Ea * (1j * k * ra - 1.0) * dna / (ra * ra * ra)
        Hp = Ep * (1j * k * rp - 1.0) * dnp / (rp * rp * rp)
        s = k * ((nrm[a, 0] * da[:, 0] + nrm[a, 1] * da[:, 1]) + nrm[a, 2] * da[:, 2])
        nn = (nrm[a, 0] * nrm[:, 0] + nrm[a, 1] * nrm[:, 1]) + nrm[a, 2] * nrm[:, 2]
        g = np.cos(s)
        f = np.sin(s) / k
        gp = -k * np.sin(s) * nn
        fp = np.cos(s) * nn
        u = phi - phi[a] * g - psi[a] * f
        up = psi - phi[a] * gp - psi[a] * fp
        terms = w * (u * (Hp - Ha) - up * (Gp - Ga))
        terms = np.where(mask, terms, 0.0)
        P[p] = phi[a] + np.sum(terms) / FOUR_PI
    return P, i0, inside


def plane_wave_at(xp, k, direction=(0.0, 0.0, 1.0)):
    dz = (xp[:, 0] * direction[0] + xp[:, 1] * direction[1]) + xp[:, 2] * direction[2]
    return np.exp(1j * k * dz)
