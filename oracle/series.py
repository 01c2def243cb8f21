"""Closed-form scattering of the plane wave exp(ikz) by one sphere (pins only).

Test infrastructure only (see the package docstring).

The paper checks its boundary-integral solutions against the analytical series
of spherical harmonics and Bessel functions (Sec. IV A).  With the outgoing
convention of Eq. inverseFourier (radiation as e^{ikr}):

    exp(ikz) = sum_n i^n (2n+1) j_n(kr) P_n(cos theta)
    P_scat   = sum_n A_n h_n(kr) P_n(cos theta),   h_n = j_n + i y_n

with A_n = -i^n (2n+1) j_n(ka)/h_n(ka) for a sound-soft sphere (P = 0 on r = a)
and A_n = -i^n (2n+1) j_n'(ka)/h_n'(ka) for a sound-hard sphere (dP/dr = 0).
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def _nmax(k, a, extra=30):
    return int(k * a) + extra


def coefficients(k: float, a: float, bc: str):
    nmax = _nmax(k, a)
    n = np.arange(nmax + 1)
    ka = k * a
    pref = (1j ** n) * (2 * n + 1)
    if bc == "soft":
        h = spherical_jn(n, ka) + 1j * spherical_yn(n, ka)
        A = -pref * spherical_jn(n, ka) / h
    elif bc == "hard":
        hp = spherical_jn(n, ka, derivative=True) + 1j * spherical_yn(n, ka, derivative=True)
        A = -pref * spherical_jn(n, ka, derivative=True) / hp
    else:
        raise ValueError(bc)
    return n, A


def scattered(k: float, a: float, bc: str, xp, center=(0.0, 0.0, 0.0)):
    """Scattered field at points xp (outside the sphere)."""
    n, A = coefficients(k, a, bc)
    A = A * np.exp(1j * k * center[2])
    d = xp - np.asarray(center)[None, :]
    r = np.sqrt(np.sum(d * d, axis=1))
    ct = d[:, 2] / r
    out = np.zeros(xp.shape[0], dtype=np.complex128)
    for nn in n:
        h = spherical_jn(nn, k * r) + 1j * spherical_yn(nn, k * r)
        out += A[nn] * h * eval_legendre(nn, ct)
    return out


def surface(k: float, a: float, bc: str, xs, center=(0.0, 0.0, 0.0)):
    """(P_scat, dP_scat/dr) at surface points xs of the sphere (r = a)."""
    n, A = coefficients(k, a, bc)
    A = A * np.exp(1j * k * center[2])
    d = xs - np.asarray(center)[None, :]
    r = np.sqrt(np.sum(d * d, axis=1))
    ct = d[:, 2] / r
    ka = k * a
    phi = np.zeros(xs.shape[0], dtype=np.complex128)
    psi = np.zeros(xs.shape[0], dtype=np.complex128)
    for nn in n:
        h = spherical_jn(nn, ka) + 1j * spherical_yn(nn, ka)
        hp = spherical_jn(nn, ka, derivative=True) + 1j * spherical_yn(nn, ka, derivative=True)
        P = eval_legendre(nn, ct)
        phi += A[nn] * h * P
        psi += A[nn] * k * hp * P
    return phi, psi


def far_field(k: float, a: float, bc: str, cos_theta):
    """Far-field amplitude f(theta): P_scat ~ f e^{ikr}/r."""
    n, A = coefficients(k, a, bc)
    out = np.zeros(np.shape(cos_theta), dtype=np.complex128)
    for nn in n:
        out += A[nn] * ((-1j) ** (nn + 1)) / k * eval_legendre(nn, cos_theta)
    return out
