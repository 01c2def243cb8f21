"""Oracle of the incident pulse spectrum and the time synthesis.

Test infrastructure only (see the package docstring).

Conventions (Sec. III, Eq. inverseFourier): h(t) = (1/2pi) int H(w) e^{-iwt} dw,
so a frequency component travels as e^{i(kz - wt)} with w = k (c = 1) and the
scattered field of a unit plane wave e^{ikz} radiates as e^{ikr}.

The incident field is a periodic train F(z - t - z_s) of period L (Sec. IV:
the fundamental pulse is replicated into an infinite train).  Sampling F at T
evenly spaced points s_n = -L/2 + n L/T (left-closed, n = 0..T-1) and taking
the DFT gives the Fourier coefficients

    c_m = (1/T) sum_n F(s_n) exp(-i k_m s_n) * exp(-i k_m z_s),   k_m = 2 pi m / L.

The space-time field at t_n = n L/T is then the inverse DFT over m:

    p(x, t_n) = sum_{m=1}^{F} alpha_m Re[ c_m U_m(x) exp(-2 pi i m n / T) ],

alpha_m = 2 for m < T/2 and 1 for m = T/2, where U_m is the field per unit
incident amplitude at k_m (scattered, optionally plus the incident e^{ik_m z}).
The m = 0 term is not part of the solved grid (k > 0) and is left out.

For the paper's pulse (Eq. pulse), tau = k0 s with k0 = 8 pi N_c / w, the
period is L = w and the time origin (pulse front touching the sphere at z = -a
at t = 0, Sec. IV A) is z_s = -(a + w/4); with the left-closed sampling this
reproduces the phase factor e^{i beta}, beta = -k_m a [w/(4a) - 1].
"""
from __future__ import annotations

import numpy as np


def pulse_samples(pulse, s):
    """F(s) of the pulse kinds used by the workloads."""
    p = pulse.params
    kind = pulse.kind
    if kind == "paper":
        Nc, alpha, w = p["Nc"], p["alpha"], p["w"]
        k0 = 8.0 * np.pi * Nc / w
        tau = k0 * s
        return np.where(np.abs(tau) < 2.0 * np.pi * Nc, np.sin(tau) * np.exp(-alpha * np.abs(tau)), 0.0)
    if kind == "gauss":
        sg = p["sigma"]
        return np.exp(-(s * s) / (2.0 * sg * sg))
    if kind == "ricker":
        sg = p["sigma"]
        q = (s * s) / (sg * sg)
        return (1.0 - q) * np.exp(-0.5 * q)
    if kind == "nwave":
        sg = p["sigma"]
        return np.where(np.abs(s) <= sg, s / sg, 0.0)
    if kind == "chirp":
        ka, kb, D = p["ka"], p["kb"], p["D"]
        return np.sin(ka * s + (kb - ka) * (s * s) / (2.0 * D)) * np.exp(-(s * s) / (2.0 * D * D))
    if kind == "gsine":
        k0, sg = p["k0"], p["sigma"]
        return np.sin(k0 * s) * np.exp(-(s * s) / (2.0 * sg * sg))
    raise ValueError(kind)


def sample_points(L: float, T: int):
    return -0.5 * L + np.arange(T, dtype=np.float64) * (L / T)


def coefficients(pulse, n_k: int, dk: float, T: int, z_shift: float):
    """c_m for m = 1..n_k on the grid k_m = m dk (see module docstring).

    The spectral pulse 'gaussk' is defined directly in k:
    c(k) = exp(-(k - k0)^2 / (2 width^2)) (Gaussian spectrum centred at k0)."""
    k = dk * np.arange(1, n_k + 1, dtype=np.float64)
    if pulse.kind == "gaussk":
        k0, wd = pulse.params["k0"], pulse.params["width"]
        c = np.exp(-((k - k0) ** 2) / (2.0 * wd * wd)).astype(np.complex128)
    else:
        L = 2.0 * np.pi / dk
        s = sample_points(L, T)
        F = pulse_samples(pulse, s)
        c = np.array([np.sum(F * np.exp(-1j * km * s)) for km in k]) / T
    return c * np.exp(-1j * k * z_shift)


def paper_time_shift(a: float, w: float) -> float:
    """z_s = -(a + w/4): the oscillatory front reaches z = -a at t = 0."""
    return -(a + 0.25 * w)


def synthesize(U, c, T: int, xp=None, dk=None, add_incident=False):
    """p[M, T] from U[M, F] (field per unit amplitude at k_m = m dk, m = 1..F)
    and the coefficients c[F]; the inverse DFT is numpy's irfft."""
    U = np.atleast_2d(U)
    M, F = U.shape
    assert 2 * F <= T
    X = U * c[None, :]
    if add_incident:
        k = dk * np.arange(1, F + 1, dtype=np.float64)
        X = X + c[None, :] * np.exp(1j * xp[:, 2:3] * k[None, :])
    Y = np.zeros((M, T // 2 + 1), dtype=np.complex128)
    Y[:, 1:F + 1] = np.conj(X)
    return T * np.fft.irfft(Y, n=T, axis=1)


def synthesize_direct(U, c, T: int):
    """The same inverse DFT written out as an explicit sum (small sizes only)."""
    U = np.atleast_2d(U)
    M, F = U.shape
    n = np.arange(T)
    out = np.zeros((M, T))
    for m in range(1, F + 1):
        alpha = 1.0 if 2 * m == T else 2.0
        out += alpha * np.real(c[m - 1] * U[:, m - 1:m] * np.exp(-2j * np.pi * m * n[None, :] / T))
    return out


def dominant(c, n_keep: int):
    """Indices of the n_keep largest |c_m| (stable: ties by lower m)."""
    order = np.lexsort((np.arange(len(c)), -np.abs(c)))
    return np.sort(order[:n_keep])


def rms_error_percent(p_trunc, p_full):
    """100 * RMS_t(p_trunc - p_full) / max_t |p_full| (reading of Table 1)."""
    return 100.0 * np.sqrt(np.mean((p_trunc - p_full) ** 2)) / np.max(np.abs(p_full))
