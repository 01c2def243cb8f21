"""Pins of the oracle's discrete non-singular boundary integral equation.

Each check is fixed by something other than the oracle itself: 50-digit brute
force of the kernel entries, exact radiating solutions (monopoles), the
closed-form sphere series, the optical theorem and reciprocity, and the
closed-form S_inf integrals of Appendix B.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import roots_legendre

from oracle import bie, series
from oracle.mesh import Surface
from workloads import Body, HARD, SOFT


def sphere(level, bc=HARD, center=(0.0, 0.0, 0.0), radius=1.0, aspect=1.0, rescale=True):
    return Surface([Body(center, radius, aspect, level, bc)], rescale_area=rescale)


def monopole(surf, k, src):
    d = surf.x - np.asarray(src)
    r = np.linalg.norm(d, axis=1)
    p = np.exp(1j * k * r) / r
    dpdn = p * (1j * k * r - 1.0) / r * np.sum(d * surf.nrm, axis=1) / r
    return p, dpdn


# ---------------------------------------------------------------- brute force
def _mp_entries(surf, k, i):
    """Row i of M_phi and M_psi in 50-digit arithmetic, written from the
    discrete equation term by term."""
    mp.mp.dps = 50
    N = surf.n
    x = [[mp.mpf(float(v)) for v in row] for row in surf.x]
    n = [[mp.mpf(float(v)) for v in row] for row in surf.nrm]
    w = [mp.mpf(float(v)) for v in surf.w]
    K = mp.mpf(k)
    I = mp.mpc(0, 1)
    rphi = [mp.mpc(0)] * N
    rpsi = [mp.mpc(0)] * N
    dphi = mp.mpc(4) * mp.pi
    dpsi = mp.mpc(0)
    for j in range(N):
        if j == i:
            continue
        d = [x[j][a] - x[i][a] for a in range(3)]
        r = mp.sqrt(sum(t * t for t in d))
        E = mp.exp(I * K * r)
        G = E / r
        H = E * (I * K * r - 1) * sum(d[a] * n[j][a] for a in range(3)) / r ** 3
        s = K * sum(n[i][a] * d[a] for a in range(3))
        nn = sum(n[i][a] * n[j][a] for a in range(3))
        g, f = mp.cos(s), mp.sin(s) / K
        gp, fp = -K * mp.sin(s) * nn, mp.cos(s) * nn
        rphi[j] = -w[j] * H
        rpsi[j] = w[j] * G
        dphi -= w[j] * (gp * G - g * H)
        dpsi -= w[j] * (fp * G - f * H)
    rphi[i] = dphi
    rpsi[i] = dpsi
    return (np.array([complex(v) for v in rphi]), np.array([complex(v) for v in rpsi]))


@pytest.mark.parametrize("level,k,rows", [(0, 1.3, [0, 5, 11]), (1, 4.7, [0, 17, 41])])
def test_entries_vs_50_digit_brute_force(level, k, rows):
    s = sphere(level, center=(0.2, -0.1, 0.4), radius=0.9, aspect=1.3)
    Mphi, Mpsi = bie.operator_matrices(s, k)
    for i in rows:
        ephi, epsi = _mp_entries(s, k, i)
        scale_phi = np.max(np.abs(ephi))
        scale_psi = np.max(np.abs(epsi))
        assert np.max(np.abs(Mphi[i] - ephi)) / scale_phi < 1e-13
        assert np.max(np.abs(Mpsi[i] - epsi)) / scale_psi < 1e-13


# ---------------------------------------------------------------- f and g
def test_f_g_conditions_of_appendix_A():
    # f(x0) = 0, n0.grad f(x0) = 1, g(x0) = 1, n0.grad g(x0) = 0, and both solve
    # the Helmholtz equation (checked by finite differences).
    rng = np.random.default_rng(3)
    k = 2.3
    n0 = rng.standard_normal(3); n0 /= np.linalg.norm(n0)
    x0 = rng.standard_normal(3)
    f = lambda x: np.sin(k * n0 @ (x - x0)) / k
    g = lambda x: np.cos(k * n0 @ (x - x0))
    h = 1e-4
    for fun, val, dn in ((f, 0.0, 1.0), (g, 1.0, 0.0)):
        assert abs(fun(x0) - val) < 1e-15
        assert abs((fun(x0 + h * n0) - fun(x0 - h * n0)) / (2 * h) - dn) < 1e-7
        xp = x0 + rng.standard_normal(3)
        lap = sum((fun(xp + h * e) - 2 * fun(xp) + fun(xp - h * e)) / h ** 2 for e in np.eye(3))
        assert abs(lap + k * k * fun(xp)) < 1e-5


# ---------------------------------------------------------------- S_inf
@pytest.mark.parametrize("k", [0.7, 2.0])
def test_s_inf_integrals_appendix_B(k):
    # Direct quadrature of I1, I2 on a sphere of radius R about x0 (outward
    # normal r/R).  I1 -> +4 pi (the value that yields the stated "4 pi P(x0)
    # on the left hand side"; the printed -4 pi carries a sign slip), I2 -> 0.
    u, wq = roots_legendre(4000)
    for R in (200.0, 2000.0):
        E = np.exp(1j * k * R)
        G = E / R
        dG = E * (1j * k * R - 1.0) / R ** 2
        g = np.cos(k * R * u)
        dg = -k * u * np.sin(k * R * u)
        f = np.sin(k * R * u) / k
        df = u * np.cos(k * R * u)
        dS = 2 * np.pi * R * R
        I1 = dS * np.sum(wq * (dg * G - dG * g))
        I2 = dS * np.sum(wq * (df * G - dG * f))
        assert abs(I1 - 4 * np.pi) < 4 * np.pi * 2.0 / (k * R)
        assert abs(I2) < 4 * np.pi * 2.0 / (k * R)


# ---------------------------------------------------------------- monopole
@pytest.mark.parametrize("bc", [HARD, SOFT])
def test_monopole_residual_converges(bc):
    k, src = 1.7, (0.15, -0.2, 0.3)
    res = []
    for L in (1, 2, 3):
        s = sphere(L, bc)
        p, dp = monopole(s, k, src)
        R = bie.residual(s, k, p, dp)
        res.append(np.linalg.norm(R) / np.linalg.norm(4 * np.pi * p))
    assert res[2] < 3e-4
    assert res[0] / res[1] > 3.0 and res[1] / res[2] > 3.0


def test_monopole_sign_of_s_inf_term_matters():
    # Reading the S_inf term with the printed I1 = -4 pi turns 4 pi phi_i into
    # -4 pi phi_i; the exact radiating data then fails the equation at O(1).
    s = sphere(3)
    p, dp = monopole(s, 1.7, (0.1, 0.0, -0.2))
    R = bie.residual(s, 1.7, p, dp)
    R_wrong = R - 8 * np.pi * p
    assert np.linalg.norm(R_wrong) / np.linalg.norm(4 * np.pi * p) > 1.0


@pytest.mark.parametrize("bc", [HARD, SOFT])
def test_monopole_solve(bc):
    k, src = 2.2, (0.0, 0.3, -0.2)
    s = sphere(3, bc, aspect=1.4)
    p, dp = monopole(s, k, src)
    y = np.where(s.bc == HARD, dp, p)
    A, b = bie.system(s, k, y)
    xs = np.linalg.solve(A, b)
    ref = np.where(s.bc == HARD, p, dp)
    assert np.linalg.norm(xs - ref) / np.linalg.norm(ref) < 5e-3


# ---------------------------------------------------------------- sphere series
@pytest.mark.parametrize("bc,k", [("hard", 1.0), ("hard", 3.0), ("soft", 1.0), ("soft", 2.6)])
def test_sphere_series_surface(bc, k):
    errs = []
    for L in (2, 3):
        s = sphere(L, HARD if bc == "hard" else SOFT)
        phi, psi = bie.scatter_plane_wave(s, k)
        ph_s, ps_s = series.surface(k, 1.0, bc, s.x)
        got, ref = (phi, ph_s) if bc == "hard" else (psi, ps_s)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert errs[1] < errs[0]
    assert errs[1] < (2e-3 if bc == "hard" else 1e-2)


def test_known_data_boundary_conditions():
    # hard nodes carry -dP_inc/dn, soft nodes -P_inc (Sec. IV A)
    s = Surface([Body((0, 0, -2.0), 1.0, 1.0, 1, HARD), Body((0, 0, 2.0), 1.0, 1.0, 1, SOFT)])
    p, dp = bie.incident_plane_wave(s, 1.5)
    y = bie.known_data(s, p, dp)
    assert np.allclose(y[:42], -1j * 1.5 * s.nrm[:42, 2] * np.exp(1j * 1.5 * s.x[:42, 2]))
    assert np.allclose(y[42:], -np.exp(1j * 1.5 * s.x[42:, 2]))


# ---------------------------------------------------------------- invariants
def _far(s, k, phi, psi, rhat):
    # f(rhat) = (1/4pi) sum_j w_j [-ik (rhat.n_j) phi_j - psi_j] e^{-ik rhat.x_j}
    # (far field of the exterior representation with normals out of the body)
    ph = np.exp(-1j * k * (s.x @ rhat))
    return np.sum(s.w * (-1j * k * (s.nrm @ rhat) * phi - psi) * ph) / (4 * np.pi)


def test_far_field_matches_series_and_optical_theorem():
    k = 1.3
    s = sphere(3)
    phi, psi = bie.scatter_plane_wave(s, k)
    ct = np.array([1.0, 0.5, -0.3, -1.0])
    st = np.sqrt(1 - ct ** 2)
    ff = np.array([_far(s, k, phi, psi, np.array([st[i], 0, ct[i]])) for i in range(4)])
    ref = series.far_field(k, 1.0, "hard", ct)
    assert np.max(np.abs(ff - ref)) / np.max(np.abs(ref)) < 3e-3
    # optical theorem on the BEM far field: int |f|^2 dOmega = (4 pi/k) Im f(dhat)
    u, wq = roots_legendre(40)
    tot = 0.0
    for ui, wi in zip(u, wq):
        sti = math.sqrt(1 - ui * ui)
        for ph in np.linspace(0, 2 * np.pi, 24, endpoint=False):
            fr = _far(s, k, phi, psi, np.array([sti * math.cos(ph), sti * math.sin(ph), ui]))
            tot += wi * (2 * np.pi / 24) * abs(fr) ** 2
    fwd = _far(s, k, phi, psi, np.array([0.0, 0.0, 1.0]))
    assert abs(tot - 4 * np.pi / k * fwd.imag) / tot < 5e-3


def test_two_sphere_reciprocity_and_energy():
    k = 2.0
    bodies = [Body((0, 0, -1.5), 1.0, 1.0, 2, HARD), Body((0, 0, 1.5), 1.0, 1.0, 2, HARD)]
    s = Surface(bodies)

    def solve_dir(dh):
        dh = np.asarray(dh, float)
        p = np.exp(1j * k * (s.x @ dh))
        dp = 1j * k * (s.nrm @ dh) * p
        phi, psi, _ = bie.solve(s, k, -dp)
        return phi, -dp

    d1 = np.array([0.0, 0.6, 0.8])
    d2 = np.array([0.48, 0.0, 0.8 * math.sqrt(1 - 0.36)])
    d2 /= np.linalg.norm(d2)
    phi1, psi1 = solve_dir(d1)
    phi2, psi2 = solve_dir(-d2)
    f12 = _far(s, k, phi1, psi1, d2)       # f(d2; d1)
    f21 = _far(s, k, phi2, psi2, -d1)      # f(-d1; -d2)
    assert abs(f12 - f21) / abs(f12) < 2e-3
