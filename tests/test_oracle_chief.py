"""Pins of the interior-point remedy for fictitious resonances (oracle/chief.py).

Sec. IV A avoids the wavenumbers where the interior of the sphere resonates;
the remedy adds conditions at points inside the body.  Pinned here against the
sphere series (Sec. IV A's analytic check): at interior Dirichlet eigenvalues
(zeros of the spherical Bessel functions, ka = pi, 4.4934, 5.7635, 2 pi) the
plain solve is off by 18-62 % while the remedied one stays at the
discretisation error; away from them the remedy changes nothing beyond that
error; and the interior identity itself is checked with an exact radiating
field (a monopole inside the body) at interior and exterior points."""
import numpy as np
import pytest

from oracle import bie, chief, series
from oracle.mesh import Surface
from workloads import Body, HARD, SOFT, interior_points


def sphere(bc, level=3):
    body = Body((0.0, 0.0, 0.0), 1.0, 1.0, level, bc)
    return body, Surface([body])


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("bc,kind,k", [(HARD, "hard", np.pi), (HARD, "hard", 4.4934),
                                       (SOFT, "soft", 5.7635), (SOFT, "soft", 2 * np.pi)])
def test_resonance_removed(bc, kind, k):
    body, s = sphere(bc)
    xc = interior_points([body], 8, seed=1)
    p, dp = bie.incident_plane_wave(s, k)
    y = bie.known_data(s, p, dp)
    ph_s, ps_s = series.surface(k, 1.0, kind, s.x)
    ref = ph_s if bc == HARD else ps_s
    _, _, xp = bie.solve(s, k, y)
    _, _, xc_sol = chief.solve(s, k, y, xc)
    A, _ = bie.system(s, k, y)
    C, _ = chief.interior_rows(s, k, xc, y)
    assert np.linalg.cond(A) > 1e3 and np.linalg.cond(np.vstack([A, C])) < 50
    assert rel(xp, ref) > 0.1                  # the plain solve carries the spurious mode
    assert rel(xc_sol, ref) < 0.03             # the remedy leaves the discretisation error


@pytest.mark.parametrize("bc,kind", [(HARD, "hard"), (SOFT, "soft")])
def test_off_resonance_unchanged(bc, kind):
    body, s = sphere(bc)
    xc = interior_points([body], 8, seed=1)
    for k in (2.0, 2.5):
        p, dp = bie.incident_plane_wave(s, k)
        y = bie.known_data(s, p, dp)
        ph_s, ps_s = series.surface(k, 1.0, kind, s.x)
        ref = ph_s if bc == HARD else ps_s
        _, _, xp = bie.solve(s, k, y)
        _, _, xq = chief.solve(s, k, y, xc)
        assert rel(xq, xp) < 2e-3
        assert rel(xq, ref) < 1.05 * rel(xp, ref) + 1e-4


def monopole(s, k, src):
    d = s.x - src
    r = np.linalg.norm(d, axis=1)
    P = np.exp(1j * k * r) / r
    dP = P * (1j * k * r - 1.0) / r * np.sum(d * s.nrm, axis=1) / r
    return P, dP


def test_interior_identity_with_a_monopole():
    """sum_j w_j (phi H - psi G) at x_c: 0 inside the body, 4 pi P(x) outside,
    up to a quadrature error that falls with the mesh (second order)."""
    k = 1.7
    src = np.array([0.15, -0.1, 0.2])
    xin = np.array([[0.3, 0.2, -0.25], [-0.4, 0.1, 0.1]])
    xout = np.array([[1.8, 0.4, -0.6], [0.0, -2.5, 1.0]])
    errs_in, errs_out = [], []
    for level in (2, 3, 4):
        _, s = sphere(HARD, level)
        P, dP = monopole(s, k, src)
        wH, wG = chief.interior_kernels(s, k, xin)
        scale = np.abs(wH) @ np.abs(P) + np.abs(wG) @ np.abs(dP)
        errs_in.append(np.max(np.abs(wH @ P - wG @ dP) / scale))
        wH, wG = chief.interior_kernels(s, k, xout)
        r = np.linalg.norm(xout - src, axis=1)
        exact = 4 * np.pi * np.exp(1j * k * r) / r
        errs_out.append(np.max(np.abs(wH @ P - wG @ dP - exact) / np.abs(exact)))
    assert errs_in[2] < 1e-6 and errs_out[2] < 1e-5, (errs_in, errs_out)
    assert errs_in[2] < errs_in[1] / 2.5 < errs_in[0] / 6, errs_in
    assert errs_out[2] < errs_out[1] / 2.5 < errs_out[0] / 6, errs_out


def test_least_squares_conditions():
    """The returned unknowns make the stacked residual orthogonal to the
    stacked matrix's columns (the normal equations), with several rhs."""
    body, s = sphere(HARD, 2)
    k = 3.0
    xc = interior_points([body], 6, seed=4)
    y = np.random.default_rng(0).normal(size=(s.n, 3)) + 0j
    _, _, xs = chief.solve(s, k, y, xc)
    A, b = bie.system(s, k, y)
    C, d = chief.interior_rows(s, k, xc, y)
    Aa = np.vstack([A, C])
    r = Aa @ xs - np.concatenate([b, d])
    assert np.max(np.abs(Aa.conj().T @ r)) < 1e-9 * np.max(np.abs(Aa.conj().T @ np.concatenate([b, d])))
