"""Pins of the quadratic-element oracle (Sec. III: quadratic interpolation and
Gauss quadrature of non-singular integrands; Sec. IV A: 500 elements, 1002
nodes, results correct to better than 2 significant figures against the
series solution and the linear-element mesh)."""
import math

import numpy as np
import pytest

from oracle import bie, field as ofield, quadratic as Q, series
from oracle.mesh import Surface
from workloads import Body, HARD, SOFT


def test_geodesic_counts_topology_and_paper_sizes():
    for nu in (1, 2, 3, 5):
        u, faces = Q.geodesic(nu)
        V, F = u.shape[0], faces.shape[0]
        assert V == 10 * nu * nu + 2 and F == 20 * nu * nu
        edges = {}
        for f in faces:
            for a, b in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0])):
                edges[(min(a, b), max(a, b))] = edges.get((min(a, b), max(a, b)), 0) + 1
        assert all(c == 2 for c in edges.values())          # closed, manifold
        assert V - len(edges) + F == 2                      # Euler characteristic
        assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-15)
        # every face counter-clockwise seen from outside
        c = np.cross(u[faces[:, 1]] - u[faces[:, 0]], u[faces[:, 2]] - u[faces[:, 0]])
        assert np.all(np.sum(c * u[faces].mean(axis=1), axis=1) > 0)
    qs = Q.QuadSurface(Body((0.0, 0.0, 0.0), 1.0, 1.0, 0, HARD), 5)
    assert (qs.n, len(qs.elems)) == (1002, 500) == Q.quadratic_counts(5)
    # midpoints: on the sphere, on the bisector of their edge
    for e in qs.elems[:50]:
        for (a, b, m) in ((e[0], e[1], e[3]), (e[1], e[2], e[4]), (e[2], e[0], e[5])):
            assert abs(np.linalg.norm(qs.x[m]) - 1.0) < 1e-15
            assert abs(np.linalg.norm(qs.x[m] - qs.x[a]) - np.linalg.norm(qs.x[m] - qs.x[b])) < 1e-14


def test_rule7_degree_five_exactly():
    xi, eta, w = Q.rule7()
    assert abs(w.sum() - 0.5) < 1e-16
    for a in range(7):
        for b in range(7 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * xi ** a * eta ** b)
            if a + b <= 5:
                assert abs(got - exact) < 1e-15, (a, b)
    # and not degree 6: some sixth-degree monomial is missed
    assert max(abs(np.sum(w * xi ** a * eta ** (6 - a)) - math.factorial(a) * math.factorial(6 - a)
                   / math.factorial(8)) for a in range(7)) > 1e-6


def test_shape_functions_interpolate_and_sum_to_one():
    nodes = np.array([[0, 0], [1, 0], [0, 1], [0.5, 0], [0.5, 0.5], [0, 0.5]], dtype=float)
    N, dxi, deta = Q.shape(nodes[:, 0], nodes[:, 1])
    assert np.allclose(N, np.eye(6), atol=1e-15)            # N_a(node b) = delta_ab
    rng = np.random.default_rng(0)
    p = rng.uniform(0, 0.5, (20, 2))
    N, dxi, deta = Q.shape(p[:, 0], p[:, 1])
    assert np.allclose(N.sum(axis=1), 1.0) and np.allclose(dxi.sum(axis=1), 0.0, atol=1e-14)
    assert np.allclose(deta.sum(axis=1), 0.0, atol=1e-14)
    # derivatives against central differences
    h = 1e-6
    Np, _, _ = Q.shape(p[:, 0] + h, p[:, 1])
    Nm, _, _ = Q.shape(p[:, 0] - h, p[:, 1])
    assert np.allclose((Np - Nm) / (2 * h), dxi, atol=1e-8)
    Np, _, _ = Q.shape(p[:, 0], p[:, 1] + h)
    Nm, _, _ = Q.shape(p[:, 0], p[:, 1] - h)
    assert np.allclose((Np - Nm) / (2 * h), deta, atol=1e-8)


def test_element_quadrature_area_convergence_and_gauss_law():
    """The isoparametric surface's area converges to 4 pi R^2 at fourth order,
    and Gauss's law int dG0/dn dS = -4 pi for a source inside (k = 0) holds on
    the quadrature (normals out of the body)."""
    errs = []
    for nu in (3, 6):
        qs = Q.QuadSurface(Body((0.0, 0.0, 0.0), 1.3, 1.0, 0, HARD), nu)
        xq, nq, wJ, _ = Q.element_quadrature(qs)
        errs.append(abs(wJ.sum() / (4 * np.pi * 1.3 ** 2) - 1.0))
        src = np.array([0.2, -0.1, 0.3])
        d = xq.reshape(-1, 3) - src
        r = np.linalg.norm(d, axis=1)
        flux = np.sum(-(np.sum(d * nq.reshape(-1, 3), axis=1)) / r ** 3 * wJ.reshape(-1))
        assert abs(flux / (-4 * np.pi) - 1.0) < (1e-4 if nu == 6 else 1e-3)
    assert errs[1] < errs[0] / 10


@pytest.mark.parametrize("bc,kind", [(HARD, "hard"), (SOFT, "soft")])
def test_sphere_series_two_significant_figures_and_linear_agreement(bc, kind):
    """Sec. IV A: the 1002-node quadratic solution, the linear-element solution
    and the series agree to better than 2 significant figures (here: the
    scattered field at the probe points of Table 1 and two more)."""
    body = Body((0.0, 0.0, 0.0), 1.0, 1.0, 3, bc)
    qs = Q.QuadSurface(body, 5)
    lin = Surface([body])
    pts = np.array([[0.0, 0.0, -1.1], [0.0, 0.0, -4.0], [2.0, 0.5, 0.3], [0.0, 1.5, 1.5]])
    for k in (1.0, 2.5):
        phi, psi = Q.scatter_plane_wave(qs, k)
        Pq = Q.field(qs, k, phi, psi, pts)[0]
        Ps = series.scattered(k, 1.0, kind, pts)
        ph_l, ps_l = bie.scatter_plane_wave(lin, k)
        Pl = ofield.field(lin, k, ph_l, ps_l, pts)[0]
        scale = np.max(np.abs(Ps))
        assert np.max(np.abs(Pq - Ps)) / scale < 1e-3        # quadratic vs series
        assert np.max(np.abs(Pq - Pl)) / scale < 1e-2        # quadratic vs linear
        # surface values against the series as well
        ph_s, ps_s = series.surface(k, 1.0, kind, qs.x)
        got, ref = (phi, ph_s) if bc == HARD else (psi, ps_s)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 5e-3     # dP/dn (soft) 2.2e-3 at k = 2.5


def test_convergence_with_mesh_frequency_and_monopole():
    """A monopole e^{ik|x-s|}/|x-s| with s inside is an exact radiating
    solution: its surface data satisfy the discrete equation up to the
    discretisation error, which falls fast with the element size; the sphere
    series error falls with it."""
    k = 2.0
    s = np.array([0.1, -0.2, 0.15])
    res, errs = [], []
    for nu in (2, 4):
        qs = Q.QuadSurface(Body((0.0, 0.0, 0.0), 1.0, 1.0, 0, HARD), nu)
        d = qs.x - s
        r = np.linalg.norm(d, axis=1)
        phi = np.exp(1j * k * r) / r
        psi = phi * (1j * k * r - 1.0) * np.sum(d * qs.nrm, axis=1) / (r * r)
        Mphi, Mpsi = Q.operator_matrices(qs, k)
        R = Mphi @ phi + Mpsi @ psi
        res.append(np.linalg.norm(R) / np.linalg.norm(Mphi @ phi))
        ph, ps = Q.scatter_plane_wave(qs, k)
        ph_s, _ = series.surface(k, 1.0, "hard", qs.x)
        errs.append(np.linalg.norm(ph - ph_s) / np.linalg.norm(ph_s))
    assert res[1] < res[0] / 8 and errs[1] < errs[0] / 8, (res, errs)


def test_field_on_a_node_is_the_nodal_value_and_inside_is_zero():
    qs = Q.QuadSurface(Body((0.0, 0.0, 0.0), 1.0, 1.0, 0, SOFT), 3)
    phi, psi = Q.scatter_plane_wave(qs, 1.7)
    pts = np.concatenate([qs.x[[4, 100]], [[0.0, 0.0, 0.2]]])
    P, i0, ins = Q.field(qs, 1.7, phi, psi, pts)
    assert list(i0[:2]) == [4, 100] and list(ins) == [0, 0, 1]
    assert P[0] == phi[4] and P[1] == phi[100] and P[2] == 0
