"""Pins of the oracle surface description (mesh counts, topology, geometry)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import mesh
from oracle.mesh import Surface, icosphere, spheroid_area
from workloads import Body, HARD, SOFT

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosphere_counts_and_topology(level):
    v, f = icosphere(level)
    assert v.shape == (10 * 4 ** level + 2, 3)
    assert f.shape == (20 * 4 ** level, 3)
    edges = {}
    for a, b, c in f:
        for e in ((a, b), (b, c), (c, a)):
            key = (min(e), max(e))
            edges[key] = edges.get(key, 0) + 1
    assert all(cnt == 2 for cnt in edges.values())          # closed 2-manifold
    assert v.shape[0] - len(edges) + f.shape[0] == 2        # Euler characteristic
    assert np.max(np.abs(np.linalg.norm(v, axis=1) - 1.0)) < 2e-16 * 4
    # counter-clockwise seen from outside: face normal along the position
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    assert np.all(np.sum(np.cross(b - a, c - a) * (a + b + c), axis=1) > 0)


def test_paper_mesh_counts_are_closed_triangulations():
    # The paper's meshes obey the same closed-surface relation V = F/2 + 2 as the
    # icospheres (linear) and V + E nodes for quadratic elements.
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    F = g["linear_mesh"]["elements"]
    assert F // 2 + 2 == g["linear_mesh"]["nodes"]
    Fq = g["quadratic_mesh"]["elements"]
    assert (Fq // 2 + 2) + 3 * Fq // 2 == g["quadratic_mesh"]["nodes"]


def test_sphere_weights_normals_and_area():
    s = Surface([Body((0.0, 0.0, 0.0), 1.0, 1.0, 3, HARD)], rescale_area=False)
    assert np.allclose(np.linalg.norm(s.nrm, axis=1), 1.0, atol=1e-15)
    assert np.allclose(s.nrm, s.x, atol=1e-15)               # sphere: n = x/|x|
    assert 0.98 * 4 * math.pi < s.w.sum() < 4 * math.pi       # inscribed polyhedron
    r = Surface([Body((0.0, 0.0, 0.0), 1.0, 1.0, 3, HARD)], rescale_area=True)
    assert abs(r.w.sum() - 4 * math.pi) < 1e-12
    assert np.all(r.w > 0)


def test_spheroid_area_and_normals():
    # prolate spheroid area: closed form vs numerical surface of revolution
    a, asp = 0.7, 2.5
    c = a * asp
    t = np.linspace(0, np.pi, 200001)
    rho = a * np.sin(t)
    dz = -c * np.sin(t)
    drho = a * np.cos(t)
    integrand = 2 * np.pi * rho * np.sqrt(drho ** 2 + dz ** 2)
    num = np.trapezoid(integrand, t)
    assert abs(spheroid_area(a, asp) - num) / num < 1e-8
    s = Surface([Body((0.3, -0.2, 1.0), a, asp, 2, SOFT)])
    u = (s.x - np.array([0.3, -0.2, 1.0])) / np.array([a, a, c])
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-14)   # nodes on the surface
    grad = u / np.array([a, a, c])
    grad /= np.linalg.norm(grad, axis=1)[:, None]
    assert np.allclose(grad, s.nrm, atol=1e-14)
    assert abs(s.w.sum() - spheroid_area(a, asp)) < 1e-12
    assert np.all(s.bc == SOFT)


def test_multibody_concatenation():
    bodies = [Body((0, 0, -2.0), 1.0, 1.0, 1, HARD), Body((0, 0, 2.0), 0.5, 1.0, 2, SOFT)]
    s = Surface(bodies)
    assert s.n == 42 + 162
    assert np.all(s.bc[:42] == HARD) and np.all(s.bc[42:] == SOFT)
    assert np.all(s.body[:42] == 0) and np.all(s.body[42:] == 1)


# ---------------------------------------------------------------- acoustic bowl
def test_bowl_mesh_against_closed_forms():
    """The bowl of Sec. IV C (Eq. dish).  Its volume follows in closed form from
    the thickness of the shell, 0.4 a sqrt(1 - (xi/a)^2) at radius xi:
    V = 2 pi int_0^a xi 0.4 sqrt(1 - xi^2/a^2) dxi = 0.8 pi a^3 / 3; the
    divergence theorem gives it from the mesh as (1/3) sum w_j x_j . n_j, which
    also pins the orientation of the normals.  The lumped area converges at
    O(h^2) to the surface of revolution's area (a library quadrature), and the
    flux of a constant field through the closed surface, sum w_j n_j, to 0."""
    import math
    from scipy.integrate import quad
    area = 2 * math.pi * quad(lambda t: math.sin(t) * math.hypot(
        math.cos(t), -0.2 * math.sin(t) - 1.2 * math.sin(t) * math.cos(t)), 0, math.pi,
        limit=200)[0]
    vol = 0.8 * math.pi / 3
    errs = []
    for nt, nph in [(8, 16), (16, 32), (32, 64)]:
        x, n, w, f = mesh.bowl(nt, nph, tilt=0.3, center=(0.5, -1.0, 2.0))
        assert (len(x), len(f)) == mesh.bowl_counts(nt, nph)
        assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-15)
        c = np.array([0.5, -1.0, 2.0])
        v = np.sum(w * np.sum((x - c) * n, axis=1)) / 3.0
        flux = np.linalg.norm(np.sum(w[:, None] * n, axis=0))
        errs.append(area - w.sum())
        if nt >= 16:
            assert abs(v - vol) < 0.005 * vol
            assert flux < 0.02
    assert errs[0] > 0 and 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0
