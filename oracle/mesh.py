"""Oracle surface description: nodes, outward normals, nodal weights, BC flags.

Test infrastructure only (see the package docstring).

The paper discretises the scatterer surfaces with elements and collocates at the
nodes (Sec. IV A: 500 quadratic elements / 1002 nodes, and 774 linear elements /
389 nodes).  The hot path uses the nodal (linear-element, lumped) variant: each
node carries a quadrature weight equal to one third of the areas of its adjacent
flat triangles, optionally rescaled so that the weights of one body sum to its
analytic area.  Normals are the analytic outward normals of the sphere/spheroid
(pointing out of the body, into the fluid).

Every floating-point expression is written in a fixed evaluation order (left to
right, no fused multiply-add) so that an independent implementation that follows
the same order reproduces every bit.
"""
from __future__ import annotations

import math

import numpy as np

_PHI = (1.0 + math.sqrt(5.0)) / 2.0

# Icosahedron: the 12 cyclic permutations of (0, +-1, +-phi), counter-clockwise
# faces seen from outside.
_ICO_V = [(-1.0, _PHI, 0.0), (1.0, _PHI, 0.0), (-1.0, -_PHI, 0.0), (1.0, -_PHI, 0.0),
          (0.0, -1.0, _PHI), (0.0, 1.0, _PHI), (0.0, -1.0, -_PHI), (0.0, 1.0, -_PHI),
          (_PHI, 0.0, -1.0), (_PHI, 0.0, 1.0), (-_PHI, 0.0, -1.0), (-_PHI, 0.0, 1.0)]
_ICO_F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
          (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
          (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
          (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]


def _unit(v):
    s = math.sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2])
    return (v[0] / s, v[1] / s, v[2] / s)


def icosphere(level: int):
    """Unit icosphere by ``level`` midpoint subdivisions.

    Returns (verts [V,3] float64, faces [F,3] int32) with V = 10*4^L + 2 and
    F = 20*4^L.  Faces are visited in order; the midpoint of edge (a,b) is
    created on first encounter (key (min,max)) as normalise((a+b)*0.5); each
    face (a,b,c) is replaced by [a,ab,ca], [b,bc,ab], [c,ca,bc], [ab,bc,ca].
    """
    verts = [_unit(v) for v in _ICO_V]
    faces = list(_ICO_F)
    for _ in range(level):
        cache = {}
        nf = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                pa, pb = verts[a], verts[b]
                m = ((pa[0] + pb[0]) * 0.5, (pa[1] + pb[1]) * 0.5, (pa[2] + pb[2]) * 0.5)
                verts.append(_unit(m))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf.extend([(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)])
        faces = nf
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int32)


def spheroid_area(radius: float, aspect: float) -> float:
    """Analytic area of the body: sphere 4 pi R^2; prolate spheroid with
    equatorial radius a = R and polar semi-axis c = R*aspect > a:
    2 pi a^2 (1 + c/(a e) asin e), e = sqrt(1 - a^2/c^2)."""
    if aspect == 1.0:
        return 4.0 * math.pi * radius * radius
    a = radius
    c = radius * aspect
    e = math.sqrt(1.0 - (a * a) / (c * c))
    return 2.0 * math.pi * a * a * (1.0 + (c / (a * e)) * math.asin(e))


def body_surface(body, rescale_area: bool = True):
    """Nodes, normals, weights and faces of one body (see module docstring)."""
    u, faces = icosphere(body.level)
    cx, cy, cz = body.center
    sx = body.radius
    sz = body.radius * body.aspect
    V = u.shape[0]
    x = np.empty((V, 3))
    nrm = np.empty((V, 3))
    for i in range(V):
        u0, u1, u2 = float(u[i, 0]), float(u[i, 1]), float(u[i, 2])
        x[i, 0] = cx + sx * u0
        x[i, 1] = cy + sx * u1
        x[i, 2] = cz + sz * u2
        g = (u0 / sx, u1 / sx, u2 / sz)
        nrm[i] = _unit(g)
    w = [0.0] * V
    total = 0.0
    for (a, b, c) in faces:
        pa, pb, pc = x[a], x[b], x[c]
        e1 = (float(pb[0] - pa[0]), float(pb[1] - pa[1]), float(pb[2] - pa[2]))
        e2 = (float(pc[0] - pa[0]), float(pc[1] - pa[1]), float(pc[2] - pa[2]))
        c0 = e1[1] * e2[2] - e1[2] * e2[1]
        c1 = e1[2] * e2[0] - e1[0] * e2[2]
        c2 = e1[0] * e2[1] - e1[1] * e2[0]
        area = 0.5 * math.sqrt((c0 * c0 + c1 * c1) + c2 * c2)
        total = total + area
        third = area / 3.0
        w[a] = w[a] + third
        w[b] = w[b] + third
        w[c] = w[c] + third
    w = np.array(w, dtype=np.float64)
    if rescale_area:
        factor = spheroid_area(body.radius, body.aspect) / total
        w = w * factor
    return x, nrm, w, faces


class Surface:
    """Concatenated surface of several bodies (body order, then node order)."""

    def __init__(self, bodies, rescale_area: bool = True):
        xs, ns, ws, bcs, fs, ids = [], [], [], [], [], []
        off = 0
        for b_i, body in enumerate(bodies):
            x, n, w, f = body_surface(body, rescale_area)
            xs.append(x); ns.append(n); ws.append(w)
            bcs.append(np.full(x.shape[0], body.bc, dtype=np.uint8))
            ids.append(np.full(x.shape[0], b_i, dtype=np.int32))
            fs.append(f + off)
            off += x.shape[0]
        self.bodies = list(bodies)
        self.x = np.concatenate(xs)
        self.nrm = np.concatenate(ns)
        self.w = np.concatenate(ws)
        self.bc = np.concatenate(bcs)
        self.body = np.concatenate(ids)
        self.faces = np.concatenate(fs)

    @property
    def n(self) -> int:
        return self.x.shape[0]


# ---------------------------------------------------------------- acoustic bowl
def bowl_counts(n_theta: int, n_phi: int):
    """(nodes, faces) of the bowl mesh: two poles and n_theta - 1 rings."""
    return 2 + (n_theta - 1) * n_phi, 2 * n_phi * (n_theta - 1)


def bowl(n_theta: int, n_phi: int, radius: float = 1.0, tilt: float = 0.0,
         center=(0.0, 0.0, 0.0)):
    """The axisymmetric bowl of Sec. IV C (Eq. dish): the closed meridian curve
    xi = a sin(theta), eta = a (0.2 cos(theta) - 0.6 sin^2(theta)),
    0 <= theta <= pi, rotated about the eta axis; a thin curved shell whose
    two faces meet at a sharp rim (xi = a, eta = -0.6 a).

    Nodes: the pole theta = 0, rings theta_i = pi i / n_theta (i = 1 ..
    n_theta - 1) of n_phi nodes at phi_j = 2 pi j / n_phi, the pole theta = pi.
    Local frame (xi cos phi, xi sin phi, eta); the eta axis is then turned by
    `tilt` about x (y' = y cos t - z sin t, z' = y sin t + z cos t) and shifted
    by `center`.  Normals are analytic: in the meridian plane the outward
    normal of the curve is (-eta', xi') / |(xi', eta')|.  Weights: one third of
    the adjacent flat-triangle areas (no rescaling).

    Returns (x [V,3], nrm [V,3], w [V], faces [F,3] int32)."""
    assert n_theta >= 2 and n_phi >= 3
    V, F = bowl_counts(n_theta, n_phi)
    ct, st = math.cos(tilt), math.sin(tilt)
    cx, cy, cz = center
    loc = []      # local (x, y, z) and normal
    # top pole
    loc.append(((0.0, 0.0, radius * (0.2 * math.cos(0.0))), (0.0, 0.0, 1.0)))
    for i in range(1, n_theta):
        th = (math.pi * i) / n_theta
        s, c = math.sin(th), math.cos(th)
        xi = radius * s
        eta = radius * (0.2 * c - 0.6 * (s * s))
        dxi = c
        deta = -0.2 * s - 1.2 * (s * c)
        m = math.sqrt(dxi * dxi + deta * deta)
        nxi, neta = -deta / m, dxi / m
        for j in range(n_phi):
            ph = (2.0 * math.pi * j) / n_phi
            cp, sp = math.cos(ph), math.sin(ph)
            loc.append(((xi * cp, xi * sp, eta), (nxi * cp, nxi * sp, neta)))
    # bottom pole
    loc.append(((0.0, 0.0, radius * (0.2 * math.cos(math.pi))), (0.0, 0.0, -1.0)))
    x = np.empty((V, 3))
    nrm = np.empty((V, 3))
    for k, ((px, py, pz), (qx, qy, qz)) in enumerate(loc):
        x[k, 0] = cx + px
        x[k, 1] = cy + (py * ct - pz * st)
        x[k, 2] = cz + (py * st + pz * ct)
        nrm[k, 0] = qx
        nrm[k, 1] = qy * ct - qz * st
        nrm[k, 2] = qy * st + qz * ct
    faces = []
    for j in range(n_phi):
        faces.append((0, 1 + j, 1 + (j + 1) % n_phi))
    for i in range(1, n_theta - 1):
        r0 = 1 + (i - 1) * n_phi
        r1 = r0 + n_phi
        for j in range(n_phi):
            j1 = (j + 1) % n_phi
            faces.append((r0 + j, r1 + j, r1 + j1))
            faces.append((r0 + j, r1 + j1, r0 + j1))
    rl = 1 + (n_theta - 2) * n_phi
    for j in range(n_phi):
        faces.append((V - 1, rl + (j + 1) % n_phi, rl + j))
    w = [0.0] * V
    for (a, b, c) in faces:
        pa, pb, pc = x[a], x[b], x[c]
        e1 = (float(pb[0] - pa[0]), float(pb[1] - pa[1]), float(pb[2] - pa[2]))
        e2 = (float(pc[0] - pa[0]), float(pc[1] - pa[1]), float(pc[2] - pa[2]))
        c0 = e1[1] * e2[2] - e1[2] * e2[1]
        c1 = e1[2] * e2[0] - e1[0] * e2[2]
        c2 = e1[0] * e2[1] - e1[1] * e2[0]
        third = (0.5 * math.sqrt((c0 * c0 + c1 * c1) + c2 * c2)) / 3.0
        w[a] = w[a] + third
        w[b] = w[b] + third
        w[c] = w[c] + third
    return x, nrm, np.array(w, dtype=np.float64), np.array(faces, dtype=np.int32)


class ArraySurface:
    """A surface given by its arrays (nodes, normals, weights, BC flags)."""

    def __init__(self, x, nrm, w, bc):
        self.x, self.nrm, self.w = x, nrm, w
        self.bc = np.asarray(bc, dtype=np.uint8)

    @property
    def n(self) -> int:
        return self.x.shape[0]
