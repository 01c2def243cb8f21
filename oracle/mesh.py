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
