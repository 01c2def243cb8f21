"""Oracle of the quadratic-element discretisation of the non-singular boundary
integral equation (Sec. III: quadratic interpolants within each element, and
integrals free of singularities evaluated by standard Gauss quadrature;
Sec. IV A: the sphere represented by 500 quadratic elements and 1002 nodes).

Test infrastructure only (see the package docstring).

Mesh.  A frequency-nu geodesic subdivision of the icosahedron: every face is
cut into nu^2 triangles on its barycentric grid and the grid points are
projected onto the unit sphere (nu = 5: 20 * 25 = 500 triangles, 252
vertices).  Each triangle becomes a six-node element: its three vertices and
the three edge midpoints (midpoint of the chord, projected onto the sphere);
nu = 5 gives 252 + 750 = 1002 nodes, the paper's count.  The unit points map
to the body as center + (R u0, R u1, R aspect u2); node normals are the
analytic outward normals (as for the nodal surfaces).

Interpolation.  On the reference triangle (xi, eta), with L0 = 1 - xi - eta,
L1 = xi, L2 = eta, the six shape functions are L_a (2 L_a - 1) at the vertices
and 4 L_a L_b at the midpoints; geometry and surface data are interpolated
with them (isoparametric elements), x(xi, eta) = sum_a N_a x_a, and the
element's normal at a quadrature point is the normalised cross product of its
two tangents.

Quadrature.  The symmetric 7-point rule of degree 5 on triangles (Radon 1948):
the centroid with weight 9/40 and the points (a, a, 1 - 2a) for
a = (6 -+ sqrt 15)/21 with weights (155 -+ sqrt 15)/1200 (fractions of the
triangle's area).

Discrete equation at collocation node i (normals out of the body), the
integrals of Eq. BRIEF over the elements:

    4 pi phi_i + int [psi - phi_i g' - psi_i f'] G dS = int [phi - phi_i g - psi_i f] H dS

with G, H, f, g, f', g' as in oracle.bie (f, g of Appendix A about x_i with
normal n_i, H = dG/dn at the quadrature point with the element's normal), and
phi, psi interpolated from the nodal values.  The integrands are regular at
x_i (the brackets vanish there), so every element, including those that touch
x_i, takes the same rule.  Collecting terms, M_phi phi + M_psi psi = 0 with

    (M_psi)_ij = sum_{e,q} N_a(q) G_q wJ_q            (node j = node a of element e)
    (M_phi)_ij = -sum_{e,q} N_a(q) H_q wJ_q
    (M_phi)_ii += 4 pi - sum_{e,q} (g'_q G_q - g_q H_q) wJ_q
    (M_psi)_ii += -sum_{e,q} (f'_q G_q - f_q H_q) wJ_q

(wJ_q = rule weight x reference area 1/2 x |dx/dxi x dx/deta|).  Boundary
conditions and the system A x = -B y are those of oracle.bie.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.sparse

from .bie import FOUR_PI, HARD
from .field import closest_node, inside_mask
from .mesh import _ICO_F, _ICO_V, _unit


# ---------------------------------------------------------------- mesh
def geodesic(nu: int):
    """Unit frequency-nu geodesic sphere: (verts [V,3], faces [F,3] int32),
    V = 10 nu^2 + 2, F = 20 nu^2.

    Points are created on first encounter, faces of the icosahedron in order,
    grid points (i, j) of face (A, B, C) in row order (i outer, j inner).  A
    grid point has the integer barycentric weights (nu - i - j, i, j) on
    (A, B, C); it is identified across faces by its nonzero (vertex, weight)
    pairs, and its position is normalise(sum c_v V_v) with the sum taken in
    increasing vertex index."""
    ico = [_unit(v) for v in _ICO_V]
    verts, index = [], {}

    def point(a, b, c, i, j):
        key = tuple(sorted((v, w) for v, w in ((a, nu - i - j), (b, i), (c, j)) if w > 0))
        idx = index.get(key)
        if idx is None:
            s = [0.0, 0.0, 0.0]
            for v, w in key:
                for d in range(3):
                    s[d] = s[d] + float(w) * ico[v][d]
            verts.append(_unit(s))
            idx = len(verts) - 1
            index[key] = idx
        return idx

    faces = []
    for (a, b, c) in _ICO_F:
        grid = {}
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                grid[(i, j)] = point(a, b, c, i, j)
        for i in range(nu):
            for j in range(nu - i):
                faces.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j < nu - 1:
                    faces.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int32)


def quadratic_counts(nu: int):
    """(nodes, elements) of the quadratic geodesic sphere."""
    return 10 * nu * nu + 2 + 30 * nu * nu, 20 * nu * nu


class QuadSurface:
    """Six-node elements on one body (sphere or prolate spheroid).

    x, nrm [N,3] (nodes: the geodesic vertices, then the edge midpoints in the
    order met walking the elements' edges (v0 v1), (v1 v2), (v2 v0)), bc [N],
    elems [F,6] = (v0, v1, v2, m01, m12, m20)."""

    def __init__(self, body, nu: int):
        u, faces = geodesic(nu)
        pts = [tuple(p) for p in u]
        mids = {}
        elems = []
        for (a, b, c) in faces:
            m = []
            for (p, q) in ((a, b), (b, c), (c, a)):
                key = (p, q) if p < q else (q, p)
                idx = mids.get(key)
                if idx is None:
                    pa, pb = pts[p], pts[q]
                    pts.append(_unit(((pa[0] + pb[0]) * 0.5, (pa[1] + pb[1]) * 0.5,
                                      (pa[2] + pb[2]) * 0.5)))
                    idx = len(pts) - 1
                    mids[key] = idx
                m.append(idx)
            elems.append((a, b, c, m[0], m[1], m[2]))
        cx, cy, cz = body.center
        sx, sz = body.radius, body.radius * body.aspect
        N = len(pts)
        self.x = np.empty((N, 3))
        self.nrm = np.empty((N, 3))
        for i, (u0, u1, u2) in enumerate(pts):
            self.x[i] = (cx + sx * u0, cy + sx * u1, cz + sz * u2)
            self.nrm[i] = _unit((u0 / sx, u1 / sx, u2 / sz))
        self.elems = np.array(elems, dtype=np.int32)
        self.bc = np.full(N, body.bc, dtype=np.uint8)
        self.body = body
        self.nu = nu

    @property
    def n(self) -> int:
        return self.x.shape[0]


# ---------------------------------------------------------------- quadrature
def rule7():
    """(xi [7], eta [7], weight [7]) of the degree-5 rule, weights summing to
    the reference triangle's area 1/2."""
    s = math.sqrt(15.0)
    a1, a2 = (6.0 - s) / 21.0, (6.0 + s) / 21.0
    w1, w2 = (155.0 - s) / 1200.0, (155.0 + s) / 1200.0
    bary = [(1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0)]
    wts = [9.0 / 40.0]
    for a, w in ((a1, w1), (a2, w2)):
        b = 1.0 - 2.0 * a
        bary += [(b, a, a), (a, b, a), (a, a, b)]
        wts += [w, w, w]
    bary = np.array(bary)
    return bary[:, 1], bary[:, 2], 0.5 * np.array(wts)


def shape(xi, eta):
    """N [Q,6], dN/dxi [Q,6], dN/deta [Q,6] at the points (xi, eta)."""
    xi, eta = np.asarray(xi, dtype=np.float64), np.asarray(eta, dtype=np.float64)
    L0, L1, L2 = 1.0 - xi - eta, xi, eta
    N = np.stack([L0 * (2 * L0 - 1), L1 * (2 * L1 - 1), L2 * (2 * L2 - 1),
                  4 * L0 * L1, 4 * L1 * L2, 4 * L2 * L0], axis=-1)
    # d/dxi: dL0 = -1, dL1 = 1, dL2 = 0; d/deta: dL0 = -1, dL1 = 0, dL2 = 1
    dxi = np.stack([-(4 * L0 - 1), 4 * L1 - 1, 0 * L2,
                    4 * (L0 - L1), 4 * L2, -4 * L2], axis=-1)
    deta = np.stack([-(4 * L0 - 1), 0 * L1, 4 * L2 - 1,
                     -4 * L1, 4 * L1, 4 * (L0 - L2)], axis=-1)
    return N, dxi, deta


def element_quadrature(qs: QuadSurface, rule=None):
    """Quadrature points of every element: xq [F,Q,3], nq [F,Q,3] (unit
    element normals), wJ [F,Q] (weight x area Jacobian), and the shape values
    N [Q,6] of the rule."""
    xi, eta, w = rule if rule is not None else rule7()
    N, dxi, deta = shape(xi, eta)
    X = qs.x[qs.elems]                                  # [F,6,3]
    xq = np.einsum("qa,fad->fqd", N, X)
    t1 = np.einsum("qa,fad->fqd", dxi, X)
    t2 = np.einsum("qa,fad->fqd", deta, X)
    c = np.cross(t1, t2)
    J = np.linalg.norm(c, axis=-1)
    return xq, c / J[..., None], w[None, :] * J, N


def shape_matrix(qs: QuadSurface, wJ, N):
    """Sparse P [(F*Q), N_nodes] with P[(e,q), elems[e,a]] = N_a(q) wJ[e,q]:
    an integral of (interpolated data) x (kernel at the quadrature points) is
    then kernel_row @ P @ data."""
    F, Q = wJ.shape
    rows = np.repeat(np.arange(F * Q), 6)
    cols = np.broadcast_to(qs.elems[:, None, :], (F, Q, 6)).reshape(-1)
    vals = (N[None, :, :] * wJ[:, :, None]).reshape(-1)
    return scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(F * Q, qs.n))


def kernel_terms(xi, ni, k, xq, nq):
    """G, H (with the normals nq), g, f, g', f' for collocation points xi [R,3]
    with normals ni [R,3] against the quadrature points xq [P,3]: arrays [R,P]."""
    d = xq[None, :, :] - xi[:, None, :]
    r = np.sqrt(np.sum(d * d, axis=-1))
    E = np.exp(1j * k * r)
    G = E / r
    dn = np.sum(d * nq[None, :, :], axis=-1)
    H = E * (1j * k * r - 1.0) * dn / (r * r * r)
    s = k * np.sum(d * ni[:, None, :], axis=-1)
    nn = np.sum(ni[:, None, :] * nq[None, :, :], axis=-1)
    return G, H, np.cos(s), np.sin(s) / k, -k * np.sin(s) * nn, np.cos(s) * nn


def operator_matrices(qs: QuadSurface, k: float, chunk: int = 256, rule=None):
    """Dense M_phi, M_psi (N x N complex128) of the quadratic-element equation."""
    xq, nq, wJ, N = element_quadrature(qs, rule)
    P = shape_matrix(qs, wJ, N)
    xq, nq, wq = xq.reshape(-1, 3), nq.reshape(-1, 3), wJ.reshape(-1)
    n = qs.n
    Mphi = np.empty((n, n), dtype=np.complex128)
    Mpsi = np.empty((n, n), dtype=np.complex128)
    for r0 in range(0, n, chunk):
        rows = np.arange(r0, min(n, r0 + chunk))
        G, H, g, f, gp, fp = kernel_terms(qs.x[rows], qs.nrm[rows], k, xq, nq)
        Mpsi[rows] = (P.T @ G.T).T
        Mphi[rows] = -(P.T @ H.T).T
        Mphi[rows, rows] += FOUR_PI - ((gp * G - g * H) @ wq)
        Mpsi[rows, rows] += -((fp * G - f * H) @ wq)
    return Mphi, Mpsi


def system(qs: QuadSurface, k: float, y):
    """A, b of A x = -B y (the BC column selection of oracle.bie)."""
    Mphi, Mpsi = operator_matrices(qs, k)
    hard = qs.bc == HARD
    A = np.where(hard[None, :], Mphi, Mpsi)
    B = np.where(hard[None, :], Mpsi, Mphi)
    return A, -(B @ y)


def incident_plane_wave(qs: QuadSurface, k: float):
    """P_inc = exp(ikz) and dP_inc/dn = ik n_z P_inc at the nodes."""
    p = np.exp(1j * k * qs.x[:, 2])
    return p, 1j * k * qs.nrm[:, 2] * p


def solve(qs: QuadSurface, k: float, y):
    """Direct dense solve (Sec. IV A); returns (phi, psi, unknowns)."""
    A, b = system(qs, k, y)
    xs = scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), b)
    hard = qs.bc == HARD
    return np.where(hard, xs, y), np.where(hard, y, xs), xs


def scatter_plane_wave(qs: QuadSurface, k: float):
    """Surface (phi, psi) of the field scattered from exp(ikz)."""
    p, dp = incident_plane_wave(qs, k)
    y = np.where(qs.bc == HARD, -dp, -p)
    phi, psi, _ = solve(qs, k, y)
    return phi, psi


def field(qs: QuadSurface, k: float, phi, psi, xp):
    """Scattered field at points xp by Eq. BRIEFdmn with the element
    quadrature (x0 the closest node a, as for the nodal surfaces):

        4 pi P(x_p) = 4 pi phi_a + int [u (H^p - H^a) - u' (G^p - G^a)] dS,
        u = phi - phi_a g - psi_a f,  u' = psi - phi_a g' - psi_a f'

    with phi, psi interpolated at the quadrature points and f, g about x_a.
    Points inside (n_a.(x_p - x_a) < 0) give 0.  Returns (P, i0, inside)."""
    xq, nq, wJ, N = element_quadrature(qs)
    phq = np.einsum("qa,fa->fq", N, phi[qs.elems]).reshape(-1)
    psq = np.einsum("qa,fa->fq", N, psi[qs.elems]).reshape(-1)
    xq, nq, wq = xq.reshape(-1, 3), nq.reshape(-1, 3), wJ.reshape(-1)
    i0 = closest_node(qs.x, xp)
    ins = inside_mask(qs.x, qs.nrm, xp, i0)
    out = np.zeros(len(xp), dtype=np.complex128)
    for p in range(len(xp)):
        if ins[p]:
            continue
        a = i0[p]
        Ga, Ha, g, f, gp, fp = kernel_terms(qs.x[a:a + 1], qs.nrm[a:a + 1], k, xq, nq)
        Gp, Hp, _, _, _, _ = kernel_terms(xp[p:p + 1], qs.nrm[a:a + 1], k, xq, nq)
        u = phq - phi[a] * g[0] - psi[a] * f[0]
        up = psq - phi[a] * gp[0] - psi[a] * fp[0]
        s = np.sum((u * (Hp[0] - Ha[0]) - up * (Gp[0] - Ga[0])) * wq)
        out[p] = phi[a] + s / FOUR_PI
    return out, i0, ins
