"""GPU parity of the surface-to-field step (Eq. BRIEFdmn) point by point,
through the C ABI: per-point and per-frequency error bounds at points close
to the surface (1e-4 to 1e-2 off it on node normals, 0.02 and 0.05 between
nodes) and next to the bowl's sharp rim, and several right-hand sides per
call, each compared with the oracle on its own."""
import numpy as np
import pytest

from oracle import bie, field as ofield
from oracle.mesh import ArraySurface, Surface, bowl
from workloads import Body, HARD, seeded_complex

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_1706_07919_amd.native")
from paper_1706_07919_amd import DeviceSurface  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    native.load()
    c = native.Context(0)
    yield c
    c.close()


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def field_gpu(ctx, ds, k, phi, psi, pts, prec):
    """U [n_rhs][m][n_k] for phi, psi [n_k][n_rhs][n]."""
    nk, nr = phi.shape[0], phi.shape[1]
    m = pts.shape[0]
    cdt = torch.complex128 if prec == native.BEM_C128 else torch.complex64
    U = torch.zeros((nr, m, nk), dtype=cdt, device="cuda")
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    native.bem_field_eval(ctx, ds.struct, nk, dev(k), nr, dev(phi), dev(psi), m, dev(pts), i0, 0,
                          ins, prec, U)
    return U.cpu().numpy().astype(np.complex128), i0.cpu().numpy(), ins.cpu().numpy()


def per_point_error(U, ref):
    """max over points and frequencies of |U - ref| / max(|ref|, scale_k), with
    scale_k the RMS of |ref| over the points at frequency k (so that points
    where the field nearly vanishes are judged against the field's size)."""
    scale = np.sqrt(np.mean(np.abs(ref) ** 2, axis=0, keepdims=True))
    return float(np.max(np.abs(U - ref) / np.maximum(np.abs(ref), scale)))


def above_centroids(s, body_nodes, deltas, count, rng):
    """Points `delta` outside a sphere body above the centroids of randomly
    chosen surface triangles (between nodes)."""
    out = []
    faces = s.faces
    for (lo, hi, centre, radius) in body_nodes:
        fsel = faces[(faces[:, 0] >= lo) & (faces[:, 0] < hi)]
        pick = fsel[rng.choice(len(fsel), count, replace=False)]
        cen = s.x[pick].mean(axis=1) - centre
        u = cen / np.linalg.norm(cen, axis=1, keepdims=True)
        for d in deltas:
            out.append(centre + (radius + d) * u)
    return np.concatenate(out)


@pytest.mark.parametrize("prec,tol", [(native.BEM_C64, 2e-6), (native.BEM_C128, 1e-11)])
def test_field_per_point_near_surface(ctx, prec, tol):
    """Two spheres (level 3, 642 nodes each) with the FP64 solution of the
    plane-wave problem as surface data, judged point by point and frequency by
    frequency: points 1e-4, 1e-3 and 1e-2 off the surface on node normals
    (there x0 is the node and the bracketed differences of Eq. BRIEFdmn nearly
    cancel), points 0.02 and 0.05 above triangle centroids (between nodes),
    and points far away.

    Points closer to the surface than about h^2/8 between nodes (h the mesh
    spacing, ~0.15 here) lie below the tangent plane of their closest node, so
    the inside test n_i0.(x_p - x_i0) < 0 marks them inside and their field is
    0: at 1e-4 and 1e-3 above centroids the GPU marks them exactly as the
    oracle does."""
    bodies = [Body((0.0, 0.0, -1.3), 1.0, 1.0, 3, HARD), Body((0.0, 0.0, 1.3), 1.0, 1.0, 3, HARD)]
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    k = np.array([0.5, 2.25, 4.0, 6.5, 9.0])
    rng = np.random.default_rng(3)
    nb = s.n // 2
    spheres = [(0, nb, np.array([0.0, 0.0, -1.3]), 1.0), (nb, 2 * nb, np.array([0.0, 0.0, 1.3]), 1.0)]
    nodes = rng.choice(s.n, 24, replace=False)
    on_normal = np.concatenate([s.x[nodes] + d * s.nrm[nodes] for d in (1e-4, 1e-3, 1e-2)])
    between = above_centroids(s, spheres, [2e-2, 5e-2], 12, rng)
    masked = above_centroids(s, spheres, [1e-4, 1e-3], 6, rng)
    far = rng.uniform(-4, 4, (40, 3))
    pts = np.concatenate([on_normal, between, masked, far])
    phi = np.zeros((len(k), 1, s.n), np.complex128)
    psi = np.zeros_like(phi)
    for q, kq in enumerate(k):
        ph, ps = bie.scatter_plane_wave(s, kq)
        phi[q, 0], psi[q, 0] = ph, ps
    U, i0, ins = field_gpu(ctx, ds, k, phi, psi, pts, prec)
    oi0 = ofield.closest_node(s.x, pts)
    assert np.array_equal(i0, oi0)
    oins = ofield.inside_mask(s.x, s.nrm, pts, oi0)
    assert np.array_equal(ins, oins)
    n_on, n_bt, n_ms = len(on_normal), len(between), len(masked)
    assert not ins[:n_on + n_bt].any()                   # on normals and 0.02+ between: fluid
    assert ins[n_on + n_bt:n_on + n_bt + n_ms].all()     # closer between nodes: marked inside
    assert np.all(U[0][ins == 1] == 0)
    out = ins == 0
    ref = np.stack([ofield.field(s, kq, phi[q, 0], psi[q, 0], pts, oi0)[0]
                    for q, kq in enumerate(k)], axis=1)
    err = per_point_error(U[0][out], ref[out])
    assert err < tol, err


def test_field_per_point_next_to_bowl_rim(ctx):
    """The bowl of Eq. dish (16 x 24 rings, axis turned by 0.15 pi): points at
    0.02 to 0.1 outside its sharp rim, around the rim, judged point by point."""
    x, nrm, w, _ = native.bem_mesh_bowl(16, 24, 1.0, 0.15 * np.pi, (0.0, 0.0, 0.0))
    bc = np.zeros(len(x), dtype=np.uint8)
    s = ArraySurface(*bowl(16, 24, 1.0, 0.15 * np.pi)[:3], bc)
    ds = DeviceSurface(x, nrm, w, bc)
    k = np.array([0.7, 24 * np.pi / 20.1, 6.1])
    t = 0.15 * np.pi
    pts = []
    for phi_r in np.linspace(0.0, 2 * np.pi, 9)[:-1] + 0.1:
        for d in (0.02, 0.05, 0.1):
            xi, eta = 1.0 + d, -0.6
            q = np.array([xi * np.cos(phi_r), xi * np.sin(phi_r), eta])
            pts.append([q[0], q[1] * np.cos(t) - q[2] * np.sin(t), q[1] * np.sin(t) + q[2] * np.cos(t)])
    pts = np.array(pts)
    phi = np.zeros((len(k), 1, s.n), np.complex128)
    psi = np.zeros_like(phi)
    for q, kq in enumerate(k):
        p, dp = bie.incident_plane_wave(s, kq)
        ph, ps, _ = bie.solve(s, kq, bie.known_data(s, p, dp))
        phi[q, 0], psi[q, 0] = ph, ps
    U, i0, ins = field_gpu(ctx, ds, k, phi, psi, pts, native.BEM_C64)
    oi0 = ofield.closest_node(s.x, pts)
    assert np.array_equal(i0, oi0)
    out = ins == 0
    ref = np.stack([ofield.field(s, kq, phi[q, 0], psi[q, 0], pts, oi0)[0]
                    for q, kq in enumerate(k)], axis=1)
    err = per_point_error(U[0][out], ref[out])
    assert err < 2e-6, err


@pytest.mark.parametrize("n_rhs", [2, 5])
@pytest.mark.parametrize("prec", [native.BEM_C64, native.BEM_C128])
def test_field_several_rhs_each_vs_oracle(ctx, n_rhs, prec):
    """n_rhs surface data sets per frequency in one call (evenly spaced k with a
    ragged last chunk, plus scattered k): each right-hand side's field equals
    the oracle's for that data alone."""
    bodies = [Body((0.0, 0.0, -1.2), 1.0, 1.0, 2, HARD), Body((0.2, 0.0, 1.3), 0.8, 1.5, 2, HARD)]
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    k = np.concatenate([0.7 * np.arange(1, 12), [3.3, 10.9]])
    rng = np.random.default_rng(10 + n_rhs)
    phi = seeded_complex(rng, (len(k), n_rhs, s.n))
    psi = seeded_complex(rng, (len(k), n_rhs, s.n))
    pts = np.concatenate([rng.uniform(-4, 4, (150, 3)), s.x[[5, 77]] * 1.0])
    U, i0, ins = field_gpu(ctx, ds, k, phi, psi, pts, prec)
    oi0 = ofield.closest_node(s.x, pts)
    assert np.array_equal(i0, oi0)
    out = ins == 0
    tol = 2e-6 if prec == native.BEM_C64 else 1e-11
    for r in range(n_rhs):
        ref = np.stack([ofield.field(s, kq, phi[q, r], psi[q, r], pts, oi0)[0]
                        for q, kq in enumerate(k)], axis=1)
        assert np.all(U[r][~out] == 0)
        err = per_point_error(U[r][out], ref[out])
        assert err < tol, (r, err)
