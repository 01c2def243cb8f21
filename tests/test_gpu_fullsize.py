"""Parity at the full size of the two-sphere workload (N = 5124 nodes, level-4
icospheres, k_m = 12 m / 512), in the launch configuration bench.py times, on
outputs the oracle can compute one by one: sampled wavenumbers, sampled
observation points of the 1024^2 plane grid, and the closest nodes of a
256^2 sub-grid (bit-exact)."""
import numpy as np
import pytest

from oracle import bie, field as ofield
from oracle.mesh import Surface
from workloads import two_spheres_workload, plane_grid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_1706_07919_amd.native")
from paper_1706_07919_amd import DeviceSurface  # noqa: E402


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available()
    ctx = native.Context(0)
    w = two_spheres_workload(512)
    ds = DeviceSurface.from_bodies(w.bodies)
    s = Surface(w.bodies)
    yield ctx, w, ds, s
    ctx.close()


def test_fullsize_solve_sampled_vs_oracle(setup):
    ctx, w, ds, s = setup
    idx = [0, 255, 511]                     # k = 0.0234, 6.0, 12.0
    k = w.k[idx]
    kd = torch.as_tensor(k).cuda()
    n = ds.n
    y = torch.empty((3, 1, n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, 3, kd, (0.0, 0.0, 1.0), y)
    x = torch.zeros((3, 1, n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    info = native.bem_solve_batched(ctx, [(ds.struct, 3, kd, 1, y)], opts, [x])
    for q in range(3):
        assert info[q].rel_resid < 1e-9 and info[q].converged == 1
    q = 1   # one oracle solve at full size (dense FP64 LAPACK)
    p, dp = bie.incident_plane_wave(s, k[q])
    _, _, xs = bie.solve(s, k[q], bie.known_data(s, p, dp))
    err = np.linalg.norm(x[q, 0].cpu().numpy() - xs) / np.linalg.norm(xs)
    assert err < 1e-6, err
    # sampled field points of the 1024^2 plane, all three frequencies, c64 kernel
    phi = torch.empty_like(x)
    psi = torch.empty_like(x)
    native.bem_split_unknowns(ctx, ds.struct, 3, 1, x, y, phi, psi)
    grid = plane_grid(1024)
    rng = np.random.default_rng(0)
    pts = grid[rng.choice(grid.shape[0], 96, replace=False)]
    m = pts.shape[0]
    U = torch.zeros((1, m, 3), dtype=torch.complex64, device="cuda")
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    native.bem_field_eval(ctx, ds.struct, 3, kd, 1, phi, psi, m, torch.as_tensor(pts).cuda(), i0,
                          0, ins, native.BEM_C64, U)
    ph = phi.cpu().numpy()
    ps = psi.cpu().numpy()
    ref = np.stack([ofield.field(s, k[j], ph[j, 0], ps[j, 0], pts)[0] for j in range(3)], axis=1)
    got = U.cpu().numpy()[0].astype(np.complex128)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5


def test_fullsize_closest_nodes_bit_exact(setup):
    ctx, w, ds, s = setup
    grid = plane_grid(256)
    m = grid.shape[0]
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    k = torch.as_tensor(np.array([1.0])).cuda()
    z = torch.zeros((1, 1, ds.n), dtype=torch.complex128, device="cuda")
    U = torch.zeros((1, m, 1), dtype=torch.complex64, device="cuda")
    native.bem_field_eval(ctx, ds.struct, 1, k, 1, z, z, m, torch.as_tensor(grid).cuda(), i0, 0,
                          ins, native.BEM_C64, U)
    ref = ofield.closest_node(s.x, grid)
    assert np.array_equal(i0.cpu().numpy(), ref)
    assert np.array_equal(ins.cpu().numpy(), ofield.inside_mask(s.x, s.nrm, grid, ref))
