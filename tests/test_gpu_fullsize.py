"""Parity at full size, on outputs the oracle can compute one by one:
the two-sphere workload (N = 5124 nodes, level-4 icospheres, k_m = 12 m / 512)
in every float32 form of the factorisation, the 3M form being the one
bench.py times (sampled wavenumbers, sampled observation points of the
1024^2 plane grid, the closest nodes of a 256^2 sub-grid, bit-exact), and
the uneven batch's largest body (10242 nodes) factored together with a 642-
and a 2562-node body."""
import json
import os

import numpy as np
import pytest

from oracle import bie, field as ofield
from oracle.mesh import Surface
from workloads import two_spheres_workload, plane_grid, uneven_bodies_workload

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


@pytest.fixture(scope="module")
def oracle_k6(setup):
    """One oracle solve at full size (dense FP64 LAPACK) at k = 6."""
    ctx, w, ds, s = setup
    k = w.k[255]
    p, dp = bie.incident_plane_wave(s, k)
    _, _, xs = bie.solve(s, k, bie.known_data(s, p, dp))
    return xs


@pytest.mark.parametrize("mode", ["3m", "4m", "b3"])
def test_fullsize_solve_sampled_vs_oracle(setup, oracle_k6, mode):
    ctx, w, ds, s = setup
    idx = [0, 255, 511]                     # k = 0.0234, 6.0, 12.0
    k = w.k[idx]
    kd = torch.as_tensor(k).cuda()
    n = ds.n
    y = torch.empty((3, 1, n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, 3, kd, (0.0, 0.0, 1.0), y)
    x = torch.zeros((3, 1, n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    opts.mode = {"3m": native.BEM_FP32_IR_3M, "4m": native.BEM_FP32_IR_4M,
                 "b3": native.BEM_FP32_IR_B3}[mode]
    info = native.bem_solve_batched(ctx, [(ds.struct, 3, kd, 1, y)], opts, [x])
    for q in range(3):
        assert 0 < info[q].rel_resid < 1e-9 and info[q].converged == 1
    xs = oracle_k6
    err = np.linalg.norm(x[1, 0].cpu().numpy() - xs) / np.linalg.norm(xs)
    assert err < 1e-6, err
    if mode != "3m":
        return
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
    # point by point, against max(|U|, RMS of U over the points) per frequency:
    # each point's float32 sum runs over 5124 nodes in 16 partial sums (642 in
    # the 2e-6 tests of test_gpu_field.py), and at k = 0.023 the scattered field
    # is 1e-3 of the incident wave while the summed terms are of the surface
    # data's size, so the bound is 5e-6 (a float32 model of the sum gives
    # 4.7e-6 at the worst point when the node sums are float32 as well; they
    # are float64 here)
    out = ins.cpu().numpy() == 0
    scale = np.sqrt(np.mean(np.abs(ref[out]) ** 2, axis=0, keepdims=True))
    assert np.max(np.abs(got[out] - ref[out]) / np.maximum(np.abs(ref[out]), scale)) < 5e-6


def test_uneven_batch_with_level5_body_vs_oracle():
    """The seeded uneven batch's first level-5 body (a prolate spheroid, 10242
    nodes, sound-soft) factored in one batched call with a 642- and a
    2562-node body, two wavenumbers each, in the 3M form.  The large body is
    compared with stored entries of the oracle's FP64 solution
    (tests/golden/make_uneven_level5_samples.py); the two small ones with the
    oracle directly."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "uneven_level5_samples.json")))
    w = uneven_bodies_workload(n_k=1024)
    ctx = native.Context(0)
    try:
        picks = [(w.bodies[0], np.array([w.k[40], w.k[900]])),
                 (w.bodies[1], np.array([w.k[300], w.k[700]])),
                 (w.bodies[gold["body_index"]], np.array(gold["k"]))]
        probs, outs, keep = [], [], []
        for body, k in picks:
            ds = DeviceSurface.from_bodies([body])
            kd = torch.as_tensor(k).cuda()
            y = torch.empty((2, 1, ds.n), dtype=torch.complex128, device="cuda")
            native.bem_incident(ctx, ds.struct, 2, kd, (0.0, 0.0, 1.0), y)
            x = torch.zeros_like(y)
            probs.append((ds.struct, 2, kd, 1, y))
            outs.append(x)
            keep.append((ds, kd, y))
        assert [d.n for d, _, _ in keep] == [642, 2562, 10242]
        opts = native.bem_solve_opts_default()
        opts.mode = native.BEM_FP32_IR_3M
        info = native.bem_solve_batched(ctx, probs, opts, outs)
        assert all(info[q].converged == 1 and 0 < info[q].rel_resid < 1e-9 for q in range(6))
        for (body, k), x in list(zip(picks, outs))[:2]:
            s = Surface([body])
            for j, kq in enumerate(k):
                p, dp = bie.incident_plane_wave(s, kq)
                _, _, xs = bie.solve(s, kq, bie.known_data(s, p, dp))
                assert np.linalg.norm(x[j, 0].cpu().numpy() - xs) / np.linalg.norm(xs) < 1e-6
        idx = np.array(gold["sample_index"])
        xl = outs[2].cpu().numpy()[:, 0]
        for j in range(2):
            ref = np.array(gold["x_re"][j]) + 1j * np.array(gold["x_im"][j])
            got = xl[j, idx]
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-6
            assert abs(np.linalg.norm(xl[j]) / gold["x_norm"][j] - 1.0) < 1e-6
    finally:
        ctx.close()


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
