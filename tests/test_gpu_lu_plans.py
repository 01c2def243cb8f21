"""Plans of the batched factorisation (the batching runtime): the GEMM tile
threshold and the persistent launch form change only which workgroup computes
which tile, so factors and pivots equal the default plan's bit for bit (also
on repeated launches, whose tile counters must start from zero, and under
hipGraph replay); the tuner tries every shape with every block width and keeps
the fastest."""
import numpy as np
import pytest

from oracle import bie
from oracle.mesh import Surface
from workloads import Body, HARD, seeded_complex

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_1706_07919_amd.native")
from paper_1706_07919_amd import DeviceSurface  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = native.Context(0)
    yield c
    c.close()


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.mark.parametrize("kind", [native.BEM_GEMM_3M, native.BEM_GEMM_4M])
def test_gemm_plans_bit_identical(ctx, kind):
    # 8 matrices of n = 1284 (ragged last tile): the first trailing updates
    # have more tiles than the resident workgroups, so the persistent form runs
    n, batch, nb = 1284, 8, 256
    rng = np.random.default_rng(11)
    M = seeded_complex(rng, (batch, n, n)) + 0.5 * np.sqrt(n) * np.eye(n)[None]
    out = []
    for narrow, persist in ((64, 0), (64, 1), (128, 0), (64, 1)):
        native.bem_lu_set_plan(ctx, native.BEM_C64, n, kind, nb, narrow, persist)
        assert native.bem_lu_tuned_plan(ctx, native.BEM_C64, n, kind) == (nb, narrow, persist)
        A = dev(M, torch.complex64)
        piv = torch.zeros((batch, n), dtype=torch.int32, device="cuda")
        info = torch.ones(batch, dtype=torch.int32, device="cuda")
        native.bem_getrf_batched(ctx, native.BEM_C64, n, n, n * n, batch, A, piv, info, 0, kind)
        out.append((A.cpu().numpy(), piv.cpu().numpy(), info.cpu().numpy()))
    a = out[0]
    assert not a[2].any()
    for b in out[1:]:
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))


def test_persistent_plan_graph_replays_match_eager(ctx):
    """A solve whose factorisation is captured and replayed with persistent
    GEMM launches returns the eager result on every replay."""
    body = Body((0.0, 0.0, 0.0), 1.0, 1.0, 3, HARD)
    s = Surface([body])
    ds = DeviceSurface.from_bodies([body])
    n = s.n
    n_k = 24
    k = np.linspace(0.3, 5.0, n_k)
    native.bem_lu_set_plan(ctx, native.BEM_C64, n, native.BEM_GEMM_3M, 128, 64, 1)
    y = np.zeros((n_k, 1, n), np.complex128)
    for q in range(n_k):
        p, dp = bie.incident_plane_wave(s, k[q])
        y[q, 0] = bie.known_data(s, p, dp)
    kd, yd = dev(k), dev(y)
    res = []
    for use_graph in (0, 1, 1, 1):
        opts = native.bem_solve_opts_default()
        opts.mode = native.BEM_FP32_IR_3M
        opts.use_graph = use_graph
        x = torch.zeros((n_k, 1, n), dtype=torch.complex128, device="cuda")
        native.bem_solve_batched(ctx, [(ds.struct, n_k, kd, 1, yd)], opts, [x])
        res.append(x.cpu().numpy())
        torch.cuda.synchronize()
    for r in res[1:]:
        assert np.array_equal(r, res[0])
    _, _, xs = bie.solve(s, k[5], y[5, 0])
    assert np.linalg.norm(res[0][5, 0] - xs) / np.linalg.norm(xs) < 1e-9


def test_autotune_tries_every_gemm_shape(ctx):
    n = 1284
    best, ms = native.bem_autotune_lu(ctx, native.BEM_C64, n, 8, native.BEM_GEMM_3M, [256, 512])
    log = native.bem_autotune_lu_results(ctx)
    assert len(log) == 6
    assert {(r[0], r[1], r[2]) for r in log} == {(nb, w, p) for nb in (256, 512)
                                                 for (w, p) in ((64, 0), (128, 0), (64, 1))}
    fastest = min(log, key=lambda r: r[3])
    assert native.bem_lu_tuned_plan(ctx, native.BEM_C64, n, native.BEM_GEMM_3M) == fastest[:3]
    assert best == fastest[0] and abs(ms - fastest[3]) < 1e-9
