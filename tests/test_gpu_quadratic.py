"""GPU parity of the quadratic-element path (Sec. III: quadratic interpolants,
Gauss quadrature of the non-singular integrands; Sec. IV A: 500 elements, 1002
nodes) against the quadratic oracle, through the C ABI: element-loop assembly
entry by entry, the solve in every mode, and the field by element quadrature."""
import numpy as np
import pytest

from oracle import quadratic as Q
from workloads import Body, HARD, SOFT, seeded_complex

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_1706_07919_amd.native")
from paper_1706_07919_amd import DeviceQuadSurface  # noqa: E402


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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("nu,bc", [(2, HARD), (3, SOFT)])
def test_assemble_quadratic_entries_diag_rhs(ctx, nu, bc):
    body = Body((0.1, -0.2, 0.3), 0.9, 1.4, 0, bc)       # a prolate spheroid
    qs = Q.QuadSurface(body, nu)
    ds = DeviceQuadSurface.from_body(body, nu)
    n = qs.n
    k = np.array([0.6, 3.3, 7.9])
    rng = np.random.default_rng(nu)
    nr = 5                                               # two assembly launches of b
    y = seeded_complex(rng, (len(k), nr, n))
    ld = n + 3
    A = torch.zeros((len(k), n, ld), dtype=torch.complex128, device="cuda")
    A32 = torch.zeros((len(k), n, ld), dtype=torch.complex64, device="cuda")
    b = torch.zeros((len(k), nr, n), dtype=torch.complex128, device="cuda")
    dg = torch.zeros((len(k), n, 2), dtype=torch.complex128, device="cuda")
    native.bem_assemble_quadratic(ctx, ds.struct, len(k), dev(k), nr, dev(y), native.BEM_C128, A,
                                  ld, b, dg)
    native.bem_assemble_quadratic(ctx, ds.struct, len(k), dev(k), nr, dev(y), native.BEM_C64, A32,
                                  ld, b, None)
    A = A.cpu().numpy()[:, :, :n]
    A32 = A32.cpu().numpy()[:, :, :n].astype(np.complex128)
    b = b.cpu().numpy()
    dg = dg.cpu().numpy()
    for q, kq in enumerate(k):
        Mphi, Mpsi = Q.operator_matrices(qs, kq)
        hard = qs.bc == HARD
        Aref = np.where(hard[None, :], Mphi, Mpsi)
        scale = np.max(np.abs(Aref), axis=1, keepdims=True)
        assert np.max(np.abs(A[q] - Aref) / scale) < 1e-12
        assert np.max(np.abs(A32[q] - Aref) / scale) < 1.2e-7
        assert np.max(np.abs(dg[q, :, 0] - np.diag(Mphi))) < 1e-11 * np.max(np.abs(np.diag(Mphi)))
        assert np.max(np.abs(dg[q, :, 1] - np.diag(Mpsi))) < 1e-11 * np.max(np.abs(np.diag(Mpsi)))
        for r in range(nr):
            _, bref = Q.system(qs, kq, y[q, r])
            assert rel(b[q, r], bref) < 1e-12


@pytest.mark.parametrize("mode", [native.BEM_FP64_DIRECT, native.BEM_FP32_IR_3M,
                                  native.BEM_FP32_IR_4M])
def test_solve_quadratic_paper_sphere_vs_oracle(ctx, mode):
    """The paper's sphere (500 elements, 1002 nodes), sound-soft, under the
    plane wave: every mode returns the oracle's FP64 direct solution."""
    body = Body((0.0, 0.0, 0.0), 1.0, 1.0, 0, SOFT)
    qs = Q.QuadSurface(body, 5)
    ds = DeviceQuadSurface.from_body(body, 5)
    k = np.array([0.5, 2.5, 16 * np.pi / 20.1, 5.1])
    y = np.zeros((len(k), 1, qs.n), np.complex128)
    for q, kq in enumerate(k):
        p, dp = Q.incident_plane_wave(qs, kq)
        y[q, 0] = -p
    x = torch.zeros((len(k), 1, qs.n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    opts.mode = mode
    info = native.bem_solve_quadratic(ctx, ds.struct, len(k), dev(k), 1, dev(y), opts, x)
    xg = x.cpu().numpy()[:, 0]
    for q, kq in enumerate(k):
        _, _, xs = Q.solve(qs, kq, y[q, 0])
        assert rel(xg[q], xs) < (1e-11 if mode == native.BEM_FP64_DIRECT else 1e-8), (kq, rel(xg[q], xs))
        assert info[q].converged == 1 and 0 < info[q].rel_resid < 1e-10
        if mode != native.BEM_FP64_DIRECT:
            assert info[q].used_fp64 == 0 and 1 <= info[q].iters <= 6


def test_solve_quadratic_fallback_forced(ctx):
    """With no refinement sweep allowed to converge (tolerance 0), every item
    is re-solved in float64 and flagged; with fallback off the call fails."""
    body = Body((0.0, 0.0, 0.0), 1.0, 1.0, 0, HARD)
    qs = Q.QuadSurface(body, 2)
    ds = DeviceQuadSurface.from_body(body, 2)
    k = np.array([1.0, 2.0])
    y = seeded_complex(np.random.default_rng(3), (2, 1, qs.n))
    x = torch.zeros((2, 1, qs.n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    opts.tol_step = 0.0
    opts.max_iter = 2
    info = native.bem_solve_quadratic(ctx, ds.struct, 2, dev(k), 1, dev(y), opts, x)
    for q in range(2):
        assert info[q].used_fp64 == 1 and info[q].converged == 1
        _, _, xs = Q.solve(qs, k[q], y[q, 0])
        assert rel(x[q, 0].cpu().numpy(), xs) < 1e-11
    opts.fallback = 0
    with pytest.raises(native.BemError):
        native.bem_solve_quadratic(ctx, ds.struct, 2, dev(k), 1, dev(y), opts, x)


def test_field_quadratic_vs_oracle(ctx):
    """Eq. BRIEFdmn by element quadrature at points near and far from a hard
    spheroid, two right-hand sides: equal to the oracle's field, the point
    on a node returning the nodal value, inside points 0."""
    body = Body((0.0, 0.0, 0.0), 1.0, 1.3, 0, HARD)
    qs = Q.QuadSurface(body, 3)
    ds = DeviceQuadSurface.from_body(body, 3)
    k = np.array([0.8, 4.1])
    rng = np.random.default_rng(5)
    phi = seeded_complex(rng, (2, 2, qs.n))
    psi = seeded_complex(rng, (2, 2, qs.n))
    pts = np.concatenate([rng.uniform(-3, 3, (60, 3)), qs.x[[7, 200]] * 1.05, qs.x[[11]],
                          [[0.0, 0.0, 0.1]]])
    m = len(pts)
    U = torch.zeros((2, m, 2), dtype=torch.complex128, device="cuda")
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    native.bem_field_eval_quadratic(ctx, ds.struct, 2, dev(k), 2, dev(phi), dev(psi), m, dev(pts),
                                    i0, ins, U)
    U = U.cpu().numpy()
    for r in range(2):
        for q, kq in enumerate(k):
            ref, oi0, oins = Q.field(qs, kq, phi[q, r], psi[q, r], pts)
            assert np.array_equal(i0.cpu().numpy(), oi0) and np.array_equal(ins.cpu().numpy(), oins)
            assert np.max(np.abs(U[r, :, q] - ref)) < 1e-11 * np.max(np.abs(ref))
            assert U[r, m - 2, q] == phi[q, r, 11]
            assert U[r, m - 1, q] == 0


def test_solve_quadratic_chunked_several_rhs(ctx):
    """A workspace limit that holds two wavenumbers at a time: the solve runs in
    ragged chunks (2, 2, 1) with three right-hand sides each and still returns
    the oracle's FP64 solutions."""
    body = Body((0.2, 0.0, -0.1), 1.0, 1.25, 0, HARD)
    qs = Q.QuadSurface(body, 3)
    ds = DeviceQuadSurface.from_body(body, 3)
    k = np.array([0.7, 1.9, 3.1, 4.4, 5.6])
    nr = 3
    y = seeded_complex(np.random.default_rng(21), (len(k), nr, qs.n))
    x = torch.zeros((len(k), nr, qs.n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_3M
    per_k = 2 * qs.n * ((qs.n + 15) // 16 * 16) * 16
    ctx.set_workspace_limit(int(2.5 * per_k))
    try:
        info = native.bem_solve_quadratic(ctx, ds.struct, len(k), dev(k), nr, dev(y), opts, x)
    finally:
        ctx.set_workspace_limit(0)
    xg = x.cpu().numpy()
    for q, kq in enumerate(k):
        for r in range(nr):
            _, _, xs = Q.solve(qs, kq, y[q, r])
            assert rel(xg[q, r], xs) < 1e-8, (kq, r)
            assert info[q * nr + r].converged == 1
