"""GPU parity of every step of the hot path against the FP64 oracle, called
through the C ABI.  Sizes are small enough for the oracle to finish in seconds
while spanning several tiles and ragged tails."""
import numpy as np
import pytest

from oracle import bie, field as ofield, pulse as opulse
from oracle.mesh import Surface
from workloads import Body, HARD, SOFT, Pulse, sphere_l2_workload, ring_points, seeded_complex

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


def mixed_bodies(level=1):
    return [Body((0.0, 0.0, -1.4), 1.0, 1.0, level, HARD),
            Body((0.3, 0.1, 1.3), 0.8, 1.6, level, SOFT)]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ------------------------------------------------------------------ S2
def test_incident_known_data(ctx):
    bodies = mixed_bodies(1)
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    k = np.array([0.3, 2.0, 7.5])
    y = torch.empty((3, s.n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, 3, dev(k), (0.0, 0.0, 1.0), y)
    got = y.cpu().numpy()
    for q in range(3):
        p, dp = bie.incident_plane_wave(s, k[q])
        ref = bie.known_data(s, p, dp)
        assert np.max(np.abs(got[q] - ref)) < 1e-13 * np.max(np.abs(ref))


# ------------------------------------------------------------------ S3/S4
# wavenumber sets: scattered values (one sincos per wavenumber), an evenly
# spaced grid with a ragged last chunk whose tail breaks the spacing (phase
# recurrence inside the uniform chunks, direct evaluation in the rest), and an
# evenly spaced grid whose last chunk is evenly spaced but partial (13 = 8 + 5)
K_SETS = {"scattered": np.array([0.7, 3.1, 9.4]),
          "grid": np.concatenate([0.75 * np.arange(1, 10), [7.9, 11.3]]),
          "even13": 0.5 * np.arange(1, 14)}


@pytest.mark.parametrize("kset", ["scattered", "grid", "even13"])
@pytest.mark.parametrize("level", [1, 2])
def test_assemble_c128_entries_diag_rhs(ctx, level, kset):
    bodies = mixed_bodies(level)
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    n = s.n
    k = K_SETS[kset]
    nk = len(k)
    rng = np.random.default_rng(0)
    nr = 5 if kset == "scattered" else 2
    y = seeded_complex(rng, (nk, nr, n))
    ld = n + 3
    A = torch.zeros((nk, n, ld), dtype=torch.complex128, device="cuda")
    b = torch.zeros((nk, nr, n), dtype=torch.complex128, device="cuda")
    dg = torch.zeros((nk, n, 2), dtype=torch.complex128, device="cuda")
    native.bem_assemble(ctx, ds.struct, nk, dev(k), nr, dev(y), native.BEM_C128, A, ld, b, dg)
    A = A.cpu().numpy()[:, :, :n]
    b = b.cpu().numpy()
    dg = dg.cpu().numpy()
    for q in range(nk):
        Mphi, Mpsi = bie.operator_matrices(s, k[q])
        Aref, _ = bie.system(s, k[q], y[q, 0])
        scale = np.max(np.abs(Aref), axis=1, keepdims=True)
        assert np.max(np.abs(A[q] - Aref) / scale) < 1e-12
        assert np.max(np.abs(dg[q, :, 0] - np.diag(Mphi))) < 1e-11
        assert np.max(np.abs(dg[q, :, 1] - np.diag(Mpsi))) < 1e-11
        for r in range(nr):
            _, bref = bie.system(s, k[q], y[q, r])
            assert rel(b[q, r], bref) < 1e-12


@pytest.mark.parametrize("k", [[0.9, 3.0e5, 3.05e5], [4.0e5, 4.0e5 + 1.0, 4.0e5 + 2.0]],
                         ids=["scattered", "grid"])
def test_assemble_phases_past_near_range(ctx, k):
    """Wavenumbers whose phases k r reach past 2^20 rad: the rows are redone
    with the library sine and cosine, and the entries, diagonal sums and b
    still match the oracle (to the phase's own rounding, k ulp(r))."""
    bodies = mixed_bodies(1)
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    n = s.n
    k = np.array(k)
    nk = len(k)
    y = seeded_complex(np.random.default_rng(7), (nk, 2, n))
    A = torch.zeros((nk, n, n), dtype=torch.complex128, device="cuda")
    b = torch.zeros((nk, 2, n), dtype=torch.complex128, device="cuda")
    dg = torch.zeros((nk, n, 2), dtype=torch.complex128, device="cuda")
    native.bem_assemble(ctx, ds.struct, nk, dev(k), 2, dev(y), native.BEM_C128, A, n, b, dg)
    A, b, dg = A.cpu().numpy(), b.cpu().numpy(), dg.cpu().numpy()
    assert np.max(k) * np.max(np.linalg.norm(s.x[:, None] - s.x[None], axis=2)) > 2.0 ** 20
    for q in range(nk):
        Mphi, Mpsi = bie.operator_matrices(s, k[q])
        Aref, _ = bie.system(s, k[q], y[q, 0])
        scale = np.max(np.abs(Aref), axis=1, keepdims=True)
        assert np.max(np.abs(A[q] - Aref) / scale) < 1e-8
        assert np.max(np.abs(dg[q, :, 0] - np.diag(Mphi)) / scale[:, 0]) < 1e-6
        assert np.max(np.abs(dg[q, :, 1] - np.diag(Mpsi)) / scale[:, 0]) < 1e-6
        for r in range(2):
            _, bref = bie.system(s, k[q], y[q, r])
            assert rel(b[q, r], bref) < 1e-6


def test_assemble_without_rhs(ctx):
    """No right-hand side (y and b NULL): the matrix and the diagonal only,
    equal to the oracle's; nothing reads y or writes b."""
    bodies = mixed_bodies(1)
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    n = s.n
    k = K_SETS["grid"]
    nk = len(k)
    A = torch.zeros((nk, n, n), dtype=torch.complex128, device="cuda")
    dg = torch.zeros((nk, n, 2), dtype=torch.complex128, device="cuda")
    native.bem_assemble(ctx, ds.struct, nk, dev(k), 0, None, native.BEM_C128, A, n, None, dg)
    A, dg = A.cpu().numpy(), dg.cpu().numpy()
    for q in range(nk):
        Mphi, Mpsi = bie.operator_matrices(s, k[q])
        Aref = np.where((s.bc == HARD)[None, :], Mphi, Mpsi)
        scale = np.max(np.abs(Aref), axis=1, keepdims=True)
        assert np.max(np.abs(A[q] - Aref) / scale) < 1e-12
        assert np.max(np.abs(dg[q, :, 0] - np.diag(Mphi))) < 1e-11
        assert np.max(np.abs(dg[q, :, 1] - np.diag(Mpsi))) < 1e-11


def test_assemble_c64_is_rounded_fp64(ctx):
    bodies = mixed_bodies(2)
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    n = s.n
    k = np.array([5.3])
    y = seeded_complex(np.random.default_rng(1), (1, 1, n))
    A = torch.zeros((1, n, n), dtype=torch.complex64, device="cuda")
    b = torch.zeros((1, 1, n), dtype=torch.complex128, device="cuda")
    native.bem_assemble(ctx, ds.struct, 1, dev(k), 1, dev(y), native.BEM_C64, A, n, b, None)
    Aref, bref = bie.system(s, k[0], y[0, 0])
    got = A.cpu().numpy()[0].astype(np.complex128)
    assert np.max(np.abs(got - Aref) / np.abs(Aref).max(axis=1, keepdims=True)) < 1.2e-7
    assert rel(b.cpu().numpy()[0, 0], bref) < 1e-12


def test_residual_entry_points_reject_nonpositive_k(ctx):
    """k <= 0 is rejected before any launch by every entry point that
    regenerates the operator (the diagonal sums divide by k)."""
    bodies = mixed_bodies(1)
    ds = DeviceSurface.from_bodies(bodies)
    n = ds.n
    k = dev(np.array([1.0, 0.0]))
    z = torch.zeros((2, 1, n), dtype=torch.complex128, device="cuda")
    dg = torch.zeros((2, n, 2), dtype=torch.complex128, device="cuda")
    with pytest.raises(native.BemError):
        native.bem_residual_check(ctx, ds.struct, 2, k, 1, z, z)
    with pytest.raises(native.BemError):
        native.bem_residual(ctx, ds.struct, 2, k, 1, z, z, dg, z)
    with pytest.raises(native.BemError):
        native.bem_assemble(ctx, ds.struct, 2, k, 1, z, native.BEM_C128, None, n, z, dg)


@pytest.mark.parametrize("kset", ["scattered", "grid", "even13"])
def test_residual_matrix_free(ctx, kset):
    bodies = mixed_bodies(2)
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    n = s.n
    k = K_SETS[kset]
    nk = len(k)
    rng = np.random.default_rng(2)
    y = seeded_complex(rng, (nk, 2, n))
    x = seeded_complex(rng, (nk, 2, n))
    A = torch.zeros((nk, n, n), dtype=torch.complex128, device="cuda")
    b = torch.zeros((nk, 2, n), dtype=torch.complex128, device="cuda")
    dg = torch.zeros((nk, n, 2), dtype=torch.complex128, device="cuda")
    r = torch.zeros((nk, 2, n), dtype=torch.complex128, device="cuda")
    native.bem_assemble(ctx, ds.struct, nk, dev(k), 2, dev(y), native.BEM_C128, A, n, b, dg)
    native.bem_residual(ctx, ds.struct, nk, dev(k), 2, dev(y), dev(x), dg, r)
    r = r.cpu().numpy()
    for q in range(nk):
        for j in range(2):
            Aref, bref = bie.system(s, k[q], y[q, j])
            ref = bref - Aref @ x[q, j]
            assert rel(r[q, j], ref) < 1e-12


# ------------------------------------------------------------------ S5/S6 building blocks
@pytest.mark.parametrize("prec", [native.BEM_C128, native.BEM_C64])
@pytest.mark.parametrize("n,nb", [(1, 0), (5, 0), (33, 0), (130, 0), (300, 64), (530, 0), (777, 0),
                                  (1100, 256)])
def test_getrf_getrs_random(ctx, prec, n, nb):
    rng = np.random.default_rng(n)
    batch = 3
    ld = n + (1 if n % 2 else 2)
    M = seeded_complex(rng, (batch, n, n)) + 0.5 * np.sqrt(n) * np.eye(n)[None]
    M[1] = M[1][rng.permutation(n)]       # forces row interchanges
    M[2] = seeded_complex(rng, (n, n))    # plain Gaussian: interchanges at most steps
    cdt = torch.complex128 if prec == native.BEM_C128 else torch.complex64
    A = torch.zeros((batch, n, ld), dtype=cdt)
    A[:, :, :n] = torch.as_tensor(M)
    A = A.cuda()
    piv = torch.zeros((batch, n), dtype=torch.int32, device="cuda")
    info = torch.ones(batch, dtype=torch.int32, device="cuda")
    native.bem_getrf_batched(ctx, prec, n, ld, n * ld, batch, A, piv, info, nb, 0)
    assert info.cpu().numpy().tolist() == [0] * batch
    B = seeded_complex(rng, (batch, 2, n))
    X = torch.zeros((batch, 2, n), dtype=cdt, device="cuda")
    native.bem_getrs_batched(ctx, prec, n, ld, n * ld, batch, A, piv, 2, dev(B, cdt), X, 2 * n)
    X = X.cpu().numpy().astype(np.complex128)
    # normwise backward error ||B - M X||_F / (||M||_F ||X||_F) of every
    # matrix: the criterion a float32 factorisation meets whatever the
    # conditioning (LAPACK's float32 factors reach 4-5e-7 at n = 1100)
    eta = 1e-14 if prec == native.BEM_C128 else 1e-6
    for b_ in range(batch):
        res = np.linalg.norm(M[b_] @ X[b_].T - B[b_].T) / (np.linalg.norm(M[b_]) * np.linalg.norm(X[b_]))
        assert res < eta, (b_, res)
    # forward error of the shifted matrices; in float32 it scales with the
    # condition number (about 9e3 for the first matrix at n = 1100, where
    # LAPACK's float32 solve is off by 3e-4)
    for b_ in range(2):
        ref = np.linalg.solve(M[b_], B[b_].T).T
        assert rel(X[b_], ref) < (1e-11 if prec == native.BEM_C128 else 2e-3)
    if n <= 600:  # P A = L U reconstruction
        LU = A.cpu().numpy()[:, :, :n].astype(np.complex128)
        p = piv.cpu().numpy()
        for b_ in range(batch):
            L = np.tril(LU[b_], -1) + np.eye(n)
            U = np.triu(LU[b_])
            PA = M[b_].copy()
            for i in range(n):
                PA[[i, p[b_, i]]] = PA[[p[b_, i], i]]
            assert np.max(np.abs(L @ U - PA)) < (1e-12 if prec == native.BEM_C128 else 1e-4) * np.sqrt(n) * 4


@pytest.mark.parametrize("kind", [native.BEM_GEMM_3M, native.BEM_GEMM_BF16X3])
@pytest.mark.parametrize("n", [130, 777])
def test_getrf_3m_and_split_gemm(ctx, n, kind):
    rng = np.random.default_rng(n + 1)
    M = seeded_complex(rng, (2, n, n)) + 0.5 * np.sqrt(n) * np.eye(n)[None]
    A = dev(M, torch.complex64)
    piv = torch.zeros((2, n), dtype=torch.int32, device="cuda")
    info = torch.ones(2, dtype=torch.int32, device="cuda")
    native.bem_getrf_batched(ctx, native.BEM_C64, n, n, n * n, 2, A, piv, info, 64, kind)
    B = seeded_complex(rng, (2, 1, n))
    X = torch.zeros((2, 1, n), dtype=torch.complex64, device="cuda")
    native.bem_getrs_batched(ctx, native.BEM_C64, n, n, n * n, 2, A, piv, 1, dev(B, torch.complex64), X, n)
    X = X.cpu().numpy().astype(np.complex128)
    for b_ in range(2):
        # The 3-product form has a larger error bound than 4M (imaginary parts
        # combine three rounded products).  The bf16 split keeps about 17 bits
        # per operand (unit roundoff ~ 2^-17 instead of 2^-24), so its backward
        # error is ~100x that of float32 (a float64 model of the same splitting
        # gives 5.6e-6 at n = 777); refinement only needs a contraction < 1.
        x = X[b_, 0]
        bwd = np.linalg.norm(M[b_] @ x - B[b_, 0]) / (np.linalg.norm(M[b_]) * np.linalg.norm(x))
        if kind == native.BEM_GEMM_3M:
            assert rel(x, np.linalg.solve(M[b_], B[b_, 0])) < 2e-3
            assert bwd < 3e-6
        else:
            assert bwd < 3e-5


@pytest.mark.parametrize("kind", [native.BEM_GEMM_4M, native.BEM_GEMM_3M])
@pytest.mark.parametrize("n,pad,nb", [(300, 0, 72), (300, 1, 72), (777, 1, 0), (1100, 0, 256),
                                      (1030, 2, 512)])
def test_getrf_fp32_forms_backward_error(ctx, kind, n, pad, nb):
    """Float32 factorisations with 4M and 3M products: an even leading dimension
    takes the LDS-streamed kernel (a block width of 72 gives depths with a
    partial last 16-k stage, 1030 rows a ragged last tile), an odd one the
    register-staged kernel; both meet the float32 normwise backward-error bound
    and reconstruct P A = L U."""
    rng = np.random.default_rng(n + pad + nb)
    batch = 3
    ld = n + pad
    M = seeded_complex(rng, (batch, n, n)) + 0.5 * np.sqrt(n) * np.eye(n)[None]
    M[1] = M[1][rng.permutation(n)]
    M[2] = seeded_complex(rng, (n, n))
    A = torch.zeros((batch, n, ld), dtype=torch.complex64)
    A[:, :, :n] = torch.as_tensor(M)
    A = A.cuda()
    piv = torch.zeros((batch, n), dtype=torch.int32, device="cuda")
    info = torch.ones(batch, dtype=torch.int32, device="cuda")
    native.bem_getrf_batched(ctx, native.BEM_C64, n, ld, n * ld, batch, A, piv, info, nb, kind)
    assert info.cpu().numpy().tolist() == [0] * batch
    B = seeded_complex(rng, (batch, 1, n))
    X = torch.zeros((batch, 1, n), dtype=torch.complex64, device="cuda")
    native.bem_getrs_batched(ctx, native.BEM_C64, n, ld, n * ld, batch, A, piv, 1,
                             dev(B, torch.complex64), X, n)
    X = X.cpu().numpy().astype(np.complex128)
    for b_ in range(batch):
        x = X[b_, 0]
        bwd = np.linalg.norm(M[b_] @ x - B[b_, 0]) / (np.linalg.norm(M[b_]) * np.linalg.norm(x))
        assert bwd < (1e-6 if kind == native.BEM_GEMM_4M else 3e-6), (b_, bwd)
    if n <= 300:
        LU = A.cpu().numpy()[:, :, :n].astype(np.complex128)
        p = piv.cpu().numpy()
        for b_ in range(batch):
            L = np.tril(LU[b_], -1) + np.eye(n)
            U = np.triu(LU[b_])
            PA = M[b_].copy()
            for i in range(n):
                PA[[i, p[b_, i]]] = PA[[p[b_, i], i]]
            assert np.max(np.abs(L @ U - PA)) < 1e-4 * np.sqrt(n) * 4


@pytest.mark.parametrize("n,nb,batch,limit", [
    (777, 64, 3, 0),                     # every trailing update in one packed launch
    (1100, 256, 5, 4 * 8 * 1024 * 1024),  # 8 MiB packing buffer: batches packed in slices
    (530, 128, 2, 4096),                 # buffer too small for one matrix: unpacked kernel
    (1300, 72, 2, 0),                    # depth 72: an odd number of 8-k blocks per stage pair
])
def test_packed_trailing_update_matches_unpacked(ctx, n, nb, batch, limit):
    """The pre-split operands feed the same products in the same order, so the
    factors and pivots equal those of the unpacked kernel bit for bit, with a
    ragged last tile and block, in slices, and when nothing can be packed."""
    rng = np.random.default_rng(n + nb)
    M = seeded_complex(rng, (batch, n, n)) + 0.5 * np.sqrt(n) * np.eye(n)[None]
    out = {}
    ctx.set_workspace_limit(limit)
    try:
        for kind in (native.BEM_GEMM_BF16X3, native.BEM_GEMM_BF16X3_UNPACKED):
            A = dev(M, torch.complex64)
            piv = torch.zeros((batch, n), dtype=torch.int32, device="cuda")
            info = torch.ones(batch, dtype=torch.int32, device="cuda")
            native.bem_getrf_batched(ctx, native.BEM_C64, n, n, n * n, batch, A, piv, info, nb, kind)
            out[kind] = (A.cpu().numpy(), piv.cpu().numpy(), info.cpu().numpy())
    finally:
        ctx.set_workspace_limit(0)
    a, b = out[native.BEM_GEMM_BF16X3], out[native.BEM_GEMM_BF16X3_UNPACKED]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]) and not a[2].any()
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))


def test_autotune_block_width_then_factor(ctx):
    """The tuner times each candidate width on pseudo-random matrices and keeps
    the fastest for the size class; a later nb = 0 factorisation of that class
    uses it and stays correct."""
    n = 300
    best, ms = native.bem_autotune_lu(ctx, native.BEM_C64, n, 4, native.BEM_GEMM_BF16X3, [64, 128])
    assert best in (64, 128) and ms > 0
    rng = np.random.default_rng(5)
    M = seeded_complex(rng, (2, n, n)) + 0.5 * np.sqrt(n) * np.eye(n)[None]
    A = dev(M, torch.complex64)
    piv = torch.zeros((2, n), dtype=torch.int32, device="cuda")
    info = torch.ones(2, dtype=torch.int32, device="cuda")
    native.bem_getrf_batched(ctx, native.BEM_C64, n, n, n * n, 2, A, piv, info, 0,
                             native.BEM_GEMM_BF16X3)
    B = seeded_complex(rng, (2, 1, n))
    X = torch.zeros((2, 1, n), dtype=torch.complex64, device="cuda")
    native.bem_getrs_batched(ctx, native.BEM_C64, n, n, n * n, 2, A, piv, 1, dev(B, torch.complex64), X, n)
    X = X.cpu().numpy().astype(np.complex128)
    for b_ in range(2):
        # backward error of the bf16-split factorisation (see the split-GEMM test)
        x = X[b_, 0]
        bwd = np.linalg.norm(M[b_] @ x - B[b_, 0]) / (np.linalg.norm(M[b_]) * np.linalg.norm(x))
        assert bwd < 3e-5
    with pytest.raises(native.BemError):
        native.bem_autotune_lu(ctx, native.BEM_C64, n, 2, 7)


def test_getrf_reports_singular(ctx):
    n = 40
    M = seeded_complex(np.random.default_rng(9), (1, n, n))
    M[0, :, 7] = 0.0
    A = dev(M, torch.complex128)
    piv = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    native.bem_getrf_batched(ctx, native.BEM_C128, n, n, n * n, 1, A, piv, info, 0, 0)
    assert int(info.item()) == 8


# ------------------------------------------------------------------ S2..S6 end to end
def _solve(ctx, bodies, k, mode, n_rhs=1, rng=None):
    ds = DeviceSurface.from_bodies(bodies)
    n = ds.n
    kd = dev(k)
    y = torch.empty((len(k), n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, len(k), kd, (0.0, 0.0, 1.0), y)
    if n_rhs > 1:
        extra = dev(seeded_complex(rng, (len(k), n_rhs - 1, n)))
        y = torch.cat([y[:, None, :], extra], dim=1).contiguous()
    x = torch.zeros((len(k), n_rhs, n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    opts.mode = mode
    info = native.bem_solve_batched(ctx, [(ds.struct, len(k), kd, n_rhs, y)], opts, [x])
    return ds, kd, y, x, info


@pytest.mark.parametrize("mode", [native.BEM_FP64_DIRECT, native.BEM_FP32_IR_4M, native.BEM_FP32_IR_3M,
                                  native.BEM_FP32_IR_B3])
def test_solve_sphere_l2_vs_oracle(ctx, mode):
    w = sphere_l2_workload()
    s = Surface(w.bodies)
    ds, kd, y, x, info = _solve(ctx, w.bodies, w.k, mode)
    x = x.cpu().numpy()[:, 0]
    errs = []
    for q, kq in enumerate(w.k):
        p, dp = bie.incident_plane_wave(s, kq)
        yq = bie.known_data(s, p, dp)
        _, _, xs = bie.solve(s, kq, yq)
        errs.append(rel(x[q], xs))
    assert max(errs) < 1e-6, max(errs)
    for q in range(len(w.k)):
        assert info[q].rel_resid < 1e-9
        if mode != native.BEM_FP64_DIRECT:
            assert info[q].used_fp64 == 0 and 2 <= info[q].iters <= 6


def test_solve_mixed_bc_multi_rhs_vs_oracle(ctx):
    bodies = mixed_bodies(2)
    s = Surface(bodies)
    k = np.array([0.5, 2.5, 4.0, 8.8, 11.9])
    rng = np.random.default_rng(4)
    ds, kd, y, x, info = _solve(ctx, bodies, k, native.BEM_FP32_IR_4M, n_rhs=3, rng=rng)
    x = x.cpu().numpy()
    y = y.cpu().numpy()
    for q in range(len(k)):
        _, _, xs = bie.solve(s, k[q], y[q].T)
        assert rel(x[q], xs.T) < 1e-6


def test_refinement_items_stopping_at_different_sweeps(ctx):
    """Items of one chunk leave the refinement at different sweeps (a tight
    step tolerance, and wavenumbers next to the interior resonances ka = pi,
    4.4934 of the sphere, whose items contract more slowly than the others):
    every item still returns the discrete FP64 solution, and its reported FP64
    residual is the residual of the x it returns (a correction dropped for an
    item that stops would break both)."""
    bodies = [Body((0.0, 0.0, 0.0), 1.0, 1.0, 3, HARD)]
    k = np.array([0.7, 2.0, 4.43, 4.46, 4.49, 4.52, 6.1, 8.3, 3.10, 3.13, 3.16, 3.19, 5.0,
                  9.7, 1.3, 11.4])
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    kd = dev(k)
    y = torch.empty((len(k), 1, ds.n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, len(k), kd, (0.0, 0.0, 1.0), y)
    x = torch.zeros((len(k), 1, ds.n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_3M
    opts.tol_step = 1e-13
    opts.max_iter = 12
    info = native.bem_solve_batched(ctx, [(ds.struct, len(k), kd, 1, y)], opts, [x])
    iters = [info[q].iters for q in range(len(k))]
    assert len(set(iters)) >= 2, iters
    rr = native.bem_residual_check(ctx, ds.struct, len(k), kd, 1, y, x)
    xg = x.cpu().numpy()[:, 0]
    for q, kq in enumerate(k):
        p, dp = bie.incident_plane_wave(s, kq)
        _, _, xs = bie.solve(s, kq, bie.known_data(s, p, dp))
        assert info[q].converged == 1 and info[q].used_fp64 == 0, (kq, iters)
        assert rel(xg[q], xs) < 1e-9, (kq, rel(xg[q], xs))
        assert abs(info[q].rel_resid - rr[q]) <= 1e-6 * rr[q] + 1e-16, (kq, info[q].rel_resid, rr[q])


def test_bowl_solve_and_field_vs_oracle(ctx):
    """The hard acoustic bowl of Sec. IV C (Eq. dish, axis turned by 0.15 pi
    from the propagation direction; 16 x 24 rings, 362 nodes, a thin shell with
    a sharp rim): refined solves at wavenumbers around the paper's carrier
    k0 a = 24 pi / 20.1 and the field at points on the concave side match the
    oracle."""
    from oracle.mesh import ArraySurface, bowl
    x, nrm, w, _ = native.bem_mesh_bowl(16, 24, 1.0, 0.15 * np.pi, (0.0, 0.0, 0.0))
    bc = np.zeros(len(x), dtype=np.uint8)
    s = ArraySurface(*bowl(16, 24, 1.0, 0.15 * np.pi)[:3], bc)
    ds = DeviceSurface(x, nrm, w, bc)
    k = np.array([0.7, 24 * np.pi / 20.1, 6.1])
    kd = dev(k)
    y = torch.empty((len(k), 1, ds.n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, len(k), kd, (0.0, 0.0, 1.0), y)
    xs = torch.zeros_like(y)
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_B3
    info = native.bem_solve_batched(ctx, [(ds.struct, len(k), kd, 1, y)], opts, [xs])
    assert all(info[q].converged == 1 for q in range(len(k)))
    phi, psi = torch.empty_like(xs), torch.empty_like(xs)
    native.bem_split_unknowns(ctx, ds.struct, len(k), 1, xs, y, phi, psi)
    X = xs.cpu().numpy()[:, 0]
    pts = np.array([[0.0, -0.3 * np.sin(0.15 * np.pi), -0.3 * np.cos(0.15 * np.pi) - 0.6],
                    [0.0, 0.0, -1.0], [0.4, 0.2, -0.9], [0.0, 1.5, 1.0]])
    m = len(pts)
    U = torch.zeros((1, m, len(k)), dtype=torch.complex64, device="cuda")
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    native.bem_field_eval(ctx, ds.struct, len(k), kd, 1, phi, psi, m, dev(pts), i0, 0, ins,
                          native.BEM_C64, U)
    U = U.cpu().numpy()[0]
    for q in range(len(k)):
        p, dp = bie.incident_plane_wave(s, k[q])
        ph, ps, xo = bie.solve(s, k[q], bie.known_data(s, p, dp))
        assert rel(X[q], xo) < 1e-8
        ref, oi0, oins = ofield.field(s, k[q], ph, ps, pts)
        assert np.array_equal(i0.cpu().numpy(), oi0) and np.array_equal(ins.cpu().numpy(), oins)
        assert np.max(np.abs(U[:, q] - ref)) < 2e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("mode", [native.BEM_FP32_IR_4M, native.BEM_FP32_IR_3M, native.BEM_FP32_IR_B3,
                                  native.BEM_FP64_DIRECT])
def test_solve_uneven_batch_vs_oracle(ctx, mode):
    """Bodies of 42, 162 and 642 nodes (one problem each, different k counts)
    factored together in one recursion per round."""
    problems = [([Body((0.0, 0.0, 0.0), 0.6, 1.0, 1, SOFT)], np.array([0.5, 3.0, 7.7])),
                ([Body((0.0, 0.0, 0.0), 0.9, 2.2, 2, HARD)], np.array([1.0, 4.4])),
                ([Body((0.0, 0.0, 0.0), 1.2, 1.0, 3, SOFT)], np.array([0.8, 2.9, 5.1, 9.9]))]
    args, outs, keep = [], [], []
    for bodies, k in problems:
        ds = DeviceSurface.from_bodies(bodies)
        kd = dev(k)
        y = torch.empty((len(k), 1, ds.n), dtype=torch.complex128, device="cuda")
        native.bem_incident(ctx, ds.struct, len(k), kd, (0.0, 0.0, 1.0), y)
        x = torch.zeros((len(k), 1, ds.n), dtype=torch.complex128, device="cuda")
        args.append((ds.struct, len(k), kd, 1, y))
        outs.append(x)
        keep.append((ds, kd, y))
    opts = native.bem_solve_opts_default()
    opts.mode = mode
    ctx.set_workspace_limit(8 * 1024 * 1024)   # forces several rounds
    try:
        info = native.bem_solve_batched(ctx, args, opts, outs)
    finally:
        ctx.set_workspace_limit(0)
    q = 0
    for (bodies, k), x in zip(problems, outs):
        s = Surface(bodies)
        for j, kq in enumerate(k):
            p, dp = bie.incident_plane_wave(s, kq)
            _, _, xs = bie.solve(s, kq, bie.known_data(s, p, dp))
            assert rel(x[j, 0].cpu().numpy(), xs) < 1e-6
            assert info[q].rel_resid < 1e-9
            q += 1


@pytest.mark.parametrize("mode", [native.BEM_FP32_IR_B3, native.BEM_FP64_DIRECT])
def test_solve_graph_replays_match_eager(ctx, mode):
    """The factorisation captured as a hipGraph and replayed: every replay,
    with eager work of another problem in between, gives the eager result bit
    for bit (same kernels on the same data); a different problem size makes a
    second capture, and the first one keeps replaying correctly."""
    import time
    problems = [([Body((0.0, 0.0, 0.0), 0.9, 2.2, 2, HARD)], np.array([1.0, 4.4, 6.1])),
                ([Body((0.0, 0.0, 0.0), 1.0, 1.0, 2, SOFT)], np.array([0.7, 2.5]))]
    prepared = []
    for bodies, k in problems:
        ds = DeviceSurface.from_bodies(bodies)
        kd = dev(k)
        y = torch.empty((len(k), 1, ds.n), dtype=torch.complex128, device="cuda")
        native.bem_incident(ctx, ds.struct, len(k), kd, (0.0, 0.0, 1.0), y)
        prepared.append((ds, kd, y, len(k)))

    def run(i, graph):
        ds, kd, y, nk = prepared[i]
        x = torch.zeros((nk, 1, ds.n), dtype=torch.complex128, device="cuda")
        opts = native.bem_solve_opts_default()
        opts.mode = mode
        opts.use_graph = 1 if graph else 0
        native.bem_solve_batched(ctx, [(ds.struct, nk, kd, 1, y)], opts, [x])
        return x.cpu().numpy()

    eager = [run(0, False), run(1, False)]
    for rep in range(3):
        t0 = time.perf_counter()
        a = run(0, True)
        t1 = time.perf_counter()
        b = run(1, False)                      # eager work between replays
        c = run(1, True)
        assert np.array_equal(a, eager[0]), f"replay {rep}, problem 0"
        assert np.array_equal(b, eager[1])
        assert np.array_equal(c, eager[1]), f"replay {rep}, problem 1"
    bodies, k = problems[0]
    s = Surface(bodies)
    for j, kq in enumerate(k):
        p, dp = bie.incident_plane_wave(s, kq)
        _, _, xs = bie.solve(s, kq, bie.known_data(s, p, dp))
        assert rel(a[j, 0], xs) < 1e-6
    print(f"\nlast graph replay solve: {1e3 * (t1 - t0):.2f} ms")


def test_solve_ir_fallback_forced(ctx):
    # max_iter = 1 cannot reach the step tolerance: every item falls back to FP64
    w = sphere_l2_workload()
    ds = DeviceSurface.from_bodies(w.bodies)
    k = w.k[:4]
    kd = dev(k)
    y = torch.empty((4, ds.n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, 4, kd, (0.0, 0.0, 1.0), y)
    x = torch.zeros((4, 1, ds.n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    opts.max_iter = 1
    info = native.bem_solve_batched(ctx, [(ds.struct, 4, kd, 1, y)], opts, [x])
    assert all(info[q].used_fp64 == 1 for q in range(4))
    opts.fallback = 0
    with pytest.raises(native.BemError) as e:
        native.bem_solve_batched(ctx, [(ds.struct, 4, kd, 1, y)], opts, [x])
    assert e.value.status == native.BEM_ENOCONV


def test_invalid_inputs_rejected(ctx):
    w = sphere_l2_workload()
    s = Surface(w.bodies)
    bad_n = s.nrm.copy()
    bad_n[5] *= 1.01
    ds = DeviceSurface(s.x, bad_n, s.w, s.bc)
    k = dev(np.array([1.0]))
    y = torch.zeros((1, 1, s.n), dtype=torch.complex128, device="cuda")
    A = torch.zeros((1, s.n, s.n), dtype=torch.complex64, device="cuda")
    b = torch.zeros((1, 1, s.n), dtype=torch.complex128, device="cuda")
    with pytest.raises(native.BemError) as e:
        native.bem_assemble(ctx, ds.struct, 1, k, 1, y, native.BEM_C64, A, s.n, b, None)
    assert e.value.status == native.BEM_EINVAL
    ds = DeviceSurface(s.x, s.nrm, s.w, s.bc)
    for kv in (0.0, -1.0, float("nan")):
        with pytest.raises(native.BemError) as e:
            native.bem_assemble(ctx, ds.struct, 1, dev(np.array([kv])), 1, y, native.BEM_C64, A,
                                s.n, b, None)
        assert e.value.status == native.BEM_EINVAL
    with pytest.raises(native.BemError):
        native.bem_assemble(ctx, ds.struct, 1, k, 1, y, native.BEM_C64, A, s.n - 1, b, None)


def test_empty_point_sets_are_no_ops(ctx):
    """Zero observation points: the field and both syntheses return at once
    and leave their outputs untouched (the index list of the sparse form is
    still checked)."""
    bodies = mixed_bodies(1)
    ds = DeviceSurface.from_bodies(bodies)
    k = dev(np.array([0.5, 1.0]))
    phi = torch.zeros((2, 1, ds.n), dtype=torch.complex128, device="cuda")
    xp = dev(np.zeros((1, 3)))
    i0 = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    ins = torch.full((1,), 5, dtype=torch.uint8, device="cuda")
    U = torch.full((1, 1, 2), 3.0, dtype=torch.complex64, device="cuda")
    native.bem_field_eval(ctx, ds.struct, 2, k, 1, phi, phi, 0, xp, i0, 0, ins,
                          native.BEM_C64, U)
    c = dev(np.ones((1, 2), dtype=np.complex128))
    p = torch.full((1, 1, 64), 2.0, dtype=torch.float32, device="cuda")
    native.pulse_synthesize(ctx, 0, 2, U[0], 1, c, 64, 0, xp, 0.1, p)
    native.pulse_synthesize_sparse(ctx, 0, np.array([3, 9], np.int32), U[0], 1, c, 64, 0, xp,
                                   0.1, p)
    with pytest.raises(native.BemError):
        native.pulse_synthesize_sparse(ctx, 0, np.array([9, 3], np.int32), U[0], 1, c, 64, 0,
                                       xp, 0.1, p)
    torch.cuda.synchronize()
    assert i0.item() == 7 and ins.item() == 5
    assert np.all(U.cpu().numpy() == 3.0) and np.all(p.cpu().numpy() == 2.0)


# ------------------------------------------------------------------ S7/S8
def _field_setup(ctx, bodies, k, xp):
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    n = s.n
    rng = np.random.default_rng(7)
    phi = seeded_complex(rng, (len(k), 1, n))
    psi = seeded_complex(rng, (len(k), 1, n))
    return s, ds, phi, psi


@pytest.mark.parametrize("prec", [native.BEM_C128, native.BEM_C64])
@pytest.mark.parametrize("kset", ["scattered", "grid"])
def test_field_eval_vs_oracle(ctx, prec, kset):
    bodies = [Body((0.0, 0.0, -1.3), 1.0, 1.0, 2, HARD), Body((0.0, 0.0, 1.3), 1.0, 1.0, 2, HARD)]
    if kset == "scattered":
        k = np.array([0.4, 3.3, 7.7, 11.9, 5.0, 2.2, 9.1, 1.1, 6.0, 10.5])   # ragged frequency tail
    else:   # evenly spaced (phase rotation in the float32 kernel), ragged last chunk
        k = 0.6 * np.arange(1, 20)
    rng = np.random.default_rng(11)
    xp = np.concatenate([rng.uniform(-4, 4, (300, 3)), ring_points(2.5, 16),
                         np.array([[0.0, 0.0, 0.0], [0.0, 0.0, -1.3 - 1.0005]])])
    s, ds, phi, psi = _field_setup(ctx, bodies, k, xp)
    xp = np.concatenate([xp, s.x[[3, 200]]])   # points on nodes
    m = xp.shape[0]
    cdt = torch.complex128 if prec == native.BEM_C128 else torch.complex64
    U = torch.zeros((1, m, len(k)), dtype=cdt, device="cuda")
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    native.bem_field_eval(ctx, ds.struct, len(k), dev(k), 1, dev(phi), dev(psi), m, dev(xp),
                          i0, 0, ins, prec, U)
    oi0 = ofield.closest_node(s.x, xp)
    assert np.array_equal(i0.cpu().numpy(), oi0)
    oins = ofield.inside_mask(s.x, s.nrm, xp, oi0)
    assert np.array_equal(ins.cpu().numpy(), oins)
    U = U.cpu().numpy()[0].astype(np.complex128)
    ref = np.stack([ofield.field(s, kq, phi[q, 0], psi[q, 0], xp, oi0)[0] for q, kq in enumerate(k)], axis=1)
    tol = 1e-11 if prec == native.BEM_C128 else 2e-6
    assert rel(U, ref) < tol, rel(U, ref)
    assert np.all(U[oins == 1] == 0)
    # given closest nodes: same result
    U2 = torch.zeros((1, m, len(k)), dtype=cdt, device="cuda")
    native.bem_field_eval(ctx, ds.struct, len(k), dev(k), 1, dev(phi), dev(psi), m, dev(xp),
                          i0, 1, ins, prec, U2)
    assert np.array_equal(U2.cpu().numpy()[0], U.astype(U2.cpu().numpy().dtype))


def test_closest_node_ties_on_symmetry_plane(ctx):
    bodies = [Body((0.0, 0.0, -1.4), 1.0, 1.0, 3, HARD), Body((0.0, 0.0, 1.4), 1.0, 1.0, 3, HARD)]
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    g = np.linspace(-3, 3, 61)
    yy, zz = np.meshgrid(g, g, indexing="ij")
    xp = np.stack([np.zeros(yy.size), yy.ravel(), zz.ravel()], axis=1)   # x = 0 plane, z = 0 ties
    m = xp.shape[0]
    k = np.array([1.0])
    phi = torch.zeros((1, 1, s.n), dtype=torch.complex128, device="cuda")
    U = torch.zeros((1, m, 1), dtype=torch.complex64, device="cuda")
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    native.bem_field_eval(ctx, ds.struct, 1, dev(k), 1, phi, phi, m, dev(xp), i0, 0, ins,
                          native.BEM_C64, U)
    assert np.array_equal(i0.cpu().numpy(), ofield.closest_node(s.x, xp))


# ------------------------------------------------------------------ S9
# transform lengths T/2 = 2^5 .. 2^11: radix-8 stages ending in a radix-8,
# radix-4 or radix-2 stage (T = 256 and 2048 end in radix 2)
@pytest.mark.parametrize("T,n_k,add", [(64, 32, 0), (128, 64, 1), (256, 100, 0), (512, 200, 1),
                                       (2048, 1024, 1), (4096, 2048, 0)])
def test_synthesis_vs_oracle(ctx, T, n_k, add):
    rng = np.random.default_rng(T)
    m = 37
    dk = 12.0 / n_k
    U = (seeded_complex(rng, (m, n_k)) / (1 + np.arange(n_k))[None, :] ** 0.5).astype(np.complex64)
    pulses = [Pulse("gauss", {"sigma": 0.8}), Pulse("chirp", {"ka": 3.0, "kb": 7.0, "D": 2.5})]
    c = np.stack([opulse.coefficients(p, n_k, dk, T, -5.0) for p in pulses])
    xp = rng.uniform(-5, 5, (m, 3))
    out = torch.zeros((2, m, T), dtype=torch.float32, device="cuda")
    native.pulse_synthesize(ctx, m, n_k, dev(U), 2, dev(c), T, add, dev(xp), dk, out)
    got = out.cpu().numpy()
    for q in range(2):
        ref = opulse.synthesize(U.astype(np.complex128), c[q], T, xp, dk, add_incident=bool(add))
        assert rel(got[q], ref) < 1e-5, rel(got[q], ref)


@pytest.mark.parametrize("T,idx,add", [
    (64, [1, 2, 5, 9, 31, 32], 0),                  # first bin and the Nyquist bin
    (128, [3, 8, 9, 10, 17, 40, 63], 1),
    (4096, list(range(5, 2048, 7)) + [2048], 1),    # 293 of 2048 bins, ragged
])
def test_sparse_synthesis_vs_oracle(ctx, T, idx, add):
    """Synthesis over a listed subset of the frequencies equals the oracle's
    inverse DFT with every other coefficient zero (Sec. IV, Table 1)."""
    rng = np.random.default_rng(T + len(idx))
    m, F = 29, T // 2
    idx = np.array(idx, dtype=np.int32)
    dk = 12.0 / F
    Us = (seeded_complex(rng, (m, len(idx))) / idx[None, :] ** 0.5).astype(np.complex64)
    pulses = [Pulse("gauss", {"sigma": 0.8}), Pulse("ricker", {"sigma": 1.1})]
    c = np.stack([opulse.coefficients(p, F, dk, T, -5.0) for p in pulses])
    cs = np.ascontiguousarray(c[:, idx - 1])
    xp = rng.uniform(-5, 5, (m, 3))
    out = torch.zeros((2, m, T), dtype=torch.float32, device="cuda")
    native.pulse_synthesize_sparse(ctx, m, idx, dev(Us), 2, dev(cs), T, add, dev(xp), dk, out)
    got = out.cpu().numpy()
    Ufull = np.zeros((m, F), dtype=np.complex128)
    Ufull[:, idx - 1] = Us
    for q in range(2):
        cz = np.zeros(F, dtype=np.complex128)
        cz[idx - 1] = c[q, idx - 1]
        ref = opulse.synthesize(Ufull, cz, T, xp, dk, add_incident=bool(add))
        assert rel(got[q], ref) < 1e-5, rel(got[q], ref)
    with pytest.raises(native.BemError):   # not increasing
        native.pulse_synthesize_sparse(ctx, m, idx[::-1].copy(), dev(Us), 2, dev(cs), T, add,
                                       dev(xp), dk, out)
    with pytest.raises(native.BemError):   # beyond T/2
        native.pulse_synthesize_sparse(ctx, m, np.array([1, F + 1], np.int32), dev(Us), 2,
                                       dev(cs), T, add, dev(xp), dk, out)


def scattered_field(ctx, ds, k, pts):
    """U[m][n_k] (c64) of the field scattered from e^{ikz} at pts, through the
    direct solve (refined FP32 factors) and the field kernel."""
    nk, n, m = len(k), ds.n, len(pts)
    kd = dev(np.asarray(k, dtype=np.float64))
    y = torch.empty((nk, 1, n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, nk, kd, (0.0, 0.0, 1.0), y)
    x = torch.zeros((nk, 1, n), dtype=torch.complex128, device="cuda")
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_B3
    info = native.bem_solve_batched(ctx, [(ds.struct, nk, kd, 1, y)], opts, [x])
    assert all(info[q].converged == 1 for q in range(nk))
    phi, psi = torch.empty_like(x), torch.empty_like(x)
    native.bem_split_unknowns(ctx, ds.struct, nk, 1, x, y, phi, psi)
    U = torch.zeros((1, m, nk), dtype=torch.complex64, device="cuda")
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    native.bem_field_eval(ctx, ds.struct, nk, kd, 1, phi, psi, m, dev(pts), i0, 0, ins,
                          native.BEM_C64, U)
    return U[0]


@pytest.mark.parametrize("level", [3, 4])
def test_dominant_frequency_truncation(ctx, level):
    """Sec. IV A, Table 1: the soft sphere under the paper's pulse (2 N_c = 4,
    alpha = 0.1, w = 20.1 a, 128 samples), its scattered wave at z = -1.1 a and
    -4 a rebuilt from only the 5, 10 and 20 frequencies of largest |c_m|, each
    solved on its own.  (i) The truncated wave matches the oracle's (FP64 BEM
    at the same frequencies) to 1e-5; (ii) the sparse synthesis of the n
    solved frequencies equals the full-grid synthesis with the other
    coefficients zero; (iii) the % RMS errors reproduce the printed table."""
    import json
    import os
    from workloads import paper_sphere_pulse
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    W, T, F = 20.1, 128, 63
    dk = 2 * np.pi / W
    c = native.bem_pulse_coeffs("paper", [2.0, 0.1, W], dk, F, T, -(1.0 + W / 4))
    pts = np.array([[0.0, 0.0, -1.1], [0.0, 0.0, -4.0]])
    bodies = [Body((0.0, 0.0, 0.0), 1.0, 1.0, level, SOFT)]
    ds = DeviceSurface.from_bodies(bodies)
    s = Surface(bodies)
    xp = dev(pts)
    Ufull = scattered_field(ctx, ds, dk * np.arange(1, F + 1), pts)
    full = torch.zeros((1, 2, T), dtype=torch.float32, device="cuda")
    native.pulse_synthesize(ctx, 2, F, Ufull, 1, dev(c[None, :]), T, 0, xp, dk, full)
    full = full.cpu().numpy()[0]
    for n, e11, e4 in zip(gold["n_terms"], gold["rms_percent_at_z_minus_1p1"],
                          gold["rms_percent_at_z_minus_4"]):
        idx = native.bem_pulse_dominant(c, n)
        assert np.array_equal(idx, opulse.dominant(c, n) + 1)
        Us = scattered_field(ctx, ds, dk * idx, pts)
        cs = dev(np.ascontiguousarray(c[idx - 1])[None, :])
        tr = torch.zeros((1, 2, T), dtype=torch.float32, device="cuda")
        native.pulse_synthesize_sparse(ctx, 2, idx, Us, 1, cs, T, 0, xp, dk, tr)
        tr = tr.cpu().numpy()[0]
        # (ii) same as zeroing the other coefficients of the full grid
        cz = np.zeros_like(c)
        cz[idx - 1] = c[idx - 1]
        zf = torch.zeros((1, 2, T), dtype=torch.float32, device="cuda")
        native.pulse_synthesize(ctx, 2, F, Ufull, 1, dev(cz[None, :]), T, 0, xp, dk, zf)
        assert rel(tr, zf.cpu().numpy()[0]) < 1e-5
        if level == 3:
            # (i) oracle: FP64 BEM at the selected frequencies only
            Uo = np.zeros((2, F), dtype=np.complex128)
            for mm in idx:
                phi, psi = bie.scatter_plane_wave(s, dk * mm)
                Uo[:, mm - 1] = ofield.field(s, dk * mm, phi, psi, pts)[0]
            ref = opulse.synthesize(Uo, cz, T)
            assert rel(tr, ref) < 1e-5, rel(tr, ref)
        # (iii) Table 1 within the printed precision
        tol = gold["printed_precision"] + 1e-9
        assert abs(opulse.rms_error_percent(tr[0], full[0]) - e11) <= tol
        assert abs(opulse.rms_error_percent(tr[1], full[1]) - e4) <= tol


@pytest.mark.parametrize("levels,nk", [((3, 3), 70), ((4, 3), 9), ((4, 4), 5)])
def test_residual_sweep_on_even_grid(ctx, levels, nk):
    """Refinement residuals on an even wavenumber grid (phases carried across
    the grid, r = b - A x; 70 wavenumbers re-anchor past 64 and end on a ragged
    chunk; rows are split into parts of 1536 columns: 1284, 3204 and 5124
    nodes take 1, 3 and 4 parts) converge to the same
    solutions as the same wavenumbers in scattered order (one sincos per pair
    and wavenumber), and to the FP64 oracle."""
    bodies = [Body((0.0, 0.0, -1.6), 1.0, 1.0, levels[0], HARD),
              Body((0.2, 0.0, 1.7), 0.9, 1.0, levels[1], SOFT)]
    ds = DeviceSurface.from_bodies(bodies)
    n = ds.n
    assert n >= 1024
    k = 0.3 + 0.11 * np.arange(nk)
    perm = np.random.default_rng(nk).permutation(nk)
    out = []
    for kk in (k, k[perm]):
        kd = dev(kk)
        y = torch.empty((nk, 1, n), dtype=torch.complex128, device="cuda")
        native.bem_incident(ctx, ds.struct, nk, kd, (0.0, 0.0, 1.0), y)
        x = torch.zeros((nk, 1, n), dtype=torch.complex128, device="cuda")
        info = native.bem_solve_batched(ctx, [(ds.struct, nk, kd, 1, y)],
                                        native.bem_solve_opts_default(), [x])
        for q in range(nk):
            assert info[q].converged == 1 and info[q].used_fp64 == 0 and info[q].rel_resid < 1e-9
        out.append(x.cpu().numpy()[:, 0])
    even, scattered = out[0], np.empty_like(out[1])
    scattered[perm] = out[1]
    for q in range(nk):
        assert rel(even[q], scattered[q]) < 1e-8
    s = Surface(bodies)
    q = nk // 2
    p, dp = bie.incident_plane_wave(s, k[q])
    _, _, xs = bie.solve(s, k[q], bie.known_data(s, p, dp))
    assert rel(even[q], xs) < 1e-8


def test_phase_sincos_accuracy_through_incident_wave(ctx):
    """The phases e^{i theta} of the operator kernels (reduction by pi/2 and
    Taylor series) agree with the libm sine and cosine to 2 ulp for theta up to
    about 3000: a soft surface under a plane wave along z has y_j = -e^{i k z_j}
    with theta = k * z_j a single rounded product, reproduced here exactly."""
    bodies = [Body((0.0, 0.0, 0.0), 1.0, 1.0, 2, SOFT), Body((0.0, 0.0, 2.6), 0.5, 1.0, 1, SOFT)]
    ds = DeviceSurface.from_bodies(bodies)
    s = Surface(bodies)
    k = np.array([0.37, 11.0, 97.5, 512.25, 1000.0 + 1.0 / 3.0])
    kd = dev(k)
    y = torch.empty((k.size, 1, ds.n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, k.size, kd, (0.0, 0.0, 1.0), y)
    got = y.cpu().numpy()[:, 0]
    z = s.x[:, 2]
    for q in range(k.size):
        theta = k[q] * z
        assert np.max(np.abs(got[q].real + np.cos(theta))) <= 2.3e-16
        assert np.max(np.abs(got[q].imag + np.sin(theta))) <= 2.3e-16
