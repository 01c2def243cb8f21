"""The no-allocation field evaluation (bem_field_eval_noalloc, node sums in
the library's fixed per-device scratch) against bem_field_eval, through the C
ABI: two calls in a row, the second smaller, in both precisions; results equal
bit for bit (same kernels, same arithmetic).  Sizes beyond the fixed scratch
are rejected on the host."""
import numpy as np
import pytest

from workloads import Body, HARD, seeded_complex

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_1706_07919_amd.native")
from paper_1706_07919_amd import DeviceSurface  # noqa: E402


def _eval(fn, ctx, ds, k, phi, psi, pts, prec):
    nk, nr = phi.shape[0], phi.shape[1]
    m = pts.shape[0]
    cdt = torch.complex128 if prec == native.BEM_C128 else torch.complex64
    U = torch.full((nr, m, nk), 7.0, dtype=cdt, device="cuda")
    i0 = torch.zeros(m, dtype=torch.int32, device="cuda")
    ins = torch.zeros(m, dtype=torch.uint8, device="cuda")
    fn(ctx, ds.struct, nk, torch.as_tensor(k).cuda(), nr, torch.as_tensor(phi).cuda(),
       torch.as_tensor(psi).cuda(), m, torch.as_tensor(pts).cuda(), i0, 0, ins, prec, U)
    torch.cuda.synchronize()
    return U.cpu().numpy(), i0.cpu().numpy(), ins.cpu().numpy()


@pytest.mark.parametrize("prec", [native.BEM_C64, native.BEM_C128])
def test_field_eval_noalloc_matches_field_eval(prec):
    assert torch.cuda.is_available()
    ctx = native.Context(0)
    try:
        bodies = [Body((0.0, 0.0, -1.3), 1.0, 1.0, 2, HARD), Body((0.0, 0.0, 1.3), 1.0, 1.0, 2, HARD)]
        ds = DeviceSurface.from_bodies(bodies)
        rng = np.random.default_rng(17)
        cases = [(0.4 * np.arange(1, 22), 3, 700),     # larger call first
                 (np.array([0.9, 5.5, 7.25]), 1, 33)]  # then a smaller one
        for k, nr, m in cases:
            phi = seeded_complex(rng, (len(k), nr, ds.n))
            psi = seeded_complex(rng, (len(k), nr, ds.n))
            pts = rng.uniform(-4, 4, (m, 3))
            ref = _eval(native.bem_field_eval, ctx, ds, k, phi, psi, pts, prec)
            got = _eval(native.bem_field_eval_noalloc, ctx, ds, k, phi, psi, pts, prec)
            assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
            assert np.array_equal(got[0].view(np.uint8), ref[0].view(np.uint8))
            assert np.isfinite(got[0]).all() and np.abs(got[0]).max() > 0
        # scratch beyond the fixed 32 MiB: rejected on the host before any
        # launch (c128: the node sums of many frequencies; c64: the grouping of
        # many points, whose arrays are never read)
        if prec == native.BEM_C128:
            nk_big, m_big = (32 << 20) // (ds.n * 16) + 1, 4
        else:
            nk_big, m_big = 4, 8_000_000
        k = np.linspace(0.1, 6.0, nk_big)
        z = torch.zeros((nk_big, 1, ds.n), dtype=torch.complex128, device="cuda")
        U = torch.zeros((1, 4, nk_big), dtype=torch.complex128 if prec == native.BEM_C128
                        else torch.complex64, device="cuda")
        i0 = torch.zeros(4, dtype=torch.int32, device="cuda")
        ins = torch.zeros(4, dtype=torch.uint8, device="cuda")
        with pytest.raises(native.BemError, match="fixed scratch"):
            native.bem_field_eval_noalloc(ctx, ds.struct, nk_big, torch.as_tensor(k).cuda(), 1, z,
                                          z, m_big, torch.zeros((4, 3), dtype=torch.float64,
                                                                device="cuda"), i0, 0, ins, prec, U)
    finally:
        ctx.close()
