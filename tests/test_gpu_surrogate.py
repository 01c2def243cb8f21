"""GPU parity of the surrogate kernels (features, dense forward/backward, loss
gradient, Adam, packing) against the FP64 reference network, and the
surrogate-filled sweep against direct solves (with the gain it brings)."""
import numpy as np
import pytest

from oracle import bie, mlp as omlp
from oracle.mesh import Surface
from workloads import Body, HARD, mlp_initial_weights

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_1706_07919_amd.native")
from paper_1706_07919_amd import DeviceSurface  # noqa: E402
from paper_1706_07919_amd import surrogate as sg  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = native.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    a = np.asarray(a)
    a = a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_features(ctx):
    k = np.linspace(0.01, 12, 77)
    x = torch.empty((77, 16), dtype=torch.float32, device="cuda")
    native.bem_mlp_features(ctx, 77, dev(k), 8, 12.0, x)
    assert np.max(np.abs(x.cpu().numpy() - omlp.features(k, 8, 12.0))) < 1e-6


@pytest.mark.parametrize("act", [0, 1])
@pytest.mark.parametrize("B,nin,nout", [(37, 20, 70), (256, 16, 512), (5, 512, 130)])
def test_dense_layer_vs_reference(ctx, act, B, nin, nout):
    rng = np.random.default_rng(B + nin)
    x = rng.standard_normal((B, nin)).astype(np.float32)
    W = (rng.standard_normal((nin, nout)) / np.sqrt(nin)).astype(np.float32)
    b = rng.standard_normal(nout).astype(np.float32)
    dy = rng.standard_normal((B, nout)).astype(np.float32)
    z = torch.empty((B, nout), dtype=torch.float32, device="cuda")
    y = torch.empty((B, nout), dtype=torch.float32, device="cuda")
    native.bem_mlp_dense_fwd(ctx, B, nin, nout, dev(x), dev(W), dev(b), act, z, y)
    x64, W64 = x.astype(np.float64), W.astype(np.float64)
    zr = x64 @ W64 + b
    yr = omlp.silu(zr) if act else zr
    assert rel(y.cpu().numpy(), yr) < 1e-5
    dW = torch.empty((nin, nout), dtype=torch.float32, device="cuda")
    db = torch.empty(nout, dtype=torch.float32, device="cuda")
    dx = torch.empty((B, nin), dtype=torch.float32, device="cuda")
    dz = torch.empty((B, nout), dtype=torch.float32, device="cuda")
    native.bem_mlp_dense_bwd(ctx, B, nin, nout, dev(x), dev(W), z if act else None, act, dev(dy),
                             dW, db, dx, dz if act else None)
    g = dy.astype(np.float64) * (omlp.silu_grad(zr) if act else 1.0)
    assert rel(dW.cpu().numpy(), x64.T @ g) < 1e-5
    assert rel(db.cpu().numpy(), g.sum(0)) < 1e-5
    assert rel(dx.cpu().numpy(), g @ W64.T) < 1e-5


def test_network_gradients_and_adam_steps_vs_reference(ctx):
    n_nodes = 40
    sizes = [16, 64, 64, 2 * n_nodes]
    init = mlp_initial_weights(sizes, seed=3)
    rng = np.random.default_rng(1)
    k = np.sort(rng.uniform(0.1, 12, 48))
    xt = rng.standard_normal((48, n_nodes)) + 1j * rng.standard_normal((48, n_nodes))
    sur = sg.Surrogate(ctx, n_nodes, init, n_oct=8, kscale=12.0)
    kd = dev(k)
    target = torch.empty((48, 2 * n_nodes), dtype=torch.float32, device="cuda")
    native.bem_mlp_pack(ctx, 48, n_nodes, dev(xt), sur.scale, 1, target)
    s = np.sqrt(np.mean(np.abs(xt) ** 2, axis=0))
    tref = np.stack([xt.real / s, xt.imag / s], axis=2).reshape(48, -1)
    assert rel(target.cpu().numpy(), tref) < 1e-6
    params = [[W.astype(np.float64), b.astype(np.float64)] for W, b in init]
    st = None
    dy = torch.empty((48, 2 * n_nodes), dtype=torch.float32, device="cuda")
    part = torch.zeros(8, dtype=torch.float64, device="cuda")
    for step in range(1, 4):
        hs, zs = sur.forward(kd, 48)
        native.bem_mlp_mse_grad(ctx, 48 * 2 * n_nodes, hs[-1], target, dy, part, 8)
        sur.backward(48, hs, zs, dy)
        yref, cache = omlp.forward(params, omlp.features(k, 8, 12.0))
        assert rel(hs[-1].cpu().numpy(), yref) < 1e-4
        loss = part.sum().item() / (48 * 2 * n_nodes)
        assert abs(loss - omlp.mse(yref, tref)) < 1e-4 * omlp.mse(yref, tref)
        grads = omlp.backward(params, cache, yref, tref)
        for i in range(len(params)):
            assert rel(sur.dW[i].cpu().numpy(), grads[i][0]) < 1e-4
            assert rel(sur.db[i].cpu().numpy(), grads[i][1]) < 1e-4
        sur.adam(1e-3)
        st = omlp.adam_step(params, grads, st, step, lr=1e-3)
        for i in range(len(params)):
            assert rel(sur.W[i].cpu().numpy(), params[i][0]) < 1e-5


def test_pack_unpack_roundtrip(ctx):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((9, 33)) + 1j * rng.standard_normal((9, 33))
    sc = torch.empty(33, dtype=torch.float64, device="cuda")
    t = torch.empty((9, 66), dtype=torch.float32, device="cuda")
    native.bem_mlp_pack(ctx, 9, 33, dev(x), sc, 1, t)
    back = torch.empty((9, 33), dtype=torch.complex128, device="cuda")
    native.bem_mlp_unpack(ctx, 9, 33, t, sc, back)
    assert rel(back.cpu().numpy(), x) < 1e-7


def _sphere():
    return [Body((0.0, 0.0, 0.0), 1.0, 1.0, 2, HARD)]


def test_refine_with_own_and_neighbour_factors(ctx):
    bodies = _sphere()
    s = Surface(bodies)
    ds = DeviceSurface.from_bodies(bodies)
    kt = np.array([1.0, 2.0, 3.0, 4.0])
    kd = dev(kt)
    y = torch.empty((4, 1, ds.n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, 4, kd, (0.0, 0.0, 1.0), y)
    LU, piv, ld, xt, info = sg.training_factors(ctx, ds, kd, y)
    for q in range(4):
        p, dp = bie.incident_plane_wave(s, kt[q])
        _, _, xs = bie.solve(s, kt[q], bie.known_data(s, p, dp))
        assert rel(xt[q, 0].cpu().numpy(), xs) < 1e-7
    # neighbouring wavenumbers refined with the factors of the nearest training k
    kp = np.array([1.04, 2.97, 3.08])
    kpd = dev(kp)
    yp = torch.empty((3, 1, ds.n), dtype=torch.complex128, device="cuda")
    native.bem_incident(ctx, ds.struct, 3, kpd, (0.0, 0.0, 1.0), yp)
    x = torch.zeros((3, 1, ds.n), dtype=torch.complex128, device="cuda")
    fi = dev(np.array([0, 2, 2], np.int32))
    inf = native.bem_refine_batched(ctx, ds.struct, 3, kpd, 1, yp, LU, ld, ds.n * ld, piv, 4, fi,
                                    1e-9, 80, x)
    for q in range(3):
        assert inf[q].converged == 1 and inf[q].rel_resid < 1e-8
        p, dp = bie.incident_plane_wave(s, kp[q])
        _, _, xs = bie.solve(s, kp[q], bie.known_data(s, p, dp))
        assert rel(x[q, 0].cpu().numpy(), xs) < 1e-6


def test_surrogate_fill_sweep_gain(ctx):
    """Dense grid from 32 training solves: every result satisfies the residual
    tolerance and matches the direct solve; starting the refinement from the
    network's prediction needs fewer sweeps than starting from zero."""
    bodies = _sphere()
    ds = DeviceSurface.from_bodies(bodies)
    k_train = 6.0 * (np.arange(1, 33) - 0.5) / 32
    k_pred = 6.0 * np.arange(1, 129) / 128
    res = sg.fill_sweep(ctx, ds, k_train, k_pred, hidden=(128, 128), epochs=3000, lr=2e-3,
                        tol=1e-6, refine_tol=1e-9, max_sweeps=80)
    base = sg.fill_sweep(ctx, ds, k_train, k_pred, use_surrogate=False, tol=1e-6,
                         refine_tol=1e-9, max_sweeps=80)
    assert res["n_oct"] == 5
    # direct reference for the whole grid
    kp = dev(k_pred)
    x_dir = torch.zeros((128, 1, ds.n), dtype=torch.complex128, device="cuda")
    native.bem_solve_batched(ctx, [(ds.struct, 128, kp, 1, res["y"])],
                             native.bem_solve_opts_default(), [x_dir])
    for r in (res, base):
        rr = native.bem_residual_check(ctx, ds.struct, 128, kp, 1, r["y"], r["x"])
        assert rr.max() < 1e-6
        err = (torch.linalg.vector_norm(r["x"] - x_dir, dim=(1, 2)) /
               torch.linalg.vector_norm(x_dir, dim=(1, 2))).max().item()
        assert err < 1e-6
    # the filled results against the oracle's direct FP64 solve at three
    # sampled wavenumbers of the dense grid
    s = Surface(bodies)
    for q in (9, 64, 127):
        p, dp = bie.incident_plane_wave(s, k_pred[q])
        _, _, xs = bie.solve(s, k_pred[q], bie.known_data(s, p, dp))
        for r in (res, base):
            assert rel(r["x"][q, 0].cpu().numpy(), xs) < 1e-6
    # the trained network's prediction is a far better start than zero
    assert np.median(res["rel_resid_prediction"]) < 0.05
    assert res["sweeps_mean"] < base["sweeps_mean"]
    assert res["fallback"] <= base["fallback"]
    print(f"\nsurrogate start: mean sweeps {res['sweeps_mean']:.2f} vs zero start "
          f"{base['sweeps_mean']:.2f}; fallbacks {res['fallback']} vs {base['fallback']}; "
          f"median prediction residual {np.median(res['rel_resid_prediction']):.2e}")
