"""Frequency surrogate: a Fourier-featured network k -> surface unknowns of a
fixed geometry, trained on direct solutions and used to fill a dense frequency
grid.  Every prediction is judged by the float64 residual of the discrete
equation; wavenumbers that fail are refined with the stored float32 factors of
the nearest training wavenumber (starting from the prediction), and whatever
still does not converge is solved directly.

This module only sequences library calls; all arithmetic (features, dense
layers, loss, gradients, Adam, packing, residuals, factorisations, solves)
runs in the HIP kernels behind include/bem.h.
"""
from __future__ import annotations

import time

import numpy as np

from . import native


class Surrogate:
    def __init__(self, ctx, n_nodes, init_weights, n_oct=8, kscale=12.0, device="cuda"):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.n = n_nodes
        self.n_oct = n_oct
        self.kscale = kscale
        self.dev = device
        self.sizes = [init_weights[0][0].shape[0]] + [W.shape[1] for W, _ in init_weights]
        assert self.sizes[0] == 2 * n_oct and self.sizes[-1] == 2 * n_nodes
        self.W = [torch.as_tensor(W).to(device).contiguous() for W, _ in init_weights]
        self.b = [torch.as_tensor(b).to(device).contiguous() for _, b in init_weights]
        self.dW = [torch.zeros_like(W) for W in self.W]
        self.db = [torch.zeros_like(b) for b in self.b]
        self.mW = [torch.zeros_like(W) for W in self.W]
        self.vW = [torch.zeros_like(W) for W in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.scale = torch.ones(n_nodes, dtype=torch.float64, device=device)
        self.step_count = 0

    # -------------------------------------------------------------- passes
    def _buffers(self, B):
        t = self.torch
        hs = [t.empty((B, self.sizes[0]), dtype=t.float32, device=self.dev)]
        zs = []
        for o in self.sizes[1:]:
            zs.append(t.empty((B, o), dtype=t.float32, device=self.dev))
            hs.append(t.empty((B, o), dtype=t.float32, device=self.dev))
        return hs, zs

    def forward(self, kd, B, bufs=None):
        hs, zs = bufs if bufs is not None else self._buffers(B)
        native.bem_mlp_features(self.ctx, B, kd, self.n_oct, self.kscale, hs[0])
        L = len(self.W)
        for i in range(L):
            act = 1 if i < L - 1 else 0
            native.bem_mlp_dense_fwd(self.ctx, B, self.sizes[i], self.sizes[i + 1], hs[i], self.W[i],
                                     self.b[i], act, zs[i], hs[i + 1])
        return hs, zs

    def backward(self, B, hs, zs, dy):
        t = self.torch
        L = len(self.W)
        g = dy
        for i in range(L - 1, -1, -1):
            act = 1 if i < L - 1 else 0
            dx = t.empty((B, self.sizes[i]), dtype=t.float32, device=self.dev) if i > 0 else None
            dz = t.empty_like(zs[i]) if act else None
            native.bem_mlp_dense_bwd(self.ctx, B, self.sizes[i], self.sizes[i + 1], hs[i], self.W[i],
                                     zs[i], act, g, self.dW[i], self.db[i], dx, dz)
            g = dx

    def adam(self, lr):
        self.step_count += 1
        for i in range(len(self.W)):
            native.bem_mlp_adam(self.ctx, self.W[i].numel(), self.W[i], self.dW[i], self.mW[i],
                                self.vW[i], self.step_count, lr)
            native.bem_mlp_adam(self.ctx, self.b[i].numel(), self.b[i], self.db[i], self.mb[i],
                                self.vb[i], self.step_count, lr)

    # -------------------------------------------------------------- training
    def fit(self, kd, x_train, epochs=2000, lr=1e-3, lr_final=1e-5, log_every=0):
        """Full-batch training on x_train (c128 [B][n] unknowns at wavenumbers kd);
        cosine learning-rate decay from lr to lr_final."""
        t = self.torch
        B = int(kd.shape[0])
        target = t.empty((B, 2 * self.n), dtype=t.float32, device=self.dev)
        native.bem_mlp_pack(self.ctx, B, self.n, x_train, self.scale, 1, target)
        bufs = self._buffers(B)
        dy = t.empty((B, 2 * self.n), dtype=t.float32, device=self.dev)
        nparts = 64
        part = t.zeros(nparts, dtype=t.float64, device=self.dev)
        hist = []
        for ep in range(epochs):
            hs, zs = self.forward(kd, B, bufs)
            native.bem_mlp_mse_grad(self.ctx, B * 2 * self.n, hs[-1], target, dy, part, nparts)
            self.backward(B, hs, zs, dy)
            a = 0.5 * (1 + np.cos(np.pi * ep / max(epochs - 1, 1)))
            self.adam(lr_final + (lr - lr_final) * a)
            if log_every and (ep % log_every == 0 or ep == epochs - 1):
                hist.append((ep, float(part.sum().item()) / (B * 2 * self.n)))
        return hist

    def predict(self, kd):
        t = self.torch
        B = int(kd.shape[0])
        hs, _ = self.forward(kd, B)
        x = t.empty((B, self.n), dtype=t.complex128, device=self.dev)
        native.bem_mlp_unpack(self.ctx, B, self.n, hs[-1], self.scale, x)
        return x


def octaves_for(k_train, kscale=12.0):
    """Number of Fourier octaves such that the highest feature frequency,
    2^(L-1) pi / kscale, stays at a quarter of the training grid's Nyquist
    rate pi / dk (higher octaves alias between training wavenumbers)."""
    dk = float(np.min(np.diff(np.sort(np.asarray(k_train)))))
    return max(1, int(np.floor(np.log2(kscale / (4.0 * dk)))) + 1)


def nearest_index(k_pred, k_train):
    """Index of the nearest training wavenumber (host-side selection only)."""
    return np.abs(np.asarray(k_pred)[:, None] - np.asarray(k_train)[None, :]).argmin(axis=1).astype(np.int32)


def training_factors(ctx, ds, kd, y, nb=0, gemm_kind=None):
    """Float32 factors of the training wavenumbers (kept for re-use) and the
    FP64-accurate training solutions obtained by refining with them."""
    if gemm_kind is None:
        gemm_kind = native.BEM_GEMM_3M
    t = __import__("torch")
    n = ds.n
    nk = int(kd.shape[0])
    ld = (n + 15) // 16 * 16
    LU = t.empty((nk, n, ld), dtype=t.complex64, device=y.device)
    b = t.empty((nk, 1, n), dtype=t.complex128, device=y.device)
    native.bem_assemble(ctx, ds.struct, nk, kd, 1, y, native.BEM_C64, LU, ld, b, None)
    piv = t.empty((nk, n), dtype=t.int32, device=y.device)
    info = t.empty(nk, dtype=t.int32, device=y.device)
    native.bem_getrf_batched(ctx, native.BEM_C64, n, ld, n * ld, nk, LU, piv, info, nb, gemm_kind)
    x = t.zeros((nk, 1, n), dtype=t.complex128, device=y.device)
    fidx = t.arange(nk, dtype=t.int32, device=y.device)
    inf = native.bem_refine_batched(ctx, ds.struct, nk, kd, 1, y, LU, ld, n * ld, piv, nk, fidx,
                                    1e-10, 20, x)
    return LU, piv, ld, x, inf


def fill_sweep(ctx, ds, k_train, k_pred, hidden=(512, 512, 512, 512), seed=0, epochs=2000,
               lr=1e-3, tol=1e-6, refine_tol=1e-8, max_sweeps=60, n_oct=None, kscale=12.0,
               use_surrogate=True):
    """Solve a dense grid k_pred from the factors and solutions at k_train.

    Returns a dict with the solutions (c128 [n_kp][1][n]), per-stage timings,
    acceptance counts and sweep statistics."""
    import torch
    from workloads import mlp_initial_weights
    if n_oct is None:
        n_oct = octaves_for(k_train, kscale)
    dev = ds.x.device
    n = ds.n
    out = {}
    kt = torch.as_tensor(np.asarray(k_train, np.float64)).to(dev)
    kp = torch.as_tensor(np.asarray(k_pred, np.float64)).to(dev)
    nkt, nkp = len(k_train), len(k_pred)
    yt = torch.empty((nkt, 1, n), dtype=torch.complex128, device=dev)
    yp = torch.empty((nkp, 1, n), dtype=torch.complex128, device=dev)
    native.bem_incident(ctx, ds.struct, nkt, kt, (0.0, 0.0, 1.0), yt)
    native.bem_incident(ctx, ds.struct, nkp, kp, (0.0, 0.0, 1.0), yp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    LU, piv, ld, xt, _ = training_factors(ctx, ds, kt, yt)
    torch.cuda.synchronize()
    out["t_train_solves"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    out["n_oct"] = n_oct
    if use_surrogate:
        init_weights = mlp_initial_weights([2 * n_oct, *hidden, 2 * n], seed)
        sur = Surrogate(ctx, n, init_weights, n_oct, kscale, device=dev)
        out["loss"] = sur.fit(kt, xt[:, 0], epochs=epochs, lr=lr, log_every=max(epochs // 10, 1))
        torch.cuda.synchronize()
        out["t_fit"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        x = sur.predict(kp).reshape(nkp, 1, n).contiguous()
    else:
        out["t_fit"] = 0.0
        x = torch.zeros((nkp, 1, n), dtype=torch.complex128, device=dev)
    rel = native.bem_residual_check(ctx, ds.struct, nkp, kp, 1, yp, x)
    out["rel_resid_prediction"] = rel
    accept = rel <= tol
    out["accepted_as_predicted"] = int(accept.sum())
    todo = np.flatnonzero(~accept)
    sweeps = np.zeros(nkp, np.int32)
    fallback = np.zeros(0, np.int64)
    if todo.size:
        near = nearest_index(np.asarray(k_pred)[todo], k_train)
        sub = x[todo].contiguous()
        info = native.bem_refine_batched(ctx, ds.struct, len(todo), kp[todo].contiguous(), 1,
                                         yp[todo].contiguous(), LU, ld, n * ld, piv, nkt,
                                         torch.as_tensor(near).to(dev), refine_tol, max_sweeps, sub)
        conv = np.array([info[q].converged for q in range(len(todo))], bool)
        relr = np.array([info[q].rel_resid for q in range(len(todo))])
        sweeps[todo] = [info[q].iters for q in range(len(todo))]
        ok = conv & (relr <= tol)
        x[todo] = sub
        fallback = todo[~ok]
    out["refined"] = int(todo.size - fallback.size)
    out["fallback"] = int(fallback.size)
    if fallback.size:
        xf = torch.zeros((fallback.size, 1, n), dtype=torch.complex128, device=dev)
        opts = native.bem_solve_opts_default()
        opts.mode = native.BEM_FP32_IR_3M
        native.bem_solve_batched(ctx, [(ds.struct, int(fallback.size), kp[fallback].contiguous(), 1,
                                        yp[fallback].contiguous())], opts, [xf])
        x[fallback] = xf
    torch.cuda.synchronize()
    out["t_fill"] = time.perf_counter() - t0
    out["sweeps_mean"] = float(sweeps[todo].mean()) if todo.size else 0.0
    out["sweeps_max"] = int(sweeps.max()) if nkp else 0
    out["x"] = x
    out["y"] = yp
    out["k"] = kp
    del LU
    return out
