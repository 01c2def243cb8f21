"""ctypes binding of ``libbem.so`` (include/bem.h): the same entry points, with
argument marshalling only.  Device buffers are torch tensors on the context's
device; every computation runs in the library's HIP kernels.

Loading fails loudly when the library has not been built: there is no fallback
implementation in this package.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbem.so")

BEM_OK, BEM_EINVAL, BEM_ENOMEM, BEM_EHIP, BEM_ESINGULAR, BEM_ENOCONV, BEM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
BEM_C64, BEM_C128 = 0, 1
BEM_BC_HARD, BEM_BC_SOFT = 0, 1
BEM_FP64_DIRECT, BEM_FP32_IR_4M, BEM_FP32_IR_3M, BEM_FP32_IR_B3 = 0, 1, 2, 3
BEM_GEMM_4M, BEM_GEMM_3M, BEM_GEMM_BF16X3, BEM_GEMM_BF16X3_UNPACKED = 0, 1, 2, 3
PULSE_KINDS = {"paper": 0, "gauss": 1, "ricker": 2, "nwave": 3, "chirp": 4, "gsine": 5, "gaussk": 6}

EXPORTED = [
    "bem_ctx_create", "bem_ctx_destroy", "bem_last_error", "bem_ctx_set_workspace_limit",
    "bem_ctx_set_profiling", "bem_ctx_set_profiling_filter", "bem_ctx_kernel_stats",
    "bem_mesh_counts", "bem_mesh_icosphere", "bem_mesh_bowl_counts", "bem_mesh_bowl", "bem_incident", "bem_assemble", "bem_residual",
    "bem_solve_opts_default", "bem_solve_batched", "bem_getrf_batched", "bem_getrs_batched",
    "bem_autotune_lu", "bem_autotune_lu_results", "bem_lu_tuned_plan", "bem_lu_set_plan",
    "bem_split_unknowns", "bem_field_eval", "bem_field_eval_noalloc", "pulse_synthesize",
    "pulse_synthesize_sparse",
    "bem_pulse_coeffs", "bem_pulse_dominant",
    "bem_residual_check", "bem_refine_batched", "bem_mlp_features", "bem_mlp_dense_fwd", "bem_mlp_dense_bwd",
    "bem_mlp_mse_grad", "bem_mlp_adam", "bem_mlp_pack", "bem_mlp_unpack",
    "bem_mesh_quadratic_counts", "bem_mesh_quadratic", "bem_assemble_quadratic",
    "bem_solve_quadratic", "bem_field_eval_quadratic", "bem_solve_chief",
]


class BemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bem status {status}: {msg}")
        self.status = status


class bem_surface(C.Structure):
    _fields_ = [("n", C.c_int32), ("x", C.c_void_p), ("nrm", C.c_void_p), ("w", C.c_void_p),
                ("bc", C.c_void_p)]


class bem_quad_surface(C.Structure):
    _fields_ = [("n", C.c_int32), ("x", C.c_void_p), ("nrm", C.c_void_p), ("bc", C.c_void_p),
                ("n_elem", C.c_int32), ("elem", C.c_void_p)]


class bem_problem(C.Structure):
    _fields_ = [("s", C.POINTER(bem_surface)), ("n_k", C.c_int32), ("k", C.c_void_p),
                ("n_rhs", C.c_int32), ("y", C.c_void_p)]


class bem_solve_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("tol_step", C.c_double), ("max_iter", C.c_int32),
                ("fallback", C.c_int32), ("use_graph", C.c_int32), ("nb", C.c_int32)]


class bem_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("used_fp64", C.c_int32), ("singular", C.c_int32),
                ("converged", C.c_int32), ("rel_resid", C.c_double), ("rel_step", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or python -m paper_1706_07919_amd.build)")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "bem_ctx_create": ([C.c_int, vp, C.POINTER(vp)], C.c_int),
        "bem_ctx_destroy": ([vp], None),
        "bem_last_error": ([vp], C.c_char_p),
        "bem_ctx_set_workspace_limit": ([vp, C.c_uint64], C.c_int),
        "bem_ctx_set_profiling": ([vp, i32], C.c_int),
        "bem_ctx_set_profiling_filter": ([vp, C.c_char_p], C.c_int),
        "bem_ctx_kernel_stats": ([vp, C.c_char_p, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl),
                                  C.POINTER(i64)], C.c_int),
        "bem_mesh_counts": ([i32, C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "bem_mesh_icosphere": ([i32, dbl, dbl, vp, i32, vp, vp, vp, vp], C.c_int),
        "bem_mesh_bowl_counts": ([i32, i32, C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "bem_mesh_bowl": ([i32, i32, dbl, dbl, vp, vp, vp, vp, vp], C.c_int),
        "bem_incident": ([vp, C.POINTER(bem_surface), i32, vp, vp, vp], C.c_int),
        "bem_assemble": ([vp, C.POINTER(bem_surface), i32, vp, i32, vp, C.c_int, vp, i32, vp, vp], C.c_int),
        "bem_residual": ([vp, C.POINTER(bem_surface), i32, vp, i32, vp, vp, vp, vp], C.c_int),
        "bem_solve_opts_default": ([C.POINTER(bem_solve_opts)], None),
        "bem_solve_batched": ([vp, C.POINTER(bem_problem), i32, C.POINTER(bem_solve_opts), vp,
                               C.POINTER(bem_solve_info)], C.c_int),
        "bem_getrf_batched": ([vp, C.c_int, i32, i32, i64, i32, vp, vp, vp, i32, i32], C.c_int),
        "bem_getrs_batched": ([vp, C.c_int, i32, i32, i64, i32, vp, vp, i32, vp, vp, i64], C.c_int),
        "bem_autotune_lu": ([vp, C.c_int, i32, i32, i32, vp, C.POINTER(i32), C.POINTER(dbl)],
                            C.c_int),
        "bem_split_unknowns": ([vp, C.POINTER(bem_surface), i32, i32, vp, vp, vp, vp], C.c_int),
        "bem_field_eval": ([vp, C.POINTER(bem_surface), i32, vp, i32, vp, vp, i32, vp, vp, i32, vp,
                            C.c_int, vp], C.c_int),
        "bem_field_eval_noalloc": ([vp, C.POINTER(bem_surface), i32, vp, i32, vp, vp, i32, vp, vp,
                                    i32, vp, C.c_int, vp], C.c_int),
        "pulse_synthesize": ([vp, i32, i32, vp, i32, vp, i32, i32, vp, dbl, vp], C.c_int),
        "pulse_synthesize_sparse": ([vp, i32, i32, vp, vp, i32, vp, i32, i32, vp, dbl, vp],
                                    C.c_int),
        "bem_pulse_coeffs": ([i32, vp, i32, dbl, i32, i32, dbl, vp], C.c_int),
        "bem_pulse_dominant": ([vp, i32, i32, vp], C.c_int),
        "bem_residual_check": ([vp, C.POINTER(bem_surface), i32, vp, i32, vp, vp, vp], C.c_int),
        "bem_refine_batched": ([vp, C.POINTER(bem_surface), i32, vp, i32, vp, vp, i32, i64, vp, i32,
                                vp, dbl, i32, vp, C.POINTER(bem_solve_info)], C.c_int),
        "bem_mlp_features": ([vp, i32, vp, i32, dbl, vp], C.c_int),
        "bem_mlp_dense_fwd": ([vp, i32, i32, i32, vp, vp, vp, i32, vp, vp], C.c_int),
        "bem_mlp_dense_bwd": ([vp, i32, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp], C.c_int),
        "bem_mlp_mse_grad": ([vp, i64, vp, vp, vp, vp, i32], C.c_int),
        "bem_mlp_adam": ([vp, i64, vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
        "bem_mlp_pack": ([vp, i32, i32, vp, vp, i32, vp], C.c_int),
        "bem_mlp_unpack": ([vp, i32, i32, vp, vp, vp], C.c_int),
        "bem_mesh_quadratic_counts": ([i32, C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "bem_mesh_quadratic": ([i32, dbl, dbl, vp, vp, vp, vp], C.c_int),
        "bem_assemble_quadratic": ([vp, C.POINTER(bem_quad_surface), i32, vp, i32, vp, C.c_int, vp,
                                    i32, vp, vp], C.c_int),
        "bem_solve_quadratic": ([vp, C.POINTER(bem_quad_surface), i32, vp, i32, vp,
                                 C.POINTER(bem_solve_opts), vp, C.POINTER(bem_solve_info)], C.c_int),
        "bem_field_eval_quadratic": ([vp, C.POINTER(bem_quad_surface), i32, vp, i32, vp, vp, i32,
                                      vp, vp, vp, vp], C.c_int),
        "bem_solve_chief": ([vp, C.POINTER(bem_surface), i32, vp, i32, vp, i32, vp, vp,
                             C.POINTER(bem_solve_info)], C.c_int),
        "bem_autotune_lu_results": ([vp, i32, vp, vp, vp, vp], i32),
        "bem_lu_tuned_plan": ([vp, C.c_int, i32, i32, C.POINTER(i32), C.POINTER(i32),
                               C.POINTER(i32)], C.c_int),
        "bem_lu_set_plan": ([vp, C.c_int, i32, i32, i32, i32, i32], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(t):
    """Device/host address of a torch tensor or numpy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _check(st, ctx=None):
    if st != BEM_OK:
        msg = load().bem_last_error(ctx.handle if ctx is not None else None)
        raise BemError(st, msg.decode() if msg else "")


# ---------------------------------------------------------------- context
class Context:
    """A library context on one device/stream (torch provides the stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = lib.bem_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != BEM_OK:
            raise BemError(st, "bem_ctx_create failed")
        self.handle = h

    def close(self):
        if self.handle:
            load().bem_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, on: bool):
        _check(load().bem_ctx_set_profiling(self.handle, int(bool(on))), self)

    def set_profiling_filter(self, names=None):
        """Count only the named kernels (an iterable or comma-separated string);
        None or empty = all."""
        if names is not None and not isinstance(names, str):
            names = ",".join(names)
        _check(load().bem_ctx_set_profiling_filter(self.handle, (names or "").encode()), self)

    def kernel_stats(self, name: str):
        """(flops, bytes, ms, launches) accumulated since profiling was switched."""
        f, b, ms = C.c_double(), C.c_double(), C.c_double()
        n = C.c_int64()
        _check(load().bem_ctx_kernel_stats(self.handle, name.encode(), C.byref(f), C.byref(b),
                                           C.byref(ms), C.byref(n)), self)
        return f.value, b.value, ms.value, n.value

    def set_workspace_limit(self, nbytes: int):
        _check(load().bem_ctx_set_workspace_limit(self.handle, int(nbytes)), self)


# ---------------------------------------------------------------- geometry (host)
def bem_mesh_counts(level: int):
    nv, nf = C.c_int32(), C.c_int32()
    _check(load().bem_mesh_counts(level, C.byref(nv), C.byref(nf)))
    return nv.value, nf.value


def bem_mesh_bowl(n_theta, n_phi, radius=1.0, tilt=0.0, center=(0.0, 0.0, 0.0)):
    nv, nf = C.c_int32(), C.c_int32()
    _check(load().bem_mesh_bowl_counts(int(n_theta), int(n_phi), C.byref(nv), C.byref(nf)))
    x = np.empty((nv.value, 3)); nrm = np.empty((nv.value, 3)); w = np.empty(nv.value)
    faces = np.empty((nf.value, 3), dtype=np.int32)
    c = np.ascontiguousarray(center, dtype=np.float64)
    _check(load().bem_mesh_bowl(int(n_theta), int(n_phi), float(radius), float(tilt),
                                c.ctypes.data, x.ctypes.data, nrm.ctypes.data, w.ctypes.data,
                                faces.ctypes.data))
    return x, nrm, w, faces


def bem_mesh_icosphere(level, radius, aspect, center, rescale_area=True):
    nv, nf = bem_mesh_counts(level)
    x = np.empty((nv, 3)); nrm = np.empty((nv, 3)); w = np.empty(nv)
    faces = np.empty((nf, 3), dtype=np.int32)
    c = np.ascontiguousarray(center, dtype=np.float64)
    _check(load().bem_mesh_icosphere(level, float(radius), float(aspect), c.ctypes.data,
                                     int(bool(rescale_area)), x.ctypes.data, nrm.ctypes.data,
                                     w.ctypes.data, faces.ctypes.data))
    return x, nrm, w, faces


def bem_pulse_coeffs(kind, params, dk, n_k, T, z_shift):
    p = np.ascontiguousarray(params, dtype=np.float64)
    out = np.empty(2 * n_k)
    kid = PULSE_KINDS[kind] if isinstance(kind, str) else int(kind)
    _check(load().bem_pulse_coeffs(kid, p.ctypes.data, len(p), float(dk), int(n_k), int(T),
                                   float(z_shift), out.ctypes.data))
    return out.view(np.complex128)


def bem_pulse_dominant(c, n_keep):
    """1-based indices of the n_keep largest |c_m|, in increasing order."""
    cc = np.ascontiguousarray(c, dtype=np.complex128)
    out = np.empty(int(n_keep), dtype=np.int32)
    _check(load().bem_pulse_dominant(cc.ctypes.data, len(cc), int(n_keep), out.ctypes.data))
    return out


# ---------------------------------------------------------------- device entry points
def bem_mesh_quadratic(nu, radius=1.0, aspect=1.0, center=(0.0, 0.0, 0.0)):
    """Six-node elements on a frequency-nu geodesic sphere: (x, nrm, elems)."""
    nn, ne = C.c_int32(), C.c_int32()
    _check(load().bem_mesh_quadratic_counts(int(nu), C.byref(nn), C.byref(ne)))
    x = np.empty((nn.value, 3)); nrm = np.empty((nn.value, 3))
    elems = np.empty((ne.value, 6), dtype=np.int32)
    c = np.ascontiguousarray(center, dtype=np.float64)
    _check(load().bem_mesh_quadratic(int(nu), float(radius), float(aspect), c.ctypes.data,
                                     x.ctypes.data, nrm.ctypes.data, elems.ctypes.data))
    return x, nrm, elems


def quad_surface_struct(n, x, nrm, bc, n_elem, elem):
    return bem_quad_surface(int(n), _ptr(x), _ptr(nrm), _ptr(bc), int(n_elem), _ptr(elem))


def bem_assemble_quadratic(ctx, qsurf, n_k, k, n_rhs, y, prec, A, ld, b, diag64=None):
    _check(load().bem_assemble_quadratic(ctx.handle, C.byref(qsurf), n_k, _ptr(k), n_rhs,
                                         _ptr(y), prec, _ptr(A), int(ld), _ptr(b), _ptr(diag64)),
           ctx)


def bem_solve_quadratic(ctx, qsurf, n_k, k, n_rhs, y, opts, x_out):
    info = (bem_solve_info * (n_k * n_rhs))()
    _check(load().bem_solve_quadratic(ctx.handle, C.byref(qsurf), n_k, _ptr(k), n_rhs, _ptr(y),
                                      C.byref(opts), _ptr(x_out), info), ctx)
    return info


def bem_autotune_lu_results(ctx):
    """Every plan the last bem_autotune_lu tried: list of (nb, narrow_max, persistent, ms)."""
    cnt = load().bem_autotune_lu_results(ctx.handle, 0, None, None, None, None)
    nb, nw, ps = (C.c_int32 * max(cnt, 1))(), (C.c_int32 * max(cnt, 1))(), (C.c_int32 * max(cnt, 1))()
    ms = (C.c_double * max(cnt, 1))()
    load().bem_autotune_lu_results(ctx.handle, cnt, nb, nw, ps, ms)
    return [(nb[i], nw[i], ps[i], ms[i]) for i in range(cnt)]


def bem_lu_set_plan(ctx, prec, n, gemm_kind, nb, narrow_max=64, persistent=0):
    _check(load().bem_lu_set_plan(ctx.handle, prec, n, gemm_kind, nb, narrow_max, persistent), ctx)


def bem_lu_tuned_plan(ctx, prec, n, gemm_kind):
    """(nb, narrow_max, persistent) kept by bem_autotune_lu for this size class."""
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().bem_lu_tuned_plan(ctx.handle, prec, n, gemm_kind, C.byref(a), C.byref(b),
                                    C.byref(c)), ctx)
    return a.value, b.value, c.value


def bem_solve_chief(ctx, surf, n_k, k, n_rhs, y, n_c, xc, x_out):
    """Least-squares solve with n_c interior-point rows; returns the info array."""
    info = (bem_solve_info * (n_k * n_rhs))()
    _check(load().bem_solve_chief(ctx.handle, C.byref(surf), n_k, _ptr(k), n_rhs, _ptr(y), n_c,
                                  _ptr(xc), _ptr(x_out), info), ctx)
    return info


def bem_field_eval_quadratic(ctx, qsurf, n_k, k, n_rhs, phi, psi, m, xp, i0, inside, U):
    _check(load().bem_field_eval_quadratic(ctx.handle, C.byref(qsurf), n_k, _ptr(k), n_rhs,
                                           _ptr(phi), _ptr(psi), m, _ptr(xp), _ptr(i0),
                                           _ptr(inside), _ptr(U)), ctx)


def surface_struct(n, x, nrm, w, bc):
    return bem_surface(int(n), _ptr(x), _ptr(nrm), _ptr(w), _ptr(bc))


def bem_incident(ctx, surf, n_k, k, direction, y):
    d = np.ascontiguousarray(direction, dtype=np.float64)
    _check(load().bem_incident(ctx.handle, C.byref(surf), n_k, _ptr(k), d.ctypes.data, _ptr(y)), ctx)


def bem_assemble(ctx, surf, n_k, k, n_rhs, y, prec, A, ld, b, diag64):
    _check(load().bem_assemble(ctx.handle, C.byref(surf), n_k, _ptr(k), n_rhs, _ptr(y), prec,
                               _ptr(A), ld, _ptr(b), _ptr(diag64)), ctx)


def bem_residual(ctx, surf, n_k, k, n_rhs, y, x, diag64, r):
    _check(load().bem_residual(ctx.handle, C.byref(surf), n_k, _ptr(k), n_rhs, _ptr(y), _ptr(x),
                               _ptr(diag64), _ptr(r)), ctx)


def bem_solve_opts_default():
    o = bem_solve_opts()
    load().bem_solve_opts_default(C.byref(o))
    return o


def bem_solve_batched(ctx, problems, opts, x_out, want_info=True):
    """problems: list of (surface_struct, n_k, k, n_rhs, y); x_out: list of tensors."""
    n = len(problems)
    surfs = [p[0] for p in problems]
    arr = (bem_problem * n)()
    for i, (s, n_k, k, n_rhs, y) in enumerate(problems):
        arr[i] = bem_problem(C.pointer(surfs[i]), n_k, _ptr(k), n_rhs, _ptr(y))
    xo = (C.c_void_p * n)(*[_ptr(t) for t in x_out])
    total = sum(p[1] * p[3] for p in problems)
    info = (bem_solve_info * total)() if want_info else None
    _check(load().bem_solve_batched(ctx.handle, arr, n, C.byref(opts), xo, info), ctx)
    return info


def bem_getrf_batched(ctx, prec, n, ld, stride, batch, A, piv, info, nb=0, gemm_kind=0):
    _check(load().bem_getrf_batched(ctx.handle, prec, n, ld, stride, batch, _ptr(A), _ptr(piv),
                                    _ptr(info), nb, gemm_kind), ctx)


def bem_autotune_lu(ctx, prec, n, batch, gemm_kind=0, candidates=None):
    """Measure the factorisation for each candidate block width; returns
    (best_nb, best_ms) and keeps the choice in the context."""
    cand = None
    if candidates is not None:
        cand = (C.c_int32 * (len(candidates) + 1))(*candidates, 0)
    best = C.c_int32()
    ms = C.c_double()
    _check(load().bem_autotune_lu(ctx.handle, prec, n, batch, gemm_kind, cand, C.byref(best),
                                  C.byref(ms)), ctx)
    return best.value, ms.value


def bem_getrs_batched(ctx, prec, n, ld, stride, batch, LU, piv, n_rhs, B, X, bstride):
    _check(load().bem_getrs_batched(ctx.handle, prec, n, ld, stride, batch, _ptr(LU), _ptr(piv),
                                    n_rhs, _ptr(B), _ptr(X), bstride), ctx)


def bem_split_unknowns(ctx, surf, n_k, n_rhs, x, y, phi, psi):
    _check(load().bem_split_unknowns(ctx.handle, C.byref(surf), n_k, n_rhs, _ptr(x), _ptr(y),
                                     _ptr(phi), _ptr(psi)), ctx)


def bem_field_eval(ctx, surf, n_k, k, n_rhs, phi, psi, m, xp, i0, i0_given, inside, prec, U):
    _check(load().bem_field_eval(ctx.handle, C.byref(surf), n_k, _ptr(k), n_rhs, _ptr(phi),
                                 _ptr(psi), m, _ptr(xp), _ptr(i0), int(i0_given), _ptr(inside),
                                 prec, _ptr(U)), ctx)


def bem_field_eval_noalloc(ctx, surf, n_k, k, n_rhs, phi, psi, m, xp, i0, i0_given, inside,
                           prec, U):
    _check(load().bem_field_eval_noalloc(ctx.handle, C.byref(surf), n_k, _ptr(k), n_rhs,
                                         _ptr(phi), _ptr(psi), m, _ptr(xp), _ptr(i0),
                                         int(i0_given), _ptr(inside), prec, _ptr(U)), ctx)


def pulse_synthesize(ctx, m, n_k, U, n_pulse, c, T, add_incident, xp, dk, p):
    _check(load().pulse_synthesize(ctx.handle, m, n_k, _ptr(U), n_pulse, _ptr(c), T,
                                   int(add_incident), _ptr(xp), float(dk), _ptr(p)), ctx)


def pulse_synthesize_sparse(ctx, m, m_index, U, n_pulse, c, T, add_incident, xp, dk, p):
    idx = np.ascontiguousarray(m_index, dtype=np.int32)
    _check(load().pulse_synthesize_sparse(ctx.handle, m, len(idx), idx.ctypes.data, _ptr(U),
                                          n_pulse, _ptr(c), T, int(add_incident), _ptr(xp),
                                          float(dk), _ptr(p)), ctx)


def bem_residual_check(ctx, surf, n_k, k, n_rhs, y, x):
    rel = np.empty(n_k * n_rhs)
    _check(load().bem_residual_check(ctx.handle, C.byref(surf), n_k, _ptr(k), n_rhs, _ptr(y),
                                     _ptr(x), rel.ctypes.data), ctx)
    return rel


def bem_mlp_features(ctx, B, k, n_oct, kscale, x):
    _check(load().bem_mlp_features(ctx.handle, B, _ptr(k), n_oct, float(kscale), _ptr(x)), ctx)


def bem_mlp_dense_fwd(ctx, B, n_in, n_out, x, W, b, act, z, y):
    _check(load().bem_mlp_dense_fwd(ctx.handle, B, n_in, n_out, _ptr(x), _ptr(W), _ptr(b),
                                    int(act), _ptr(z), _ptr(y)), ctx)


def bem_mlp_dense_bwd(ctx, B, n_in, n_out, x, W, z, act, dy, dW, db, dx, dz):
    _check(load().bem_mlp_dense_bwd(ctx.handle, B, n_in, n_out, _ptr(x), _ptr(W), _ptr(z),
                                    int(act), _ptr(dy), _ptr(dW), _ptr(db), _ptr(dx), _ptr(dz)), ctx)


def bem_mlp_mse_grad(ctx, count, y, t, dy, partial, n_partial):
    _check(load().bem_mlp_mse_grad(ctx.handle, int(count), _ptr(y), _ptr(t), _ptr(dy),
                                   _ptr(partial), int(n_partial)), ctx)


def bem_mlp_adam(ctx, n, p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    _check(load().bem_mlp_adam(ctx.handle, int(n), _ptr(p), _ptr(g), _ptr(m), _ptr(v), int(step),
                               float(lr), float(b1), float(b2), float(eps)), ctx)


def bem_mlp_pack(ctx, B, n, x, scale, compute_scale, t):
    _check(load().bem_mlp_pack(ctx.handle, B, n, _ptr(x), _ptr(scale), int(compute_scale),
                               _ptr(t)), ctx)


def bem_mlp_unpack(ctx, B, n, t, scale, x):
    _check(load().bem_mlp_unpack(ctx.handle, B, n, _ptr(t), _ptr(scale), _ptr(x)), ctx)


def bem_refine_batched(ctx, surf, n_k, k, n_rhs, y, LU, ld, stride, piv, n_fac, fac_index,
                       tol_step, max_iter, x, want_info=True):
    info = (bem_solve_info * (n_k * n_rhs))() if want_info else None
    _check(load().bem_refine_batched(ctx.handle, C.byref(surf), n_k, _ptr(k), n_rhs, _ptr(y),
                                     _ptr(LU), ld, stride, _ptr(piv), n_fac, _ptr(fac_index),
                                     float(tol_step), int(max_iter), _ptr(x), info), ctx)
    return info
