#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload: two sound-hard spheres of radius 1, level-4 icospheres (N = 5124
nodes), 512 wavenumbers k_m = 12 m / 512 (m = 1..512), incident plane wave
along +z.  One step = one pass of the whole path over the 512 wavenumbers:
incident data, float64-accurate assembly, complex float32 LU on MFMA,
refinement with the float64 matrix-free residual to ||dx||/||x|| <= 1e-8
(FP64 fallback armed), surface data split, closest node + field at a grid of
observation points for all 512 frequencies, and synthesis of one pulse.

value = frequency solves per second (whole step time).  The field metric
(point x frequency evaluations per second) and the plain FP64 direct path
are reported beside it.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_F32_MFMA = 157.3e12
PEAK_BF16_MFMA = 2500.0e12
PEAK_F64_MFMA = 78.6e12
PEAK_HBM = 8.0e12


# dominant kernel of the factorisation per GEMM form: (stats name, kernel,
# issued MFMA flops per 4M-equivalent flop, MFMA peak)
DOMINANT = {
    "3m": ("gemm_3m", "gemm_c32_lds_kernel<3M, 128x128> (LU trailing updates, complex 3M on "
                      "MFMA f32, operands streamed into LDS)", 0.75, PEAK_F32_MFMA),
    "4m": ("gemm_c32", "gemm_c32_lds_kernel<4M, 128x128> (LU trailing updates, complex 4M on "
                       "MFMA f32, operands streamed into LDS)", 1.0, PEAK_F32_MFMA),
    "b3": ("gemm_b3_packed", "gemm_c32_b3p_kernel (LU trailing updates, bf16x3 split on MFMA "
                             "bf16, operands pre-split)", 3.0, PEAK_BF16_MFMA),
}
MODES = None     # filled on first use (needs the binding)
# VALU instructions per field term: the compiled node loop of
# field_grouped_kernel<8, 1> issues 261 per pass over two nodes and a chunk of
# 8 frequencies (the float64 geometry and phases of the pair included), i.e.
# about 16.3 per (point, frequency, node) term, one lane each
FIELD_VALU_PER_TERM = 261.0 / 16.0
# the FP32 vector peak (157.3 TFLOP/s) as lane instructions, one multiply-add
# each: 7.87e13/s (the SIMDs issue float32 instructions faster than one per 4
# cycles per wave64, as the VALU counters of the field kernel show)
PEAK_VALU_LANE_OPS = 157.3e12 / 2


class KernelTotals:
    """Per-kernel statistics summed over every profiling window of the run
    (the library resets its counters whenever profiling is switched)."""

    def __init__(self, ctx, names):
        self.ctx, self.names = ctx, tuple(names)
        self.tot = {k: [0.0, 0.0, 0.0, 0] for k in self.names}

    def harvest(self):
        for k in self.names:
            f, b, ms, n = self.ctx.kernel_stats(k)
            t = self.tot[k]
            t[0] += f
            t[1] += b
            t[2] += ms
            t[3] += n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-k", type=int, default=512)
    ap.add_argument("--field-grid", type=int, default=64, help="points per side on x = 0")
    ap.add_argument("--fp64-every", type=int, default=8,
                    help="every this many wavenumbers of the sweep are also solved by the plain "
                         "FP64 direct path (0: none)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-k", type=int, default=8)
    ap.add_argument("--mode", choices=["b3", "4m", "3m"], default="3m",
                    help="complex GEMM form of the float32 factorisation")
    ap.add_argument("--field-rhs", type=int, default=4,
                    help="right-hand sides of the multi-rhs field measurement (0: off)")
    ap.add_argument("--b3-steps", type=int, default=2,
                    help="steps of the bf16x3 variant timed after the headline (0: none)")
    ap.add_argument("--spacetime", type=int, default=1,
                    help="1: time the space-time reconstruction (2048 solves, 1024^2 points, "
                         "4 pulses, T = 4096) after the headline")
    ap.add_argument("--workload", choices=["spheres", "surrogate", "uneven", "spacetime",
                                           "truncation", "bowl", "chief", "quadratic"],
                    default="spheres",
                    help="spheres: the headline sweep; surrogate: the learned-fill gain "
                         "test (256 training / 4096 predicted wavenumbers, N = 5124); "
                         "uneven: eight bodies of 642 to 10242 nodes solved together; "
                         "spacetime: 2048 solves, field on a 1024^2 grid, 4 pulses; "
                         "truncation: the paper's soft sphere and pulse rebuilt from the "
                         "5/10/20 frequencies of largest amplitude vs all 63; "
                         "bowl: the hard acoustic bowl's focusing of a 6-cycle pulse; "
                         "chief: interior-point rows against fictitious resonances; "
                         "quadratic: the paper's 500-element sphere, whole path")
    ap.add_argument("--bowl-rings", type=int, default=48,
                    help="bowl: rings of the meridian (twice as many nodes per ring)")
    ap.add_argument("--tr-level", type=int, default=5,
                    help="icosphere level of the sphere for --workload truncation")
    ap.add_argument("--tr-grid", type=int, default=256,
                    help="points per side of the x = 0 field grid for --workload truncation")
    ap.add_argument("--st-grid", type=int, default=1024,
                    help="points per side of the field grid of the space-time reconstruction")
    ap.add_argument("--uneven-k", type=int, default=1024,
                    help="wavenumbers per body for --workload uneven")
    ap.add_argument("--uneven-steps", type=int, default=1,
                    help="timed passes of --workload uneven")
    ap.add_argument("--nb", type=int, default=0, help="LU block width (0 = library default)")
    ap.add_argument("--gemm-narrow-max", type=int, default=0,
                    help="set the plan of the size class by hand: 128 x 64 GEMM tiles up to this "
                         "many columns (0: leave the plan alone)")
    ap.add_argument("--gemm-persistent", type=int, default=0,
                    help="with --gemm-narrow-max: 1 = persistent GEMM launches")
    ap.add_argument("--autotune", type=int, default=0,
                    help="measure the LU block width on this many matrices before the run")
    ap.add_argument("--sur-epochs", type=int, default=100,
                    help="training epochs of the surrogate (100: the fit costs about what it saves)")
    ap.add_argument("--sur-sweeps", type=int, default=20)
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run one plain elementwise copy of 256 MiB (reads 256 MiB, "
                         "writes 256 MiB: the reference for the HBM byte counters of a "
                         "profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(frequencies shard across GPUs by design, but this build measures one GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.workload == "surrogate":
        run_surrogate(args)
        return
    if args.workload == "uneven":
        run_uneven(args)
        return
    if args.workload == "spacetime":
        print(json.dumps(run_spacetime(args)))
        return
    if args.workload == "truncation":
        run_truncation(args)
        return
    if args.workload == "bowl":
        run_bowl(args)
        return
    if args.workload == "chief":
        run_chief(args)
        return
    if args.workload == "quadratic":
        run_quadratic(args)
        return

    from paper_1706_07919_amd import DeviceSurface, native
    from workloads import two_spheres_workload, plane_grid

    if args.copy_calib:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    modes = {"b3": native.BEM_FP32_IR_B3, "4m": native.BEM_FP32_IR_4M, "3m": native.BEM_FP32_IR_3M}
    gname, kdesc, issue_per_alg, peak = DOMINANT[args.mode]
    w = two_spheres_workload(args.n_k)
    n_k = len(w.k)
    dev = torch.device("cuda:0")
    ctx = native.Context(0)
    totals = KernelTotals(ctx, (gname,))
    ds = DeviceSurface.from_bodies(w.bodies)
    n = ds.n
    kd = torch.as_tensor(w.k).to(dev)
    xp = torch.as_tensor(plane_grid(args.field_grid)).to(dev)
    m = xp.shape[0]
    T = w.T
    pulse = w.pulses[0]
    c = native.bem_pulse_coeffs(pulse.kind, [pulse.params["k0"], pulse.params["sigma"]], w.dk,
                                n_k, T, w.z_shift)
    cd = torch.as_tensor(c).to(dev)
    y = torch.empty((n_k, 1, n), dtype=torch.complex128, device=dev)
    x = torch.zeros((n_k, 1, n), dtype=torch.complex128, device=dev)
    phi = torch.empty_like(x)
    psi = torch.empty_like(x)
    U = torch.zeros((1, m, n_k), dtype=torch.complex64, device=dev)
    i0 = torch.zeros(m, dtype=torch.int32, device=dev)
    ins = torch.zeros(m, dtype=torch.uint8, device=dev)
    p = torch.zeros((1, m, T), dtype=torch.float32, device=dev)
    opts = native.bem_solve_opts_default()
    opts.mode = modes[args.mode]
    opts.nb = args.nb
    tuned = tuned_plan = tune_log = None
    if args.gemm_narrow_max > 0:
        gk = {"b3": native.BEM_GEMM_BF16X3, "4m": native.BEM_GEMM_4M, "3m": native.BEM_GEMM_3M}[args.mode]
        native.bem_lu_set_plan(ctx, native.BEM_C64, n, gk, args.nb or 512, args.gemm_narrow_max,
                               args.gemm_persistent)
    if args.autotune > 0:
        gk = {"b3": native.BEM_GEMM_BF16X3, "4m": native.BEM_GEMM_4M, "3m": native.BEM_GEMM_3M}[args.mode]
        tuned = native.bem_autotune_lu(ctx, native.BEM_C64, n, args.autotune, gk)
        tune_log = native.bem_autotune_lu_results(ctx)
        tuned_plan = native.bem_lu_tuned_plan(ctx, native.BEM_C64, n, gk)
        print(f"autotuned plan {tuned_plan} ({tuned[1]:.1f} ms for {args.autotune} matrices)",
              file=sys.stderr, flush=True)
    infos = []

    def step():
        native.bem_incident(ctx, ds.struct, n_k, kd, (0.0, 0.0, 1.0), y)
        info = native.bem_solve_batched(ctx, [(ds.struct, n_k, kd, 1, y)], opts, [x])
        native.bem_split_unknowns(ctx, ds.struct, n_k, 1, x, y, phi, psi)
        native.bem_field_eval(ctx, ds.struct, n_k, kd, 1, phi, psi, m, xp, i0, 0, ins,
                              native.BEM_C64, U)
        native.pulse_synthesize(ctx, m, n_k, U[0], 1, cd, T, 1, xp, w.dk, p)
        infos.append(info)

    # every launch of the dominant kernel is bracketed by HIP events on the
    # stream it runs on, over the whole run (the roofline averages all of them)
    ctx.set_profiling_filter((gname,))
    ctx.set_profiling(True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    totals.harvest()
    # the timed steps bracket the dominant kernel, the field and the synthesis
    timed_kernels = (gname, "field", "synth")
    ctx.set_profiling_filter(timed_kernels)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    stats = {kname: ctx.kernel_stats(kname) for kname in timed_kernels}
    totals.harvest()
    # one more step, untimed, with every counted kernel bracketed: the split of
    # the step by kernel
    ctx.set_profiling_filter(None)
    ctx.set_profiling(True)
    step()
    torch.cuda.synchronize()
    split_names = (gname, gname + "_narrow", "gemm_b3", "gemm_b3_narrow", "gemm_small", "pack",
                   "panel", "laswp", "trsm", "assemble", "residual", "getrs", "field", "synth")
    split = {kname: ctx.kernel_stats(kname)[2] for kname in split_names
             if kname in DOMINANT_SPLIT_OK or ctx.kernel_stats(kname)[3] > 0}
    totals.harvest()
    ctx.set_profiling_filter((gname,))
    ctx.set_profiling(True)
    solves_per_s = n_k * args.steps / elapsed
    info = infos[-1]
    iters = [info[q].iters for q in range(n_k)]
    fallbacks = sum(info[q].used_fp64 for q in range(n_k))
    max_resid = max(info[q].rel_resid for q in range(n_k))
    ff, fb, fms, fl = stats["field"]
    field_rate = (m * n_k * args.steps) / (fms * 1e-3) if fms > 0 else 0.0
    sf, sb, sms, sl = stats["synth"]

    # plain FP64 direct path on every fp64_every-th wavenumber of the sweep
    # (spread over the whole band): its rate, and the float32 + refinement
    # result's distance from it
    fp64_rate, rel64, rel64_max = None, None, None
    if args.fp64_every > 0:
        sel = torch.arange(0, n_k, args.fp64_every, device=dev)
        kk = int(sel.numel())
        ks = kd[sel].contiguous()
        ys = y[sel].contiguous()
        x64 = torch.zeros((kk, 1, n), dtype=torch.complex128, device=dev)
        o64 = native.bem_solve_opts_default()
        o64.mode = native.BEM_FP64_DIRECT
        native.bem_solve_batched(ctx, [(ds.struct, kk, ks, 1, ys)], o64, [x64])
        torch.cuda.synchronize()
        ta = time.perf_counter()
        native.bem_solve_batched(ctx, [(ds.struct, kk, ks, 1, ys)], o64, [x64])
        torch.cuda.synchronize()
        fp64_rate = kk / (time.perf_counter() - ta)
        d = torch.linalg.vector_norm(x64 - x[sel], dim=(1, 2)) / torch.linalg.vector_norm(x64, dim=(1, 2))
        rel64, rel64_max = (torch.linalg.vector_norm(x64 - x[sel]) / torch.linalg.vector_norm(x64)).item(), d.max().item()
        del x64, ys

    # the bf16x3 variant of the same step (not the headline: the products of
    # its factorisation are bf16)
    b3 = None
    if args.b3_steps > 0 and args.mode != "b3":
        ob3 = native.bem_solve_opts_default()
        ob3.mode = native.BEM_FP32_IR_B3
        xb3 = torch.zeros_like(x)   # x keeps the headline mode's solution
        native.bem_solve_batched(ctx, [(ds.struct, n_k, kd, 1, y)], ob3, [xb3])
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(args.b3_steps):
            native.bem_incident(ctx, ds.struct, n_k, kd, (0.0, 0.0, 1.0), y)
            native.bem_solve_batched(ctx, [(ds.struct, n_k, kd, 1, y)], ob3, [xb3])
        torch.cuda.synchronize()
        b3 = n_k * args.b3_steps / (time.perf_counter() - tb)
        del xb3

    # the field with several right-hand sides (the step's solution and phase-
    # rotated copies): every generated kernel value is applied to all of them
    mrhs = None
    if args.field_rhs > 1:
        R = args.field_rhs
        rot = torch.exp(1j * 0.7 * torch.arange(R, device=dev, dtype=torch.float64)).view(1, R, 1)
        phr = (phi * rot).contiguous()
        psr = (psi * rot).contiguous()
        Ur = torch.zeros((R, m, n_k), dtype=torch.complex64, device=dev)

        def fr(nr, a, b, out):
            native.bem_field_eval(ctx, ds.struct, n_k, kd, nr, a, b, m, xp, i0, 1, ins,
                                  native.BEM_C64, out)
        fr(R, phr, psr, Ur)
        fr(1, phi, psi, U)
        torch.cuda.synchronize()
        reps = 3
        ta = time.perf_counter()
        for _ in range(reps):
            fr(R, phr, psr, Ur)
        torch.cuda.synchronize()
        t_multi = (time.perf_counter() - ta) / reps
        ta = time.perf_counter()
        for _ in range(reps):
            fr(1, phi, psi, U)
        torch.cuda.synchronize()
        t_one = (time.perf_counter() - ta) / reps
        mrhs = {"n_rhs": R, "points": m, "n_k": n_k,
                "pt_freq_rhs_per_s": m * n_k * R / t_multi,
                "ms": 1e3 * t_multi, "ms_one_rhs": 1e3 * t_one,
                "vs_separate_calls": R * t_one / t_multi,
                "note": "both passes of bem_field_eval (nodes and points); vs_separate_calls = "
                        "n_rhs single-rhs calls' time over one n_rhs call"}
        del phr, psr, Ur

    st = None
    if args.spacetime:
        del U, p, phi, psi
        st = run_spacetime(args, ctx=ctx, mode=opts.mode)
    totals.harvest()
    ctx.set_profiling(False)

    gf, gb, gms, gl = totals.tot[gname]
    achieved = issue_per_alg * gf / (gms * 1e-3) if gms > 0 else 0.0
    alg_rate = gf / (gms * 1e-3) if gms > 0 else 0.0

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, x, args.cpu_k)

    out = {
        "metric": "BEM freq-solves/sec at N=5124 (rel err <=1e-6 vs FP64); field pt*freq evals/sec",
        "value": solves_per_s,
        "unit": "freq-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"b3": "c64 LU (bf16x3 split products on bf16 MFMA, f32 accumulate)",
                  "4m": "c64 LU (complex 4M on f32 MFMA, f32 accumulate)",
                  "3m": "c64 LU (complex 3M on f32 MFMA, f32 accumulate)"}[args.mode]
                 + " + f64 residual refinement",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "n_k": n_k, "field_points": m, "T": T,
                   "mode": {"b3": "FP32_IR_B3", "4m": "FP32_IR_4M", "3m": "FP32_IR_3M"}[args.mode],
                   "nb": opts.nb, "autotuned_nb": tuned[0] if tuned else None,
                   "gemm_plan_set": ({"narrow_max": args.gemm_narrow_max,
                                      "persistent": args.gemm_persistent}
                                     if args.gemm_narrow_max > 0 else None),
                   "autotuned_plan": ({"nb": tuned_plan[0], "narrow_max": tuned_plan[1],
                                       "persistent": tuned_plan[2]} if tuned else None)},
        "autotune_log": ([{"nb": r[0], "narrow_max": r[1], "persistent": r[2], "ms": r[3]}
                          for r in tune_log] if tuned else None),
        "field_pt_freq_per_s": st["value"] if st else field_rate,
        "field_pt_freq_per_s_note": ("space-time reconstruction at 1024^2 points x 2048 frequencies "
                                     "(the step's own 4096-point field is field_pt_freq_per_s_step)"
                                     if st else "4096 points x 512 frequencies of the step"),
        "field_pt_freq_per_s_step": field_rate,
        "field_multi_rhs": mrhs,
        "fp64_direct_solves_per_s": fp64_rate,
        "fp32ir_vs_fp64_direct_rel_err": rel64,
        "fp32ir_vs_fp64_direct_max_rel_err_per_k": rel64_max,
        "fp64_direct_sample": f"every {args.fp64_every}th wavenumber of the sweep" if args.fp64_every else None,
        "b3_solves_per_s": b3,
        "ir_iters_max": max(iters),
        "ir_fallbacks": fallbacks,
        "max_rel_resid": max_resid,
        "roofline": {"kernel": kdesc,
                     "bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "achieved_note": "MFMA flops the kernel issues (3M: 6 MNK, 4M: 8 MNK, bf16x3: "
                                      "24 MNK per complex update) over the HIP-event time of every "
                                      "launch of the run",
                     "traffic": measured_traffic(gname, args.nb or (tuned[0] if tuned else "default"),
                                                 gb / max(gl, 1)),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "scaled by a copy kernel)",
                     "algorithmic_bytes_per_launch": gb / max(gl, 1),
                     "algorithmic_flops_per_launch": gf / max(gl, 1),
                     "launches": gl, "avg_launch_ms": gms / max(gl, 1),
                     "algorithmic_tflops": alg_rate / 1e12,
                     "algorithmic_tflops_note": "8 MNK per complex update (the 4M count)",
                     "share_of_step": stats[gname][2] * 1e-3 / elapsed},
        "kernels_ms_per_step": split,
        "kernels_ms_per_step_note": "one extra step with every kernel bracketed by events "
                                    "(the timed steps bracket only the roofline kernel, field "
                                    "and synthesis)",
        "synth_hbm_frac_step": (sb / (sms * 1e-3)) / PEAK_HBM if sms > 0 else None,
        "spacetime": st,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


DOMINANT_SPLIT_OK = ("gemm_small", "panel", "laswp", "trsm", "assemble", "residual", "getrs",
                     "field", "synth")


def run_spacetime(args, ctx=None, mode=None):
    """Whole space-time path at full size: 2048 frequency solves of the two
    spheres, closest node + field at a grid of points on x = 0 for every
    frequency, and synthesis of four pulses (T = 4096).  Returns one dict with
    the field rate (point x frequency evaluations/s) as the value; the solves
    run in the given mode (default: 3M refinement)."""
    import torch

    from paper_1706_07919_amd import DeviceSurface, native
    from workloads import spacetime_workload

    w = spacetime_workload(n_grid=args.st_grid)
    own_ctx = ctx is None
    if own_ctx:
        ctx = native.Context(0)
    dev = torch.device("cuda:0")
    ds = DeviceSurface.from_bodies(w.bodies)
    n, nk, T = ds.n, len(w.k), w.T
    xp = torch.as_tensor(w.points).to(dev)
    m = xp.shape[0]
    npulse = len(w.pulses)
    U = torch.empty((1, m, nk), dtype=torch.complex64, device=dev)
    p = torch.empty((npulse, m, T), dtype=torch.float32, device=dev)
    i0 = torch.empty(m, dtype=torch.int32, device=dev)
    ins = torch.empty(m, dtype=torch.uint8, device=dev)
    kinds = {"gauss": ["sigma"], "ricker": ["sigma"], "nwave": ["sigma"], "chirp": ["ka", "kb", "D"]}
    c = np.stack([native.bem_pulse_coeffs(pu.kind, [pu.params[q] for q in kinds[pu.kind]], w.dk, nk, T,
                                          w.z_shift) for pu in w.pulses])
    cd = torch.as_tensor(c).to(dev)
    kd = torch.as_tensor(w.k).to(dev)
    y = torch.empty((nk, 1, n), dtype=torch.complex128, device=dev)
    x = torch.zeros((nk, 1, n), dtype=torch.complex128, device=dev)
    phi = torch.empty_like(x)
    psi = torch.empty_like(x)
    opts = native.bem_solve_opts_default()
    opts.mode = mode if mode is not None else native.BEM_FP32_IR_3M

    def stamp():
        torch.cuda.synchronize()
        return time.perf_counter()

    # every input of the timed path (geometry, wavenumbers, points, pulse
    # coefficients) is resident before t0; the solver's workspace is sized by
    # its first call, made here on the same wavenumbers
    native.bem_incident(ctx, ds.struct, nk, kd, (0.0, 0.0, 1.0), y)
    native.bem_solve_batched(ctx, [(ds.struct, nk, kd, 1, y)], opts, [x])
    x.zero_()
    t0 = stamp()
    native.bem_incident(ctx, ds.struct, nk, kd, (0.0, 0.0, 1.0), y)
    info = native.bem_solve_batched(ctx, [(ds.struct, nk, kd, 1, y)], opts, [x])
    native.bem_split_unknowns(ctx, ds.struct, nk, 1, x, y, phi, psi)
    t1 = stamp()
    print(f"{nk} solves: {t1 - t0:.2f} s", file=sys.stderr, flush=True)
    native.bem_field_eval(ctx, ds.struct, nk, kd, 1, phi, psi, m, xp, i0, 0, ins, native.BEM_C64, U)
    t2 = stamp()
    print(f"field {m} x {nk}: {t2 - t1:.2f} s", file=sys.stderr, flush=True)
    native.pulse_synthesize(ctx, m, nk, U[0], npulse, cd, T, 1, xp, w.dk, p)
    t3 = stamp()
    print(f"synthesis: {t3 - t2:.3f} s", file=sys.stderr, flush=True)
    syn_bytes = 8.0 * m * nk + 4.0 * npulse * m * T
    terms = float(m) * nk * n
    # after the timed region: the FP64 residual of every 128th solution, checked
    # independently of the solver's own report
    sel = torch.arange(0, nk, 128, device=dev)
    rr_check = native.bem_residual_check(ctx, ds.struct, int(sel.numel()), kd[sel].contiguous(), 1,
                                         y[sel].contiguous(), x[sel].contiguous())
    out = {"metric": "field pt*freq evals/sec (space-time path at full size)",
           "value": m * nk / (t2 - t1), "unit": "pt*freq/s", "higher_is_better": True,
           "data": "synthetic", "dtype": "c64 field kernel (f64-centred geometry), f32 synthesis",
           "config": {"workload": w.name, "n": n, "n_k": nk, "points": m, "pulses": npulse,
                      "T": T},
           "solve_s": t1 - t0, "solves_per_s": nk / (t1 - t0), "field_s": t2 - t1,
           "field_terms_per_s": terms / (t2 - t1),
           "field_alu_frac": terms * FIELD_VALU_PER_TERM / (t2 - t1) / PEAK_VALU_LANE_OPS,
           "field_alu_note": f"{FIELD_VALU_PER_TERM:.1f} issued VALU instructions per term (one lane "
                             "each) against the FP32 vector peak as lane multiply-adds "
                             "(157.3 TFLOP/s / 2 = 7.87e13/s)",
           "inside_points": int(ins.sum().item()),
           "synthesis_s": t3 - t2, "synthesis_GBps": syn_bytes / (t3 - t2) / 1e9,
           "synthesis_hbm_frac": syn_bytes / (t3 - t2) / PEAK_HBM,
           "ir_iters_max": max(info[q].iters for q in range(nk)),
           "ir_fallbacks": sum(info[q].used_fp64 for q in range(nk)),
           "max_rel_resid": max(info[q].rel_resid for q in range(nk)),
           "min_rel_resid": min(info[q].rel_resid for q in range(nk)),
           "converged": sum(info[q].converged for q in range(nk)),
           "checked_rel_resid_max": float(rr_check.max()),
           "checked_sample": "every 128th wavenumber, bem_residual_check",
           "y_norm": torch.linalg.vector_norm(y).item(), "x_norm": torch.linalg.vector_norm(x).item(),
           "total_s": t3 - t0}
    del U, p, x, y, phi, psi
    if own_ctx:
        ctx.close()
    return out


def run_truncation(args):
    """Dominant-frequency truncation (Sec. IV A, Fig. RMSerror, Table 1): the
    soft unit sphere under the paper's pulse (2 N_c = 4, alpha = 0.1, w = 20.1,
    T = 128, 63 frequencies) rebuilt in space and time on a grid of the x = 0
    plane (the paper's 20 a square) plus the two probe points of Table 1,
    once from all frequencies and once from only the n of largest |c_m|
    (n = 5, 10, 20), each solved on its own.  Times the whole path (incident
    data, solves, field, synthesis) per n; the errors are the table's % RMS at
    the probes and the largest % RMS over the grid points."""
    import torch

    from paper_1706_07919_amd import DeviceSurface, native
    from workloads import Body, SOFT, plane_grid

    W, T, F = 20.1, 128, 63
    dk = 2.0 * np.pi / W
    bodies = [Body((0.0, 0.0, 0.0), 1.0, 1.0, args.tr_level, SOFT)]
    ctx = native.Context(0)
    dev = torch.device("cuda:0")
    ds = DeviceSurface.from_bodies(bodies)
    n = ds.n
    probes = np.array([[0.0, 0.0, -1.1], [0.0, 0.0, -4.0]])
    pts = np.concatenate([probes, plane_grid(args.tr_grid)])
    xp = torch.as_tensor(pts).to(dev)
    m = xp.shape[0]
    c = native.bem_pulse_coeffs("paper", [2.0, 0.1, W], dk, F, T, -(1.0 + W / 4))
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_3M
    i0 = torch.empty(m, dtype=torch.int32, device=dev)
    ins = torch.empty(m, dtype=torch.uint8, device=dev)

    def rebuild(idx):
        nk = len(idx)
        kd = torch.as_tensor(dk * idx.astype(np.float64)).to(dev)
        y = torch.empty((nk, 1, n), dtype=torch.complex128, device=dev)
        x = torch.zeros((nk, 1, n), dtype=torch.complex128, device=dev)
        phi, psi = torch.empty_like(x), torch.empty_like(x)
        U = torch.empty((1, m, nk), dtype=torch.complex64, device=dev)
        p = torch.empty((1, m, T), dtype=torch.float32, device=dev)
        cs = torch.as_tensor(np.ascontiguousarray(c[idx - 1])[None, :]).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        native.bem_incident(ctx, ds.struct, nk, kd, (0.0, 0.0, 1.0), y)
        info = native.bem_solve_batched(ctx, [(ds.struct, nk, kd, 1, y)], opts, [x])
        native.bem_split_unknowns(ctx, ds.struct, nk, 1, x, y, phi, psi)
        native.bem_field_eval(ctx, ds.struct, nk, kd, 1, phi, psi, m, xp, i0, 0, ins,
                              native.BEM_C64, U)
        native.pulse_synthesize_sparse(ctx, m, idx, U[0], 1, cs, T, 0, xp, dk, p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert all(info[q].converged == 1 for q in range(nk))
        return p[0].cpu().numpy().astype(np.float64), dt

    all_idx = np.arange(1, F + 1, dtype=np.int32)
    rebuild(all_idx)                     # warm-up (first launches, allocations)
    full, t_full = rebuild(all_idx)
    outside = ins.cpu().numpy() == 0
    res = {}
    for nkeep in (5, 10, 20):
        idx = native.bem_pulse_dominant(c, nkeep)
        tr, dt = rebuild(idx)
        err = np.sqrt(np.mean((tr - full) ** 2, axis=1)) / np.maximum(np.max(np.abs(full), axis=1), 1e-30)
        grid = err[2:][outside[2:]]
        res[str(nkeep)] = {"s": dt, "speedup": t_full / dt,
                           "rms_percent_z_-1.1": 100 * err[0], "rms_percent_z_-4": 100 * err[1],
                           "grid_median_rms_percent": 100 * float(np.median(grid)),
                           "grid_max_rms_percent": 100 * float(np.max(grid))}
        print(f"top {nkeep}: {dt:.3f} s, probes {100 * err[0]:.2f}% / {100 * err[1]:.2f}%",
              file=sys.stderr, flush=True)
    out = {"metric": "space-time reconstruction from the 10 dominant of 63 frequencies, speedup",
           "value": res["10"]["speedup"], "unit": "x vs all frequencies", "higher_is_better": True,
           "data": "synthetic", "dtype": "c64 factors refined to f64, c64 field, f32 synthesis",
           "config": {"workload": f"paper soft sphere, level {args.tr_level}", "n": n, "n_k": F,
                      "T": T, "points": m},
           "all_frequencies_s": t_full, "truncated": res,
           "table1_printed": {"5": [4.4, 4.9], "10": [1.6, 1.7], "20": [0.5, 0.6]}}
    print(json.dumps(out))


def run_quadratic(args):
    """The paper's quadratic-element sphere (Sec. IV A: 500 six-node elements,
    1002 nodes, sound-soft) under its pulse (2 N_c = 4, alpha = 0.1, w = 20.1,
    63 frequencies, T = 128): incident data, element-quadrature assembly and
    the float32 3M solve refined against the float64 operator, the field by
    element quadrature on the paper's 80 x 80 grid over the 20 a square of the
    x = 0 plane, and the synthesis.  Times the whole path (after one untimed
    pass) and reports the assembly and field kernels' rates."""
    import torch

    from paper_1706_07919_amd import DeviceQuadSurface, native
    from workloads import Body, SOFT, plane_grid

    W, T, F = 20.1, 128, 63
    dk = 2.0 * np.pi / W
    body = Body((0.0, 0.0, 0.0), 1.0, 1.0, 0, SOFT)
    qs = DeviceQuadSurface.from_body(body, 5)
    n = qs.n
    ctx = native.Context(0)
    dev = torch.device("cuda:0")
    # the nodal struct for incident data and the split of the unknowns (their
    # kernels read no weights)
    ns = native.surface_struct(n, qs.x, qs.nrm, qs.x, qs.bc)
    k = dk * np.arange(1, F + 1)
    kd = torch.as_tensor(k).to(dev)
    pts = plane_grid(80)
    xp = torch.as_tensor(pts).to(dev)
    m = len(pts)
    c = native.bem_pulse_coeffs("paper", [2.0, 0.1, W], dk, F, T, -(1.0 + W / 4))
    cd = torch.as_tensor(c[None, :]).to(dev)
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_3M
    y = torch.empty((F, 1, n), dtype=torch.complex128, device=dev)
    x = torch.zeros_like(y)
    phi, psi = torch.empty_like(y), torch.empty_like(y)
    U = torch.empty((1, m, F), dtype=torch.complex128, device=dev)
    U32 = torch.empty((1, m, F), dtype=torch.complex64, device=dev)
    p = torch.empty((1, m, T), dtype=torch.float32, device=dev)
    i0 = torch.empty(m, dtype=torch.int32, device=dev)
    ins = torch.empty(m, dtype=torch.uint8, device=dev)
    marks = {}

    def run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        native.bem_incident(ctx, ns, F, kd, (0.0, 0.0, 1.0), y)
        info = native.bem_solve_quadratic(ctx, qs.struct, F, kd, 1, y, opts, x)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        native.bem_split_unknowns(ctx, ns, F, 1, x, y, phi, psi)
        native.bem_field_eval_quadratic(ctx, qs.struct, F, kd, 1, phi, psi, m, xp, i0, ins, U)
        U32.copy_(U)
        native.pulse_synthesize(ctx, m, F, U32[0], 1, cd, T, 1, xp, dk, p)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        marks.update(solve=t1 - t0, rest=t2 - t1)
        return info

    run()
    ctx.set_profiling_filter(("assemble_quad", "field_quad"))
    ctx.set_profiling(True)
    info = run()
    fa = ctx.kernel_stats("assemble_quad")
    ff = ctx.kernel_stats("field_quad")
    ctx.set_profiling(False)
    # about 60 float64 operations per kernel value (distance, sincos, G, dG/dn
    # and the f, g terms of the diagonal integrals)
    out = {"metric": "quadratic elements (500 el, 1002 nodes): whole-path time, 63 frequencies",
           "value": marks["solve"] + marks["rest"], "unit": "s", "higher_is_better": False,
           "data": "synthetic",
           "dtype": "f64 element-quadrature assembly, c64 LU (3M on f32 MFMA) refined to f64, f64 field",
           "config": {"workload": "paper soft sphere, quadratic elements nu = 5", "n": n,
                      "elements": qs.n_elem, "n_k": F, "T": T, "points": m},
           "solves_per_s": F / marks["solve"], "solve_s": marks["solve"],
           "field_and_synthesis_s": marks["rest"],
           "assemble_quad_ms": fa[2], "assemble_kernel_values_per_s": fa[0] / (fa[2] * 1e-3),
           "assemble_f64_frac_est": 60.0 * fa[0] / (fa[2] * 1e-3) / 78.6e12,
           "field_quad_ms": ff[2], "field_pt_freq_per_s": m * F / (ff[2] * 1e-3),
           "ir_iters_max": max(info[q].iters for q in range(F)),
           "ir_fallbacks": sum(info[q].used_fp64 for q in range(F)),
           "max_rel_resid": max(info[q].rel_resid for q in range(F))}
    print(json.dumps(out))


def run_chief(args):
    """The remedy for fictitious resonances on a hard unit sphere (level 4,
    2562 nodes) under the plane wave: the six interior eigenvalues below 8
    and six wavenumbers between them, 16 interior points.  Times the plain
    solve (FP32 3M LU refined to FP64) and the least-squares solve with the
    interior rows (FP64 normal equations) and reports how far the plain
    solution moves when the interior rows are added: tens of per cent at the
    eigenvalues (the spurious interior mode), the discretisation error between
    them."""
    import torch

    from paper_1706_07919_amd import DeviceSurface, native
    from workloads import Body, HARD, SPHERE_RESONANCES, interior_points

    body = Body((0.0, 0.0, 0.0), 1.0, 1.0, 4, HARD)
    ds = DeviceSurface.from_bodies([body])
    n = ds.n
    res = np.array(SPHERE_RESONANCES)
    off = np.array([2.5, 3.8, 5.1, 6.0, 6.6, 7.4])
    k = np.concatenate([res, off])
    n_k = len(k)
    xc = interior_points([body], 16, seed=3)
    dev = torch.device("cuda:0")
    ctx = native.Context(0)
    kd = torch.as_tensor(k).to(dev)
    xcd = torch.as_tensor(xc).to(dev)
    y = torch.empty((n_k, 1, n), dtype=torch.complex128, device=dev)
    native.bem_incident(ctx, ds.struct, n_k, kd, (0.0, 0.0, 1.0), y)
    xp = torch.zeros_like(y)
    xl = torch.zeros_like(y)
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_3M

    def plain():
        xp.zero_()
        return native.bem_solve_batched(ctx, [(ds.struct, n_k, kd, 1, y)], opts, [xp])

    def remedied():
        return native.bem_solve_chief(ctx, ds.struct, n_k, kd, 1, y, len(xc), xcd, xl)

    plain()
    remedied()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info_p = plain()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info_c = remedied()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    d = (torch.linalg.vector_norm(xp - xl, dim=(1, 2)) / torch.linalg.vector_norm(xl, dim=(1, 2))).cpu().numpy()
    out = {"metric": "interior-point least-squares solves/sec at N=2562 (hard sphere at and between "
                     "interior eigenvalues)",
           "value": n_k / (t2 - t1), "unit": "freq-solves/s", "higher_is_better": True,
           "data": "synthetic", "dtype": "c128 normal equations (rocBLAS zgemm) + f64-MFMA LU",
           "config": {"workload": "hard unit sphere, level 4", "n": n, "n_k": n_k,
                      "interior_points": len(xc), "k_resonant": res.tolist(), "k_between": off.tolist()},
           "plain_solves_per_s": n_k / (t1 - t0),
           "plain_vs_remedied_rel_diff_at_eigenvalues": d[:len(res)].tolist(),
           "plain_vs_remedied_rel_diff_between": d[len(res):].tolist(),
           "plain_ir_iters": [info_p[q].iters for q in range(n_k)],
           "plain_fallbacks": sum(info_p[q].used_fp64 for q in range(n_k)),
           "least_squares_rel_resid": [info_c[q].rel_resid for q in range(n_k)]}
    print(json.dumps(out))


def run_bowl(args):
    """The hard axisymmetric bowl of Sec. IV C (Eq. dish; axis turned by
    0.15 pi from the propagation direction +z; 48 x 96 rings, 4514 nodes)
    under the paper's pulse with 2 N_c = 6 cycles, alpha = 0.001, w = 20.1
    (63 frequencies, T = 128): the total field on a 192 x 192 grid of the
    x = 0 plane, y, z in [-3, 3].  Reports the whole-path time and the
    focusing gain, the largest |p| over the grid and the 128 time samples
    relative to the incident pulse's peak (the paper quotes about 4.5; this is
    a check of the physics, not of parity)."""
    import torch

    from paper_1706_07919_amd import DeviceSurface, native

    W, T, F = 20.1, 128, 63
    dk = 2.0 * np.pi / W
    tilt = 0.15 * np.pi
    nr_ = args.bowl_rings
    x, nrm, w, _ = native.bem_mesh_bowl(nr_, 2 * nr_, 1.0, tilt, (0.0, 0.0, 0.0))
    bc = np.zeros(len(x), dtype=np.uint8)
    ctx = native.Context(0)
    dev = torch.device("cuda:0")
    ds = DeviceSurface(x, nrm, w, bc)
    n = ds.n
    g = (np.arange(192) + 0.5) / 192 * 6.0 - 3.0
    Y, Z = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([np.zeros(Y.size), Y.ravel(), Z.ravel()], axis=1)
    xp = torch.as_tensor(pts).to(dev)
    m = len(pts)
    params = [3.0, 0.001, W]
    zs = -(1.0 + W / 4)
    c = native.bem_pulse_coeffs("paper", params, dk, F, T, zs)
    k = dk * np.arange(1, F + 1)
    kd = torch.as_tensor(k).to(dev)
    cd = torch.as_tensor(c[None, :]).to(dev)
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_3M
    y = torch.empty((F, 1, n), dtype=torch.complex128, device=dev)
    xs = torch.zeros_like(y)
    phi, psi = torch.empty_like(y), torch.empty_like(y)
    U = torch.empty((1, m, F), dtype=torch.complex64, device=dev)
    p = torch.empty((1, m, T), dtype=torch.float32, device=dev)
    i0 = torch.empty(m, dtype=torch.int32, device=dev)
    ins = torch.empty(m, dtype=torch.uint8, device=dev)

    def run():
        xs.zero_()
        native.bem_incident(ctx, ds.struct, F, kd, (0.0, 0.0, 1.0), y)
        info = native.bem_solve_batched(ctx, [(ds.struct, F, kd, 1, y)], opts, [xs])
        native.bem_split_unknowns(ctx, ds.struct, F, 1, xs, y, phi, psi)
        native.bem_field_eval(ctx, ds.struct, F, kd, 1, phi, psi, m, xp, i0, 0, ins,
                              native.BEM_C64, U)
        native.pulse_synthesize(ctx, m, F, U[0], 1, cd, T, 1, xp, dk, p)
        return info

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out_mask = ins.cpu().numpy() == 0
    P = p[0].cpu().numpy()[out_mask]
    # incident peak from the same synthesis with no scatterer
    p0 = torch.empty((1, 1, T), dtype=torch.float32, device=dev)
    native.pulse_synthesize(ctx, 1, F, torch.zeros((1, F), dtype=torch.complex64, device=dev), 1,
                            cd, T, 1, torch.zeros((1, 3), dtype=torch.float64, device=dev), dk, p0)
    inc_peak = float(np.max(np.abs(p0.cpu().numpy())))
    gain = float(np.max(np.abs(P))) / inc_peak
    out = {"metric": "hard acoustic bowl: space-time focusing gain (max |p| / incident peak)",
           "value": gain, "unit": "x incident peak", "higher_is_better": True,
           "data": "synthetic", "dtype": "c64 factors refined to f64, c64 field, f32 synthesis",
           "config": {"workload": f"paper acoustic bowl, {nr_} x {2 * nr_} rings, tilt 0.15 pi", "n": n,
                      "n_k": F, "T": T, "points": m},
           "paper_gain": 4.5, "whole_path_s": dt, "solves_per_s": F / dt,
           "ir_iters_max": max(info[q].iters for q in range(F)),
           "ir_fallbacks": sum(info[q].used_fp64 for q in range(F)),
           "max_rel_resid": max(info[q].rel_resid for q in range(F)),
           "inside_points": int((~out_mask).sum())}
    print(json.dumps(out))


def run_uneven(args):
    """Eight independent scatterers of uneven size (spheres and prolate
    spheroids, 642 / 2562 / 10242 nodes, hard and soft) solved in one batched
    call, 1024 wavenumbers each by default: the solver takes them in rounds
    that fit the device, and every launch of a round covers all matrices of
    all sizes.  One JSON line: solves/s over the whole call (one timed pass
    after a short untimed pass that sizes the workspace)."""
    import torch

    from paper_1706_07919_amd import DeviceSurface, native
    from workloads import uneven_bodies_workload

    w = uneven_bodies_workload(n_k=args.uneven_k)
    nk = len(w.k)
    ctx = native.Context(0)
    dev = torch.device("cuda:0")
    kd = torch.as_tensor(w.k).to(dev)
    probs, xs, surfs = [], [], []
    for b in w.bodies:
        ds = DeviceSurface.from_bodies([b])
        y = torch.empty((nk, 1, ds.n), dtype=torch.complex128, device=dev)
        native.bem_incident(ctx, ds.struct, nk, kd, (0.0, 0.0, 1.0), y)
        surfs.append(ds)
        probs.append((ds.struct, nk, kd, 1, y))
        xs.append(torch.zeros((nk, 1, ds.n), dtype=torch.complex128, device=dev))
    mode = {"b3": native.BEM_FP32_IR_B3, "4m": native.BEM_FP32_IR_4M, "3m": native.BEM_FP32_IR_3M}[args.mode]
    gk = {"b3": native.BEM_GEMM_BF16X3, "4m": native.BEM_GEMM_4M, "3m": native.BEM_GEMM_3M}[args.mode]
    opts = native.bem_solve_opts_default()
    opts.mode = mode
    plans = None
    if args.autotune > 0:
        # the batch is planned by its largest size class
        nmax = max(ds.n for ds in surfs)
        native.bem_autotune_lu(ctx, native.BEM_C64, nmax, args.autotune, gk)
        plans = {"n": nmax, "kept": native.bem_lu_tuned_plan(ctx, native.BEM_C64, nmax, gk),
                 "log": native.bem_autotune_lu_results(ctx)}
    # untimed pass on the first 16 wavenumbers of every body (first launches,
    # workspace)
    small = [(s_, 16, k_[:16], 1, y_[:16]) for (s_, _, k_, _, y_) in probs]
    native.bem_solve_batched(ctx, small, opts, [x_[:16] for x_ in xs])
    torch.cuda.synchronize()
    steps = max(1, args.uneven_steps)
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        infos.append(native.bem_solve_batched(ctx, probs, opts, xs))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info = infos[-1]
    tot = len(w.bodies) * nk
    sizes = [ds.n for ds in surfs]
    flops = sum(8.0 * n ** 3 / 3.0 * nk for n in sizes)
    out = {"metric": "uneven batch: frequency solves/s (8 bodies, N in {642, 2562, 10242})",
           "value": tot / dt, "unit": "freq-solves/s", "higher_is_better": True,
           "steps": steps, "ms_per_step": 1e3 * dt,
           "data": "synthetic", "dtype": "c64 LU (" + args.mode + " on f32 MFMA) + f64 residual refinement",
           "config": {"workload": w.name, "sizes": sizes, "k_per_body": nk,
                      "mode": args.mode},
           "autotune": plans,
           "lu_algorithmic_tflops": flops / dt / 1e12,
           "ir_iters_max": max(info[q].iters for q in range(len(info))),
           "ir_fallbacks": sum(info[q].used_fp64 for q in range(len(info))),
           "max_rel_resid": max(info[q].rel_resid for q in range(len(info)))}
    print(json.dumps(out))


def run_surrogate(args):
    """Gain test of the learned fill (one JSON line): the 4096-wavenumber sweep
    of the two-sphere workload solved (i) directly, (ii) from 256 direct
    training solves + network prediction + FP64 residual check + refinement
    with the nearest training factors + direct fallback, (iii) as (ii) without
    the network (refinement from zero).  All three reach the same FP64-residual
    tolerance; times are whole-path wall clock with inputs resident."""
    import torch

    from paper_1706_07919_amd import DeviceSurface, native
    from paper_1706_07919_amd import surrogate as sg
    from workloads import surrogate_workload, surrogate_train_k

    w = surrogate_workload()
    k_train = surrogate_train_k(256)
    k_pred = w.k
    ctx = native.Context(0)
    ds = DeviceSurface.from_bodies(w.bodies)
    n, nkp = ds.n, len(k_pred)
    dev = torch.device("cuda:0")
    kp = torch.as_tensor(k_pred).to(dev)
    yp = torch.empty((nkp, 1, n), dtype=torch.complex128, device=dev)
    native.bem_incident(ctx, ds.struct, nkp, kp, (0.0, 0.0, 1.0), yp)
    opts = native.bem_solve_opts_default()
    opts.mode = native.BEM_FP32_IR_3M
    x_dir = torch.zeros((nkp, 1, n), dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    native.bem_solve_batched(ctx, [(ds.struct, nkp, kp, 1, yp)], opts, [x_dir])
    torch.cuda.synchronize()
    t_direct = time.perf_counter() - t0
    print(f"direct solves of {nkp} wavenumbers: {t_direct:.2f} s", file=sys.stderr, flush=True)
    out = {"metric": "surrogate fill of 4096 wavenumbers at N=5124: wall time vs direct",
           "unit": "s", "higher_is_better": False, "data": "synthetic",
           "config": {"workload": w.name, "n": n, "n_train": len(k_train), "n_pred": nkp,
                      "hidden": [512] * 4, "acceptance_tol": 1e-6},
           "direct_s": t_direct}
    for name, use in (("surrogate", True), ("zero_start", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = sg.fill_sweep(ctx, ds, k_train, k_pred, hidden=(512, 512, 512, 512),
                            epochs=args.sur_epochs, lr=1e-3, tol=1e-6, refine_tol=1e-8,
                            max_sweeps=args.sur_sweeps, use_surrogate=use)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        print(f"{name}: {total:.2f} s", file=sys.stderr, flush=True)
        err = (torch.linalg.vector_norm(res["x"] - x_dir, dim=(1, 2)) /
               torch.linalg.vector_norm(x_dir, dim=(1, 2))).max().item()
        rr = native.bem_residual_check(ctx, ds.struct, nkp, kp, 1, res["y"], res["x"])
        out[name] = {"total_s": total, "train_solves_s": res["t_train_solves"],
                     "fit_s": res["t_fit"], "fill_s": res["t_fill"],
                     "accepted_as_predicted": res["accepted_as_predicted"],
                     "refined": res["refined"], "fallback": res["fallback"],
                     "sweeps_mean": res["sweeps_mean"], "sweeps_max": res["sweeps_max"],
                     "median_prediction_residual": float(np.median(res["rel_resid_prediction"])),
                     "max_rel_err_vs_direct": err, "max_rel_resid": float(rr.max()),
                     "n_oct": res["n_oct"]}
        if use:
            out[name]["final_loss"] = res["loss"][-1][1] if res.get("loss") else None
        del res
    out["value"] = out["surrogate"]["total_s"]
    out["gain_vs_direct"] = t_direct / out["surrogate"]["total_s"]
    out["gain_vs_zero_start"] = out["zero_start"]["total_s"] / out["surrogate"]["total_s"]
    print(json.dumps(out))


# lu.hip section (from its header to the next) holding each profiled kernel
KERNEL_SECTIONS = {
    "gemm_3m": ("GEMM f32, operands streamed into LDS", "GEMM f32 via bf16 split\n"),
    "gemm_c32": ("GEMM f32, operands streamed into LDS", "GEMM f32 via bf16 split\n"),
    "gemm_b3_packed": ("GEMM f32 via bf16 split, packed operands", "GEMM f64"),
}


def kernel_source_sha256(kernel="gemm_3m"):
    """Hash of the kernel's source section of lu.hip (its block comment,
    helpers and kernels, up to the next section header)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_1706_07919_amd", "csrc", "lu.hip")).read()
    head = "// ============================================================== "
    first, last = KERNEL_SECTIONS[kernel]
    a = src.index(head + first)
    b = src.index(head + last)
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def measured_traffic(kernel, block_width="default", alg_bytes_per_launch=None, profiles=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none, the kernel's source changed since the
    counters were taken, or the factorisation's block width or the mix of
    launch sizes differs (the mix is identified by the algorithmic bytes per
    launch, which every step of the sweep repeats)."""
    path = os.path.join(profiles or os.path.join(ROOT, "profiles"),
                        f"pmc_{kernel}_two_spheres_N5124_nk512.txt")
    if not os.path.exists(path) or kernel not in KERNEL_SECTIONS:
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            key, _, val = line.partition(":")
            vals[key.strip()] = val.strip()
    if vals.get("kernel_source_sha256") != kernel_source_sha256(kernel) or \
            vals.get("block_width") != str(block_width) or "traffic_bytes_per_launch" not in vals:
        return None
    if alg_bytes_per_launch is not None:
        ref = float(vals.get("algorithmic_bytes_per_launch", "nan"))
        if not abs(alg_bytes_per_launch - ref) <= 1e-3 * ref:
            return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(w, x_gpu, n_cpu_k):
    """The FP64 oracle (numpy/scipy assembly + LAPACK LU) timed on the host for
    a bounded sample of the same workload: n_cpu_k wavenumbers spread over the
    sweep at N = 5124, each compared with the GPU result."""
    from oracle import bie
    from oracle.mesh import Surface
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    s = Surface(w.bodies)
    idx = np.linspace(0, len(w.k) - 1, n_cpu_k).round().astype(int)
    errs = []
    t0 = time.perf_counter()
    for q in idx:
        p, dp = bie.incident_plane_wave(s, w.k[q])
        yq = bie.known_data(s, p, dp)
        _, _, xs = bie.solve(s, w.k[q], yq)
        xg = x_gpu[q, 0].cpu().numpy()
        errs.append(float(np.linalg.norm(xg - xs) / np.linalg.norm(xs)))
    dt = time.perf_counter() - t0
    return {"value": len(idx) / dt, "unit": "freq-solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(idx)} wavenumbers k={','.join(f'{w.k[q]:.4g}' for q in idx)} "
                      f"of the same N=5124 workload, FP64 assembly + LAPACK LU ({dt:.1f} s)",
            "gpu_rel_err_vs_oracle": max(errs),
            "gpu_rel_err_vs_oracle_per_k": errs}


if __name__ == "__main__":
    main()
