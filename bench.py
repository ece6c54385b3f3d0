"""Benchmark: voxel-frequencies inverted per second on one MI355X.

One step = one fl_invert call (the whole hot path: FFT of the data,
classification and regularized solves of every (frequency, wavenumber)
system, inverse FFT, zero-padded 3D convolution, xi) over one batch of
synthetic input that is already resident in HBM.

Prints one JSON line. Default workload: the 128x128x64 single-frequency grid
(256x256 torus, 64 data planes, omega = 2 pi, delta = 0.01, Born data from a
3-blob contrast). The roofline block describes the kernel that takes the most
time in the timed region, its duration measured with HIP events recorded on
the plan's stream around every stage.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0
PEAK_FP64_VALU_TFLOPS = 78.6  # 256 CUs x 2.4 GHz x 128 FP64 flop/clk/CU

WORKLOAD_TEXT = {
    "single": "128x128x64 X, 256x256 torus, 64 data planes, omega=2pi, 3 blobs",
    "multi5": "128x128x64 X, 256x256 torus, 64 data planes, omega=2pi*{0.5..2.5}, 5 blobs",
    "small": "32x32x16 X, 64x64 torus, 16 data planes, omega=2pi, 3 blobs",
}


def stage_units(p, active, factorized, n, b=16):
    """Algorithmic work per timed step and stage: HBM bytes that the stage
    must move at least (b bytes per complex element of the FFT-side arrays,
    16 for the complex128 input W, the FP64 v, u, u0 and xi), or FP64 flops.
    active: systems solved; factorized: matrices bidiagonalized (one per
    active symmetry orbit when factorizations are shared)."""
    F, N, nd, nz = p.n_omega, p.px * p.py, p.nd, p.nz
    nvox = p.nx * p.ny * p.nz
    rows_y = F * nz * p.ny * p.px      # rows of X's y-window on the padded x axis
    planes_n = F * nz * N              # one value per (f, z, system)
    u = {
        "norm": ("GB/s", F * nd * N * 16),
        "fft_rows": ("GB/s", F * nd * N * (16 + b)),
        "fft_cols": ("GB/s", 2 * F * nd * N * b),
        # read W^, write ||w||^2 and flags, read flags twice, write the list,
        # zero v^
        "classify": ("GB/s", F * nd * N * b + F * N * (8 + 4 * 3) + active * 4 + planes_n * b),
        "ifft_cols": ("GB/s", planes_n * b + rows_y * b),
        "crop_pad": ("GB/s", rows_y * b + F * nvox * 16 + rows_y * b),
        "conv_cols": ("GB/s", rows_y * b + planes_n * b),
        # read the nz nonzero z samples and the 2 nz kernel values, write nz
        "conv_z": ("GB/s", planes_n * b + 2 * planes_n * b + planes_n * b),
        "conv_icols": ("GB/s", planes_n * b + rows_y * b),
        "conv_irows": ("GB/s", rows_y * b + 2 * F * nvox * 16),
        "xi": ("GB/s", 2 * F * nvox * 16 + nvox * 16),
        # complex Householder bidiagonalization of an n x n matrix: 4 x (8/3) n^3
        "bidiag": ("TFLOP/s", factorized * 32.0 / 3.0 * n ** 3),
        # per system: 3 search rounds x 16 trial alphas (four systems share
        # a wave, one per 16-lane group) x 20 flops per row of the
        # discrepancy recurrence, q = U^H w and v^ = V y (8 n^2 flops each),
        # the bidiagonal Tikhonov solve (about 40 n)
        "dp": ("TFLOP/s", active * (3 * 16 * 20.0 * n + 16.0 * n * n + 40.0 * n)),
        "backtransform": ("GB/s", 0),
    }
    return u


FFT_STAGES = ("fft_rows", "fft_cols", "ifft_cols", "crop_pad", "conv_cols", "conv_z",
              "conv_icols", "conv_irows")


PROFILE_COUNTERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                "counters_single_128x128x64.json")


def profiled_traffic(workload, prec, kernel):
    """HBM bytes per dispatch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE profile of this workload (already scaled by the calibration
    factors), or None when there is none or the HIP sources changed since."""
    from paper_1911_10487_amd.build import source_sha256
    if workload != "single" or not os.path.exists(PROFILE_COUNTERS):
        return None
    with open(PROFILE_COUNTERS) as fh:
        js = json.load(fh)
    if js.get("source_sha256") != source_sha256():
        return None
    k = js.get("kernels", {}).get("mixed" if prec else "fp64", {}).get(kernel)
    if not k:
        return None
    return {"bytes": k["fetch_bytes"] + k["write_bytes"], "fetch_bytes": k["fetch_bytes"],
            "write_bytes": k["write_bytes"], "profiled_avg_us": k["avg_us"]}


def cpu_baseline(p, Wd, u0, delta, vf):
    from threadpoolctl import threadpool_info

    from oracle import invert
    t0 = time.perf_counter()
    xi = invert.invert(p, Wd, u0, delta)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return ({"value": vf / dt, "unit": "voxel-freq/s", "cores": int(threads), "kind": "oracle",
             "sample": f"the whole workload once ({vf} voxel-frequencies), NumPy FP64 oracle, "
                       f"{dt:.1f} s; LAPACK SVDs on {threads} threads, FFTs single-threaded"}, xi)


def _event_ms(torch, fn, reps, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_variants(p, Wd, u0, delta, args, torch, dev):
    """Secondary figures on the same data, none of them the headline: the
    derivatives of W -> xi (one VJP, one JVP, one power-iteration step =
    JVP + VJP; per-system factorizations, as the derivative path needs), and
    the inversion with the truncated-SVD regularizer."""
    from paper_1911_10487_amd.autograd import power_iteration
    from paper_1911_10487_amd.flayer import Plan
    out = {}
    vf = p.voxel_frequencies
    for label, prec in (("fp64", 0), ("mixed", 1)):
        plan = Plan.from_problem(p, precision=prec)
        g = torch.randn((p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        dW = torch.randn(Wd.shape, dtype=Wd.dtype, device=dev)
        t_vjp = _event_ms(torch, lambda: plan.vjp(Wd, u0, delta, g), args.steps)
        t_jvp = _event_ms(torch, lambda: plan.jvp(Wd, u0, delta, dW), args.steps)
        power_iteration(plan, Wd, u0, delta, iters=1)  # warm-up (library set-up)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        est, _ = power_iteration(plan, Wd, u0, delta, iters=5)
        torch.cuda.synchronize()
        t_pi = (time.perf_counter() - t0) * 1e3 / 5
        plan.close()
        tplan = Plan.from_problem(p, precision=prec, regularizer=1)
        xi = torch.empty((p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        t_tsvd = _event_ms(torch, lambda: tplan.invert(Wd, u0, delta, xi), args.steps)
        tplan.close()
        out[label] = {"vjp_ms": t_vjp, "jvp_ms": t_jvp, "power_iteration_ms_per_step": t_pi,
                      "power_iteration_sigma_after_5": est[-1],
                      "tsvd_ms_per_step": t_tsvd, "tsvd_value": vf / (t_tsvd * 1e-3)}
        print(f"[bench] {label}: vjp {t_vjp:.3f} ms, jvp {t_jvp:.3f} ms, power step "
              f"{t_pi:.3f} ms, tsvd inversion {t_tsvd:.3f} ms", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="single", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--delta", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="time one precision only (profiling runs)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the solver schedule on the data before timing (the "
                         "default schedule is the tuner's choice for this workload)")
    ap.add_argument("--no-prefactor", action="store_true",
                    help="skip the secondary timing of plans that factorize every matrix at "
                         "plan creation")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the secondary timings of the derivatives and of the TSVD "
                         "regularizer")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing "
                         "(a known-size kernel for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the inversion runs on a single GPU; --gpus {args.gpus} is not "
              "supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1911_10487_amd import synth
    from paper_1911_10487_amd.flayer import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    p = synth.workload(args.workload)[0]
    delta = p.deltas[0] if args.delta is None else args.delta
    print(f"[bench] workload {args.workload} delta={delta}", file=sys.stderr, flush=True)

    xi_true = torch.from_numpy(synth.contrast(p)).to(dev)
    u0_np = synth.incident_field(p)
    u0 = torch.from_numpy(u0_np).to(dev)
    gen = Plan.from_problem(p)
    # total-field data: BiCGSTAB on u - omega^2 K(xi u) = u0 to 1e-12, then
    # the data operator (the generator of the 32x32x16 configuration)
    W = gen.forward(xi_true, u0, maxit=500, tol=1e-12)
    torch.cuda.synchronize()
    gen.close()
    Wd_np = synth.add_noise(p, W.cpu().numpy(), delta)
    Wd = torch.from_numpy(Wd_np).to(dev)
    del W

    if args.calibrate_copy_mb:
        # known-size kernels: a fill (writes nb bytes), a sum (reads nb bytes)
        # and an out-of-place copy (reads and writes nb bytes)
        nb = args.calibrate_copy_mb << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        s = src.sum()
        dst = src * 1.0
        torch.cuda.synchronize()
        print(f"[bench] calibration kernels over {nb} bytes (sum {float(s):.0f})", file=sys.stderr,
              flush=True)
        del src, dst

    runs = {}
    precs = (("fp64", 0), ("mixed", 1))
    if args.only:
        precs = tuple(x for x in precs if x[0] == args.only)
    for label, prec in precs:
        runs[label] = time_precision(p, prec, Wd, u0, delta, args, torch, dev)
        print(f"[bench] {label}: {runs[label]['ms']:.3f} ms/step", file=sys.stderr, flush=True)
    if args.only:
        r = runs[args.only]
        print(json.dumps({"metric": "voxel-frequencies inverted/s", "precision": args.only,
                          "value": p.voxel_frequencies / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
                          "schedule": r["tuning"], "roofline": r["roofline"],
                          "fft_stages": r["fft_stages"], "hbm_stages": r["hbm_stages"],
                          "stages_ms_per_step": r["stages"]}), flush=True)
        return
    pre = None
    if not args.no_prefactor:
        # secondary figure, not the headline: A_m does not depend on the data,
        # so a plan can factorize every matrix once (prefactor = 1) and each
        # inversion then only classifies and solves
        r = time_precision(p, 1, Wd, u0, delta, args, torch, dev, prefactor=1)
        pre = {"value": p.voxel_frequencies / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
               "plan_ms": r["plan_ms"], "precision": "mixed",
               "xi_rel_l2_vs_per_call": float(np.linalg.norm(r["xi"] - runs["mixed"]["xi"])
                                              / np.linalg.norm(runs["mixed"]["xi"])),
               "stages_ms_per_step": r["stages"]}
        print(f"[bench] mixed, plan-time factorization: {r['ms']:.3f} ms/step", file=sys.stderr,
              flush=True)
    variants = None
    if not args.no_variants:
        variants = time_variants(p, Wd, u0, delta, args, torch, dev)
    xi64 = runs["fp64"]["xi"]
    ximx = runs["mixed"]["xi"]
    mixed_vs_fp64 = float(np.linalg.norm(ximx - xi64) / np.linalg.norm(xi64))

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu, xi_ref = cpu_baseline(p, Wd_np, u0_np, delta, p.voxel_frequencies)
        for r in runs.values():
            r["vs_oracle"] = float(np.linalg.norm(r["xi"] - xi_ref) / np.linalg.norm(xi_ref))
    # headline: the mixed path when it meets the 1e-4 gate, else FP64
    ok = mixed_vs_fp64 <= 1e-4 and runs["mixed"].get("vs_oracle", 0.0) <= 1e-4
    head = "mixed" if ok and runs["mixed"]["ms"] < runs["fp64"]["ms"] else "fp64"
    h = runs[head]
    vf = p.voxel_frequencies
    out = {
        "metric": "voxel-frequencies inverted/s",
        "value": vf / (h["ms"] * 1e-3),
        "unit": "voxel-freq/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 FFT/convolution + f64 solve and division" if head == "mixed" else "f64",
        "data": "synthetic: total-field data (GPU BiCGSTAB, tol 1e-12) of seeded Gaussian "
                "blobs, seeded complex noise of relative level delta",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}",
                   "delta": delta, "precision": head, "active_systems": h["active"],
                   "factorized_systems": h["factorized"],
                   "systems": p.n_omega * p.px * p.py, "n": p.nz, "plan_ms": h["plan_ms"],
                   "tune_ms": h["tune_ms"], "schedule": h["tuning"]},
        "roofline": h["roofline"],
        "fft_stages": h["fft_stages"],
        "hbm_stages": h["hbm_stages"],
        "stages_ms_per_step": h["stages"],
        "fp64": {"value": vf / (runs["fp64"]["ms"] * 1e-3), "ms_per_step": runs["fp64"]["ms"],
                 "xi_rel_l2_vs_oracle": runs["fp64"].get("vs_oracle"),
                 "schedule": runs["fp64"]["tuning"], "fft_stages": runs["fp64"]["fft_stages"],
                 "roofline": runs["fp64"]["roofline"]},
        "mixed": {"value": vf / (runs["mixed"]["ms"] * 1e-3), "ms_per_step": runs["mixed"]["ms"],
                  "xi_rel_l2_vs_fp64_gpu": mixed_vs_fp64,
                  "xi_rel_l2_vs_oracle": runs["mixed"].get("vs_oracle"),
                  "schedule": runs["mixed"]["tuning"], "fft_stages": runs["mixed"]["fft_stages"],
                  "roofline": runs["mixed"]["roofline"]},
    }
    if pre is not None:
        out["prefactored_plan"] = pre
    if variants is not None:
        out["variants"] = variants
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def time_precision(p, prec, Wd, u0, delta, args, torch, dev, prefactor=0):
    from paper_1911_10487_amd.flayer import Plan
    t0 = time.perf_counter()
    plan = Plan.from_problem(p, precision=prec, prefactor=prefactor)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)
    xi = torch.empty((p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
    tune_ms = 0.0
    if args.tune:
        t0 = time.perf_counter()
        plan.tune(Wd, u0, delta, reps=3)
        tune_ms = 1e3 * (time.perf_counter() - t0)
    tuning = dict(plan.tuning(), schedule=plan.tuning_variants()[plan.tuning()["bidiag_variant"]])
    for _ in range(args.warmup):
        plan.invert(Wd, u0, delta, xi)
    torch.cuda.synchronize()
    active = plan.active_systems()
    factorized = plan.factorized_systems()
    # the timed steps: K inversions bracketed by events on the plan's stream
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(args.steps):
        plan.invert(Wd, u0, delta, xi)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # the same K inversions again with the library's stage events (they add
    # a few microseconds per stage, so they stay out of the timed steps)
    plan.profile(True)
    plan.profile_read()
    for _ in range(args.steps):
        plan.invert(Wd, u0, delta, xi)
    torch.cuda.synchronize()
    stages = plan.profile_read()
    plan.profile(False)
    esz = 8 if prec else 16
    units = stage_units(p, active, factorized, p.nz, esz)
    dom = max(stages, key=lambda k: stages[k][0])
    if factorized == 0 and dom == "bidiag":
        dom = "dp"
    dms, dcount = stages[dom]
    per_launch_ms = dms / max(dcount, 1)
    unit, work = units.get(dom, ("GB/s", 0))
    work_per_launch = work / max(dcount / args.steps, 1)
    if unit == "GB/s":
        achieved = work_per_launch / (per_launch_ms * 1e-3) / 1e9
        peak, bound = PEAK_HBM_GBS, "hbm"
    else:
        achieved = work_per_launch / (per_launch_ms * 1e-3) / 1e12
        peak, bound = PEAK_FP64_VALU_TFLOPS, "alu"
    kname = dom
    if dom == "bidiag":
        tr, tc, wpe = tuning["schedule"]
        kname = (f"k_bidiag<{tr}, {tc}, {p.nz // tr}, {p.nz // tc}, double, {wpe}>")
    elif dom == "dp":
        spw = tuning['dp_systems_per_wave'] or (4 if p.nz <= 64 else 2)
        kname = f"k_dp_solve<{64 if p.nz <= 64 else 128}, {spw}>"
    tr_ = profiled_traffic(args.workload, prec, kname)
    roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": tr_["bytes"] if tr_ else None,
            "kernel": kname, "avg_launch_ms": per_launch_ms}
    if tr_:
        roof["traffic_detail"] = dict(tr_, source=os.path.relpath(PROFILE_COUNTERS,
                                                                   os.path.dirname(PROFILE_COUNTERS) + "/.."))
    # HBM-bound stages: algorithmic bytes / event-timed stage duration
    hbm = {}
    for k, (sms, cnt) in stages.items():
        uu, wk = units.get(k, ("", 0))
        if uu == "GB/s" and wk and sms > 0:
            gbs = wk * args.steps / (sms * 1e-3) / 1e9
            hbm[k] = {"GB/s": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 3)}
    fb = sum(units[k][1] for k in FFT_STAGES) * args.steps
    fms = sum(stages[k][0] for k in FFT_STAGES)
    fft_all = {"GB/s": round(fb / (fms * 1e-3) / 1e9, 1),
               "frac": round(fb / (fms * 1e-3) / 1e9 / PEAK_HBM_GBS, 3),
               "ms_per_step": fms / args.steps}
    out = {"ms": ms, "plan_ms": plan_ms, "tune_ms": tune_ms, "tuning": tuning,
           "hbm_stages": hbm, "fft_stages": fft_all, "active": active,
           "factorized": factorized, "roofline": roof,
           "stages": {k: v[0] / args.steps for k, v in stages.items()},
           "xi": xi.cpu().numpy()}
    plan.close()
    return out


if __name__ == "__main__":
    main()
