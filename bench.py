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
    "single": "128x128x64 X, 256x256 torus, 64 data planes, omega=2pi, Born data of 3 blobs",
    "multi5": "128x128x64 X, 256x256 torus, 64 data planes, omega=2pi*{0.5..2.5}, Born data of 5 blobs",
    "small": "32x32x16 X, 64x64 torus, 16 data planes, omega=2pi, Born data of 3 blobs",
}


def stage_units(p, active, n):
    """Algorithmic bytes (HBM-bound stages) or FP64 flops per call, per stage."""
    F, N, nd, nz = p.n_omega, p.px * p.py, p.nd, p.nz
    nvox = p.nx * p.ny * p.nz
    b = 16
    rows_y = F * nz * p.ny * p.px
    u = {
        "norm": ("GB/s", F * nd * N * b),
        "fft_rows": ("GB/s", 2 * F * nd * N * b),
        "fft_cols": ("GB/s", 2 * F * nd * N * b),
        "classify": ("GB/s", F * nd * N * b + F * N * 8),
        "ifft_cols": ("GB/s", F * nz * N * b + rows_y * b),
        "crop_pad": ("GB/s", rows_y * b + F * nvox * b + rows_y * b),
        "conv_cols": ("GB/s", rows_y * b + F * nz * N * b),
        "conv_z": ("GB/s", 2 * F * nz * N * b + 2 * F * nz * N * b),
        "conv_icols": ("GB/s", F * nz * N * b + rows_y * b),
        "conv_irows": ("GB/s", rows_y * b + 2 * F * nvox * b),
        "xi": ("GB/s", 2 * F * nvox * b + nvox * b),
        # complex Householder bidiagonalization of an n x n matrix: 4 x (8/3) n^3
        "bidiag": ("TFLOP/s", active * 32.0 / 3.0 * n ** 3),
        # per system: about 60 Newton trials of ~60 flops per row (estimate)
        "dp": ("TFLOP/s", active * 60.0 * 60.0 * n),
        # reflector application: n^2/2 complex multiply-adds twice
        "backtransform": ("GB/s", active * (n * n * b // 2 + 2 * n * b)),
    }
    return u


def cpu_baseline(p, Wd, u0, delta, vf):
    from threadpoolctl import threadpool_info

    from oracle import invert
    t0 = time.perf_counter()
    invert.invert(p, Wd, u0, delta)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": vf / dt, "unit": "voxel-freq/s", "cores": int(threads), "kind": "oracle",
            "sample": f"the whole workload once ({vf} voxel-frequencies), NumPy FP64 oracle, "
                      f"{dt:.1f} s; LAPACK SVDs on {threads} threads, FFTs single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="single", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--delta", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1911_10487_amd import synth
    from paper_1911_10487_amd.flayer import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    p = synth.workload(args.workload)[0]
    delta = p.deltas[0] if args.delta is None else args.delta
    print(f"[bench] workload {args.workload} delta={delta}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    plan = Plan.from_problem(p)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)

    xi_true = torch.from_numpy(synth.contrast(p)).to(dev)
    u0_np = synth.incident_field(p)
    u0 = torch.from_numpy(u0_np).to(dev)
    W = plan.forward(xi_true, u0)
    torch.cuda.synchronize()
    Wd_np = synth.add_noise(p, W.cpu().numpy(), delta)
    Wd = torch.from_numpy(Wd_np).to(dev)
    xi = torch.empty((p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)

    for _ in range(args.warmup):
        plan.invert(Wd, u0, delta, xi)
    torch.cuda.synchronize()
    active = plan.active_systems()
    print(f"[bench] warmup done, {active} active systems", file=sys.stderr, flush=True)

    plan.profile(True)
    plan.profile_read()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(args.steps):
        plan.invert(Wd, u0, delta, xi)
    e1.record(st)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    stages = plan.profile_read()
    plan.profile(False)
    ms = total_ms / args.steps
    vf = p.voxel_frequencies
    value = vf / (ms * 1e-3)
    print(f"[bench] timed {args.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    units = stage_units(p, active, p.nz)
    dom = max(stages, key=lambda k: stages[k][0])
    dms, dcount = stages[dom]
    per_launch_ms = dms / max(dcount, 1)
    unit, work = units.get(dom, ("GB/s", 0))
    launches_per_step = dcount / args.steps
    work_per_launch = work / max(launches_per_step, 1)
    if unit == "GB/s":
        achieved = work_per_launch / (per_launch_ms * 1e-3) / 1e9
        peak, bound = PEAK_HBM_GBS, "hbm"
    else:
        achieved = work_per_launch / (per_launch_ms * 1e-3) / 1e12
        peak, bound = PEAK_FP64_VALU_TFLOPS, "alu"
    roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": None, "kernel": dom,
            "avg_launch_ms": per_launch_ms}

    out = {
        "metric": "voxel-frequencies inverted/s",
        "value": value,
        "unit": "voxel-freq/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}",
                   "delta": delta, "precision": "fp64", "active_systems": active,
                   "systems": p.n_omega * p.px * p.py, "n": p.nz, "plan_ms": plan_ms},
        "roofline": roof,
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
        "mixed": None,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p, Wd_np, u0_np, delta, vf)
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
