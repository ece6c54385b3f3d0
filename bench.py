"""Benchmark: voxel-frequencies inverted per second on one MI355X.

One step = one fl_invert call (the whole hot path: FFT of the data,
classification and regularized solves of every (frequency, wavenumber)
system, inverse FFT, zero-padded 3D convolution, xi) over one batch of
synthetic input that is already resident in HBM. The inversion is captured
once as a HIP graph (fl_graph_create) and the graph is replayed: W untimed
replays, then exactly K timed replays with a HIP event recorded on the
plan's stream before the first and after every replay; ms_per_step is the
median of the K per-replay intervals (the mean is reported beside it).

Prints one JSON line. Default workload: the 256x256x128 grid (512x512
torus, 128 data planes, omega = 2 pi {0.5, 0.75, ..., 2.0}, delta = 0.01,
total-field data of a 5-blob contrast computed on the GPU by BiCGSTAB, then
seeded noise). Both precisions are timed on the same data: FP64 throughout,
and mixed (FP32 inverse transforms, convolution and their storage; FP64
data transform, solves and division). The headline is the mixed path when
its xi is within 1e-4 of the FP64 path's and it is faster.

The roofline block describes the kernel that takes the most time per step:
its duration per step from HIP events the library records on its own
stream around every stage (a separate pass of K eager inversions), its
algorithmic work per step from `stage_units`. `cpu_baseline` times the
CPU oracle on a bounded sample of the same workload and states how it was
extrapolated; the same leg compares sampled systems of the GPU result with
the oracle.
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
    "large": "256x256x128 X, 512x512 torus, 128 data planes, omega=2pi*{0.5..2.0 step 0.25}, "
             "5 blobs",
    "multi5": "128x128x64 X, 256x256 torus, 64 data planes, omega=2pi*{0.5..2.5}, 5 blobs",
    "single": "128x128x64 X, 256x256 torus, 64 data planes, omega=2pi, 3 blobs",
    "small": "32x32x16 X, 64x64 torus, 16 data planes, omega=2pi, 3 blobs",
    "uneven": "four instances 64^2x32, 96^2x48, 160^2x80, 192^2x96 (tori 2x), "
              "omega=2pi*{0.75,1.25,1.75}, 3-8 blobs each",
}

FFT_STAGES = ("fft_rows", "fft_cols", "ifft_cols", "crop_pad", "conv_cols", "conv_z",
              "conv_icols", "conv_irows")


def stage_units(p, active, factorized, n, b, spw):
    """Algorithmic work per timed step and stage: HBM bytes that the stage
    must move at least (b bytes per complex element of the FFT-side arrays
    in the stage's precision, 16 for the complex128 W, W^, v, u, u0 and xi),
    or FP64 flops. active: systems solved; factorized: matrices
    bidiagonalized (one per active symmetry orbit when factorizations are
    shared); spw: systems per wave of the discrepancy kernel."""
    F, N, nd, nz = p.n_omega, p.px * p.py, p.nd, p.nz
    nvox = p.nx * p.ny * p.nz
    rows_y = F * nz * p.ny * p.px      # rows of X's y-window on the padded x axis
    planes_n = F * nz * N              # one value per (f, z, system)
    g = 64 // spw                      # trial alphas per search round and system
    u = {
        # the norms come with the row transform (its rowsq output): only the
        # per-row sums are read here
        "norm": ("GB/s", F * nd * p.py * 8),
        # stage (a) runs in FP64 in both precisions
        "fft_rows": ("GB/s", F * nd * N * 32),
        "fft_cols": ("GB/s", F * nd * N * 32),
        # read W^, write ||w||^2 and the flag, zero v^ of the inactive systems,
        # then the orbit / system compaction (flags read three times, lists)
        "classify": ("GB/s", F * nd * N * 16 + F * N * (8 + 4 * 4) + active * 4 +
                     (planes_n - active * nz) * b),
        "ifft_cols": ("GB/s", planes_n * b + rows_y * b),
        "crop_pad": ("GB/s", rows_y * b + F * nvox * 16 + rows_y * b),
        "conv_cols": ("GB/s", rows_y * b + planes_n * b),
        # read the nz nonzero z samples and the kernel's transform, write nz;
        # the transform is even in k, so only its entries 0..nz of 2 nz are
        # read
        "conv_z": ("GB/s", planes_n * b + F * (nz + 1) * N * b + planes_n * b),
        "conv_icols": ("GB/s", planes_n * b + rows_y * b),
        "conv_irows": ("GB/s", rows_y * b + 2 * F * nvox * 16),
        "xi": ("GB/s", 2 * F * nvox * 16 + nvox * 16),
        # complex Householder bidiagonalization of an n x n matrix: 4 x (8/3) n^3
        "bidiag": ("TFLOP/s", factorized * 32.0 / 3.0 * n ** 3),
        # per system: 3 search rounds x g trial alphas x 20 flops per row of
        # the discrepancy recurrence, q = U^H w and v^ = V y (8 n^2 flops
        # each), the bidiagonal Tikhonov solve (about 40 n)
        "dp": ("TFLOP/s", active * (3 * g * 20.0 * n + 16.0 * n * n + 40.0 * n)),
        "backtransform": ("GB/s", 0),
    }
    return u


def counters_path(workload):
    """profiles/counters_<workload>_<nx>x<ny>x<nz>.json"""
    from paper_1911_10487_amd import synth
    p = synth.workload(workload)[0]
    return os.path.join(ROOT, "profiles", f"counters_{workload}_{p.nx}x{p.ny}x{p.nz}.json")


def profiled_traffic(workload, prec, kernel):
    """HBM bytes per step of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE profile of this workload (scaled by the calibration factors),
    or None when there is none or the HIP sources changed since."""
    from paper_1911_10487_amd.build import source_sha256
    path = counters_path(workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        js = json.load(fh)
    if js.get("source_sha256") != source_sha256():
        return None
    k = js.get("kernels", {}).get("mixed" if prec else "fp64", {}).get(kernel)
    if not k:
        return None
    return {"bytes": k["fetch_bytes"] + k["write_bytes"], "fetch_bytes": k["fetch_bytes"],
            "write_bytes": k["write_bytes"], "profiled_avg_us": k["avg_us"],
            "source": os.path.relpath(path, ROOT)}


def _short_kernel_name(name):
    """'void fl::k_bidiag<32, 16, 4, 8, double, 1>(fl::...)' ->
    'k_bidiag<32, 16, 4, 8, double, 1>'."""
    s = name.strip()
    if s.startswith("void "):
        s = s[5:]
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            s = s[:i]
            break
    return s[4:] if s.startswith("fl::") else s


def ingest_counters(fetch_csv, write_csv, stats_csv, workload, prec, copy_mb):
    """Per-dispatch HBM bytes of every fl:: kernel from two rocprofv3 --pmc
    CSVs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), scaled by what the same
    counters read for the run's calibration kernels (a fill and a sum over
    copy_mb MiB), merged into profiles/counters_<workload>.json under the
    digest of the current HIP sources."""
    import csv
    from collections import defaultdict

    from paper_1911_10487_amd.build import source_sha256
    nb_kib = copy_mb * 1024.0
    raw = {}
    calib = {}
    for cname, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = defaultdict(list)
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != cname:
                    continue
                full, v = r["Kernel_Name"], float(r["Counter_Value"])
                if "FillFunctor<double>" in full:
                    calib[f"fill_kernel_{cname}_KiB"] = v
                elif "reduce_kernel" in full and "ReduceOp<double" in full:
                    calib[f"sum_kernel_{cname}_KiB"] = v
                elif "fl::" in full:
                    per[_short_kernel_name(full)].append(v)
        raw[cname] = per
    fetch_factor = nb_kib / calib["sum_kernel_FETCH_SIZE_KiB"]
    write_factor = nb_kib / calib["fill_kernel_WRITE_SIZE_KiB"]
    avg_us = {}
    if stats_csv:
        with open(stats_csv) as fh:
            for r in csv.DictReader(fh):
                avg_us[_short_kernel_name(r["Name"])] = float(r["AverageNs"]) * 1e-3
    kernels = {}
    for k, vals in raw["FETCH_SIZE"].items():
        w = raw["WRITE_SIZE"].get(k)
        if not w:
            continue
        kernels[k] = {"calls": len(vals),
                      "fetch_bytes": float(np.mean(vals)) * 1024.0 * fetch_factor,
                      "write_bytes": float(np.mean(w)) * 1024.0 * write_factor,
                      "avg_us": avg_us.get(k)}
    path = counters_path(workload)
    digest = source_sha256()
    js = {}
    if os.path.exists(path):
        with open(path) as fh:
            js = json.load(fh)
        if js.get("source_sha256") != digest:
            js = {}
    from paper_1911_10487_amd import synth
    p = synth.workload(workload)[0]
    js["source_sha256"] = digest
    js["workload"] = f"{workload}: {WORKLOAD_TEXT[workload]}"
    js.setdefault("calibration", {})[prec] = dict(calib, fetch_factor=fetch_factor,
                                                  write_factor=write_factor,
                                                  calibration_bytes=copy_mb << 20)
    js.setdefault("kernels", {})[prec] = kernels
    js["grid"] = [p.nx, p.ny, p.nz, p.n_omega]
    with open(path, "w") as fh:
        json.dump(js, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(f"wrote {os.path.relpath(path, ROOT)}: {len(kernels)} kernels ({prec}), "
          f"fetch x{fetch_factor:.4f}, write x{write_factor:.4f}")


# ------------------------------------------------------------------ data

def make_data(p, delta, torch, dev):
    """Total-field data: BiCGSTAB on u - omega^2 K(xi u) = u0 to 1e-12 on
    the GPU, the data operator, then seeded noise of relative level delta
    per frequency (on the host). Returns (W^delta host, W^delta device, u0
    host, u0 device)."""
    from paper_1911_10487_amd import synth
    from paper_1911_10487_amd.flayer import Plan
    xi_true = torch.from_numpy(synth.contrast(p)).to(dev)
    u0_np = synth.incident_field(p)
    u0 = torch.from_numpy(u0_np).to(dev)
    gen = Plan.from_problem(p)
    W = gen.forward(xi_true, u0, maxit=500, tol=1e-12)
    torch.cuda.synchronize()
    gen.close()
    Wd_np = synth.add_noise(p, W.cpu().numpy(), delta)
    del W
    return Wd_np, torch.from_numpy(Wd_np).to(dev), u0_np, u0


# ------------------------------------------------------------------ GPU timing

def replay_times(torch, launch, st, steps, warmup):
    """K graph replays bracketed by synchronizations, a HIP event on the
    plan's stream before the first and after each: per-replay ms."""
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(st)
    for i in range(steps):
        launch()
        ev[i + 1].record(st)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]


def time_precision(p, prec, Wd, u0, delta, args, torch, dev, workload, prefactor=0):
    from paper_1911_10487_amd.flayer import Graph, Plan
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
    st = torch.cuda.current_stream()
    plan.invert(Wd, u0, delta, xi)
    torch.cuda.synchronize()
    active = plan.active_systems()
    factorized = plan.factorized_systems()
    if args.eager:
        times = replay_times(torch, lambda: plan.invert(Wd, u0, delta, xi), st, args.steps,
                             args.warmup)
        method = "eager fl_invert calls"
    else:
        g = Graph(plan, Wd, u0, delta, xi)
        times = replay_times(torch, g.launch, st, args.steps, args.warmup)
        g.close()
        method = "HIP graph replays"
    ms = float(np.median(times))
    # the same K inversions again, eager, with the library's stage events
    # (they add a few microseconds per stage, so they stay out of the timed
    # steps)
    plan.profile(True)
    plan.profile_read()
    for _ in range(args.steps):
        plan.invert(Wd, u0, delta, xi)
    torch.cuda.synchronize()
    stages = plan.profile_read()
    plan.profile(False)
    esz = 8 if prec else 16
    # systems per search wave: the orbit-by-orbit solve (shared
    # factorizations, the default) takes 4 unless tuned
    spw = tuning["dp_systems_per_wave"] or 4
    units = stage_units(p, active, factorized, p.nz, esz, spw)
    per_step = {k: v[0] / args.steps for k, v in stages.items()}
    dom = max(per_step, key=per_step.get)
    unit, work = units.get(dom, ("GB/s", 0))
    dms = per_step[dom]
    if unit == "GB/s":
        achieved = work / (dms * 1e-3) / 1e9
        peak, bound = PEAK_HBM_GBS, "hbm"
    else:
        achieved = work / (dms * 1e-3) / 1e12
        peak, bound = PEAK_FP64_VALU_TFLOPS, "alu"
    kname = dom
    if dom == "bidiag":
        tr, tc, wpe = tuning["schedule"]
        kname = f"k_bidiag<{tr}, {tc}, {p.nz // tr}, {p.nz // tc}, double, {wpe}>"
    elif dom == "dp":
        kname = f"k_dpo_search<{64 if p.nz <= 64 else 128}, {spw}>"
    tr_ = profiled_traffic(workload, prec, kname)
    roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": tr_["bytes"] if tr_ else None,
            "kernel": kname, "ms_per_step": dms,
            "launches_per_step": stages[dom][1] / args.steps,
            "work_per_step": work}
    if tr_:
        roof["traffic_detail"] = tr_
    hbm = {}
    for k, v in per_step.items():
        uu, wk = units.get(k, ("", 0))
        if uu == "GB/s" and wk and v > 0:
            gbs = wk / (v * 1e-3) / 1e9
            hbm[k] = {"GB/s": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 3)}
    fb = sum(units[k][1] for k in FFT_STAGES)
    fms = sum(per_step[k] for k in FFT_STAGES)
    fft_all = {"GB/s": round(fb / (fms * 1e-3) / 1e9, 1),
               "frac": round(fb / (fms * 1e-3) / 1e9 / PEAK_HBM_GBS, 3), "ms_per_step": fms}
    out = {"ms": ms, "ms_mean": float(np.mean(times)), "ms_min": float(np.min(times)),
           "timing": method, "plan_ms": plan_ms, "tune_ms": tune_ms, "tuning": tuning,
           "hbm_stages": hbm, "fft_stages": fft_all, "active": active,
           "factorized": factorized, "roofline": roof, "stages": per_step,
           "xi": xi.cpu().numpy(), "plan": plan}
    return out


def gpu_sample(plan, p, ms_by_f):
    """The GPU's v^, alpha and branch at the sampled systems (stage taps)."""
    from paper_1911_10487_amd.flayer import TAP_ALPHA, TAP_BRANCH, TAP_VHAT
    F, N = p.n_omega, p.px * p.py
    info = plan.info()
    cw = np.complex64 if info.precision == 1 else np.complex128
    vh = plan.tap(TAP_VHAT, cw, (F, p.nz, N))
    al = plan.tap(TAP_ALPHA, np.float64, (F, N))
    br = plan.tap(TAP_BRANCH, np.int8, (F, N))
    return {f: (vh[f][:, ms].T.astype(np.complex128), al[f][ms], br[f][ms])
            for f, ms in ms_by_f.items()}


def sample_systems(p, f, count, seed):
    """Seeded wavenumbers to check at frequency f, drawn from the geometry
    only: half inside |k| <= 1.5 k0 (where the data carry signal above the
    noise), half uniform over the torus."""
    from paper_1911_10487_amd import synth  # noqa: F401  (geometry helpers only)
    rng = np.random.default_rng([seed, f])
    sx = np.where(np.arange(p.px) <= p.px // 2, np.arange(p.px), np.arange(p.px) - p.px)
    sy = np.where(np.arange(p.py) <= p.py // 2, np.arange(p.py), np.arange(p.py) - p.py)
    kx = 2 * np.pi * sx / (p.px * p.h)
    ky = 2 * np.pi * sy / (p.py * p.h)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    k0 = p.omegas[f] / p.c0
    inner = np.nonzero((k2 <= (1.5 * k0) ** 2).ravel())[0]
    a = rng.choice(inner, size=min(count // 2, len(inner)), replace=False)
    b = rng.choice(p.px * p.py, size=count - len(a), replace=False)
    return np.unique(np.concatenate([a, b]))


# ------------------------------------------------------------------ CPU oracle leg

def _oracle_systems_worker(job):
    """One worker of the all-core oracle timing: the oracle's per-system
    solve of its share of the sampled systems, single-threaded."""
    from threadpoolctl import threadpool_limits

    from oracle import model
    from oracle.regularize import tikhonov_dp
    p, f, tab, idx, w, dm = job
    with threadpool_limits(1):
        t0 = time.perf_counter()
        A = model.system_matrices(p, f, tab, idx, None)
        tikhonov_dp(A, w, dm)
        return time.perf_counter() - t0


def cpu_leg(p, Wd_np, u0_np, delta, runs, ms_by_f, workers, timing=True):
    """The oracle on the host: (1) parity of sampled systems (v^, alpha,
    branch) of both GPU precisions, or of the whole xi when the workload is
    small enough; (2) the oracle's time on a bounded sample, extrapolated to
    the whole workload: serial (one thread) and on `workers` processes."""
    from threadpoolctl import threadpool_limits

    from oracle import invert, model
    from oracle.regularize import tikhonov_dp
    F, N = p.n_omega, p.px * p.py
    vf = p.voxel_frequencies
    parity = {}
    full = timing and N * p.nz <= 70000 * 64 and F <= 1
    if full:
        t0 = time.perf_counter()
        xi_ref = invert.invert(p, Wd_np, u0_np, delta)
        t_full = time.perf_counter() - t0
        for k, r in runs.items():
            parity[k] = {"xi_rel_l2_vs_oracle":
                         float(np.linalg.norm(r["xi"] - xi_ref) / np.linalg.norm(xi_ref))}
    # sampled systems (both routes), with their tables by the sampled DFT
    samp = {}
    t_tab = 0.0
    for f, ms in ms_by_f.items():
        t0 = time.perf_counter()
        w = model.dft2_at(Wd_np[f], ms, p.px, p.py).T
        tab, idx = model.system_table_at(p, f, ms)
        t_tab += time.perf_counter() - t0
        dm = invert.system_noise_level(Wd_np[f], delta)
        samp[f] = (tab, idx, w, dm)
    for k, r in runs.items():
        worst_v, worst_a, mism, n = 0.0, 0.0, 0, 0
        for f, ms in ms_by_f.items():
            tab, idx, w, dm = samp[f]
            A = model.system_matrices(p, f, tab, idx, None)
            v_ref, a_ref, b_ref = tikhonov_dp(A, w, dm)
            v, a, b = r["sample"][f]
            mism += int(np.count_nonzero(b != b_ref))
            n += len(ms)
            nr = np.linalg.norm(v_ref, axis=1)
            ok = nr > 0
            if ok.any():
                e = np.linalg.norm(v - v_ref, axis=1)[ok] / nr[ok]
                worst_v = max(worst_v, float(e.max()))
            fin = np.isfinite(a_ref) & np.isfinite(a)
            if fin.any():
                worst_a = max(worst_a, float(np.max(np.abs(a[fin] - a_ref[fin]) / a_ref[fin])))
        parity.setdefault(k, {}).update({
            "sampled_systems": n, "sampled_branch_mismatches": mism,
            "sampled_vhat_max_rel_err": worst_v, "sampled_alpha_max_rel_err": worst_a})
    if not timing:
        return None, parity
    # --- timing (the oracle as it stands, on a bounded sample): stage (a)
    # (np.fft.fft2 of every frequency's data, the oracle's library step)
    # whole; stage (c) (inverse transform, crop, the 3D volume potential) and
    # the xi step whole for one frequency, scaled by F; the per-system solves
    # (the oracle's A_m gather + tikhonov_dp, as in its solve_systems) on
    # per_f uniformly sampled wavenumbers of every frequency, scaled by
    # N / per_f. Each frequency's full table is built untimed (plan-time
    # work, excluded as on the GPU).
    per_f = min(N, max(64, int(640 * (128.0 / p.nz) ** 2)))
    rng = np.random.default_rng(29)
    t_a = t_sys = 0.0
    jobs = []
    with threadpool_limits(1):
        for f in range(F):
            t0 = time.perf_counter()
            What = np.fft.fft2(Wd_np[f])
            t_a += time.perf_counter() - t0
            tab, idx = model.system_table(p, f)
            ms = np.sort(rng.choice(N, size=per_f, replace=False))
            wsys = What.reshape(p.nd, N).T[ms]
            dm = invert.system_noise_level_hat(What, delta, N)
            tab_s = tab.reshape(tab.shape[0], -1)[:, ms]
            del tab, What
            t0 = time.perf_counter()
            A = model.system_matrices(p, f, tab_s, idx, None)
            tikhonov_dp(A, wsys, dm)
            t_sys += time.perf_counter() - t0
            del A
            for part in np.array_split(np.arange(per_f), workers):
                if len(part):
                    jobs.append((p, f, tab_s[:, part], idx, wsys[part], dm))
        # stage (c) and (d) of one frequency (the work does not depend on
        # the values)
        t0 = time.perf_counter()
        v = model.crop(p, np.fft.ifft2(np.zeros((p.nz, p.py, p.px), np.complex128)))
        u = u0_np[0] + model.volume_potential(p, 0, v)
        invert.combine_lsq(u[None], v[None])
        t_c = time.perf_counter() - t0
    serial_s = t_a + F * t_c + t_sys * N / per_f
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_systems_worker, jobs[:workers])  # start-up and imports
        t0 = time.perf_counter()
        pool.map(_oracle_systems_worker, jobs)
        t_par = time.perf_counter() - t0
    par_s = t_a + F * t_c + t_par * N / per_f
    sample = (f"stage (a) whole ({t_a:.1f} s); stage (c) and xi for one frequency "
              f"({t_c:.1f} s, scaled by {F}); the per-system Tikhonov/discrepancy solves on "
              f"{per_f} uniformly sampled wavenumbers per frequency ({F * per_f} of {F * N} "
              f"systems: {t_sys:.1f} s on one thread, {t_par:.1f} s on {workers} processes), "
              f"scaled by {N}/{per_f}; tables excluded (plan-time work, as on the GPU); "
              f"NumPy FFTs single-threaded")
    if full:
        sample += f"; the whole oracle inversion (tables included) took {t_full:.1f} s here"
    cpu = {"value": vf / par_s, "unit": "voxel-freq/s", "cores": workers, "kind": "oracle",
           "sample": sample,
           "serial": {"value": vf / serial_s, "cores": 1, "seconds_extrapolated": serial_s},
           "seconds_extrapolated": par_s}
    return cpu, parity


# ------------------------------------------------------------------ variants

def _event_ms(torch, fn, reps, warmup=1):
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


def time_variants(p, Wd, u0, delta, args, torch, dev, iters):
    """Secondary figures on the same data, none of them the headline: the
    derivatives of W -> xi (one VJP, one JVP), `iters` power iterations on
    J^T J (each a JVP and a VJP), and the inversion with the truncated-SVD
    regularizer where the plan supports it."""
    from paper_1911_10487_amd.autograd import power_iteration
    from paper_1911_10487_amd.flayer import FlError, Plan
    out = {}
    vf = p.voxel_frequencies
    reps = max(1, min(args.steps, 5))
    for label, prec in (("fp64", 0), ("mixed", 1)):
        if args.only and label != args.only:
            continue
        plan = Plan.from_problem(p, precision=prec)
        g = torch.randn((p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        dW = torch.randn(Wd.shape, dtype=Wd.dtype, device=dev)
        t_vjp = _event_ms(torch, lambda: plan.vjp(Wd, u0, delta, g), reps)
        t_jvp = _event_ms(torch, lambda: plan.jvp(Wd, u0, delta, dW), reps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        est, _ = power_iteration(plan, Wd, u0, delta, iters=iters)
        torch.cuda.synchronize()
        t_pi = (time.perf_counter() - t0) * 1e3
        plan.close()
        r = {"vjp_ms": t_vjp, "jvp_ms": t_jvp, "power_iterations": iters,
             "power_iteration_ms": t_pi, "power_iteration_sigma": est[-1]}
        try:
            tplan = Plan.from_problem(p, precision=prec, regularizer=1)
        except FlError as e:
            r["tsvd"] = f"not run: {e}"
        else:
            xi = torch.empty((p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
            t_tsvd = _event_ms(torch, lambda: tplan.invert(Wd, u0, delta, xi), reps)
            tplan.close()
            r["tsvd_ms_per_step"] = t_tsvd
            r["tsvd_value"] = vf / (t_tsvd * 1e-3)
        out[label] = r
        print(f"[bench] {label}: vjp {t_vjp:.2f} ms, jvp {t_jvp:.2f} ms, {iters} power "
              f"iterations {t_pi:.1f} ms", file=sys.stderr, flush=True)
    return out


# ------------------------------------------------------------------ workloads

def run_single(p, delta, args, torch, dev, workload, with_cpu=True, samples=96):
    """Both precisions on one instance; returns the summary dict."""
    print(f"[bench] {workload}: data", file=sys.stderr, flush=True)
    Wd_np, Wd, u0_np, u0 = make_data(p, delta, torch, dev)
    runs = {}
    precs = (("fp64", 0), ("mixed", 1))
    if args.only:
        precs = tuple(x for x in precs if x[0] == args.only)
    F = p.n_omega
    fs = sorted({0, F // 2, F - 1})
    ms_by_f = {f: sample_systems(p, f, samples, 17) for f in fs}
    for label, prec in precs:
        r = time_precision(p, prec, Wd, u0, delta, args, torch, dev, workload)
        plan = r.pop("plan")
        r["sample"] = gpu_sample(plan, p, ms_by_f)
        plan.close()
        runs[label] = r
        print(f"[bench] {workload} {label}: {r['ms']:.3f} ms/step (median of {args.steps} "
              f"{r['timing']})", file=sys.stderr, flush=True)
    out = {"runs": runs, "ms_by_f": ms_by_f, "Wd_np": Wd_np, "u0_np": u0_np, "Wd": Wd, "u0": u0}
    if not args.no_cpu_baseline:
        print(f"[bench] {workload}: CPU oracle leg", file=sys.stderr, flush=True)
        cpu, parity = cpu_leg(p, Wd_np, u0_np, delta, runs, ms_by_f, args.cpu_workers,
                              timing=with_cpu)
        out["parity"] = parity
        if cpu is not None:
            out["cpu"] = cpu
    return out


def summarize(p, res, delta):
    runs = res["runs"]
    vf = p.voxel_frequencies
    summ = {}
    for k, r in runs.items():
        summ[k] = {"value": vf / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
                   "ms_mean": r["ms_mean"], "ms_min": r["ms_min"], "timing": r["timing"],
                   "active_systems": r["active"], "factorized_systems": r["factorized"],
                   "plan_ms": r["plan_ms"], "schedule": r["tuning"],
                   "fft_stages": r["fft_stages"], "roofline": r["roofline"]}
        summ[k].update(res.get("parity", {}).get(k, {}))
    if "fp64" in runs and "mixed" in runs:
        a, b = runs["mixed"]["xi"], runs["fp64"]["xi"]
        summ["mixed"]["xi_rel_l2_vs_fp64_gpu"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return summ


def secondary_multi5(args, torch, dev):
    """Config with 5 frequencies on the 128x128x64 grid at both of its noise
    levels (a second line inside the JSON)."""
    from paper_1911_10487_amd import synth
    p = synth.workload("multi5")[0]
    out = {"workload": f"multi5: {WORKLOAD_TEXT['multi5']}"}
    for d in p.deltas:
        res = run_single(p, d, args, torch, dev, "multi5", with_cpu=False, samples=64)
        out[f"delta={d}"] = summarize(p, res, d)
    return out


def secondary_uneven(args, torch, dev):
    """The four uneven instances inverted together (fl_batch_invert: one
    stream per instance, forked from and joined to the caller's), mixed
    precision, against each instance alone."""
    from paper_1911_10487_amd import synth
    from paper_1911_10487_amd.flayer import Batch, Plan
    insts = synth.workload("uneven")
    plans, Ws, us, ds, xis, alone = [], [], [], [], [], []
    for p in insts:
        d = p.deltas[0]
        _, Wd, _, u0 = make_data(p, d, torch, dev)
        plan = Plan.from_problem(p, precision=1)
        xi = torch.empty((p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        alone.append(_event_ms(torch, lambda: plan.invert(Wd, u0, d, xi), args.steps))
        plans.append(plan)
        Ws.append(Wd)
        us.append(u0)
        ds.append(d)
        xis.append(xi)
    b = Batch(plans)
    t_b = _event_ms(torch, lambda: b.invert(Ws, us, ds, xis), args.steps)
    b.close()
    for pl in plans:
        pl.close()
    vf = sum(p.voxel_frequencies for p in insts)
    return {"workload": f"uneven: {WORKLOAD_TEXT['uneven']}", "precision": "mixed",
            "batch_ms_per_step": t_b, "value": vf / (t_b * 1e-3),
            "instances_ms_each_alone": alone, "sum_alone_ms": float(sum(alone))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large",
                    choices=["large", "multi5", "single", "small"])
    ap.add_argument("--delta", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="time one precision only (profiling runs; its derivative "
                         "figures too unless --no-variants)")
    ap.add_argument("--eager", action="store_true",
                    help="time eager fl_invert calls instead of graph replays")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the solver schedule on the data before timing")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the derivative and TSVD timings")
    ap.add_argument("--power-iterations", type=int, default=20)
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 5-frequency and uneven-batch workloads")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run one plain device fill, sum and copy of this many MiB before "
                         "timing (known-size kernels for scaling HBM counters)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU work: turn two rocprofv3 --pmc CSVs (FETCH_SIZE, WRITE_SIZE) "
                         "of a run with --calibrate-copy-mb into the workload's counters "
                         "profile (precision from --only)")
    ap.add_argument("--ingest-stats", metavar="KERNEL_STATS_CSV", default=None,
                    help="with --ingest-counters: rocprofv3 --stats kernel CSV for avg_us")
    args = ap.parse_args()
    if args.ingest_counters:
        if not args.only or not args.calibrate_copy_mb:
            ap.error("--ingest-counters needs --only and --calibrate-copy-mb")
        ingest_counters(*args.ingest_counters, args.ingest_stats, args.workload, args.only,
                        args.calibrate_copy_mb)
        return
    if args.gpus != 1:
        print(f"bench.py: the inversion runs on a single GPU; --gpus {args.gpus} is not "
              "supported (the systems are independent per frequency and wavenumber, so a "
              "multi-GPU run would split the frequencies and all-reduce two per-voxel sums; "
              "not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1911_10487_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    p = synth.workload(args.workload)[0]
    delta = p.deltas[0] if args.delta is None else args.delta
    print(f"[bench] workload {args.workload} delta={delta}", file=sys.stderr, flush=True)

    if args.calibrate_copy_mb:
        nb = args.calibrate_copy_mb << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        s = src.sum()
        dst = src * 1.0
        torch.cuda.synchronize()
        print(f"[bench] calibration kernels over {nb} bytes (sum {float(s):.0f})",
              file=sys.stderr, flush=True)
        del src, dst

    res = run_single(p, delta, args, torch, dev, args.workload)
    runs = res["runs"]
    summ = summarize(p, res, delta)
    vf = p.voxel_frequencies
    if args.only:
        r = runs[args.only]
        # the derivative figures of this precision too, unless --no-variants
        var = (None if args.no_variants else
               time_variants(p, res["Wd"], res["u0"], delta, args, torch, dev,
                             args.power_iterations))
        print(json.dumps({"metric": "voxel-frequencies inverted/s; mixed vs FP64 plain at ξ rel-L2 ≤1e-4", "precision": args.only,
                          "value": vf / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
                          "schedule": r["tuning"],
                          "roofline": r["roofline"], "fft_stages": r["fft_stages"],
                          "hbm_stages": r["hbm_stages"], "stages_ms_per_step": r["stages"],
                          "variants": var}),
              flush=True)
        return
    variants = None
    if not args.no_variants:
        variants = time_variants(p, res["Wd"], res["u0"], delta, args, torch, dev,
                                 args.power_iterations)
    secondary = {}
    if not args.no_secondary and args.workload == "large":
        secondary["multi5"] = secondary_multi5(args, torch, dev)
        secondary["uneven"] = secondary_uneven(args, torch, dev)
    # headline: the mixed path when it is within 1e-4 of the FP64 path (and of
    # the oracle's sampled systems) and faster
    gate = summ["mixed"]["xi_rel_l2_vs_fp64_gpu"] <= 1e-4
    if "xi_rel_l2_vs_oracle" in summ["mixed"]:
        gate = gate and summ["mixed"]["xi_rel_l2_vs_oracle"] <= 1e-4
    head = "mixed" if gate and runs["mixed"]["ms"] < runs["fp64"]["ms"] else "fp64"
    h = runs[head]
    out = {
        "metric": "voxel-frequencies inverted/s; mixed vs FP64 plain at ξ rel-L2 ≤1e-4",
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
                   "delta": delta, "precision": head, "timing": h["timing"] +
                   f", median of {args.steps} after {args.warmup} warm-up",
                   "active_systems": h["active"], "factorized_systems": h["factorized"],
                   "systems": p.n_omega * p.px * p.py, "n": p.nz, "plan_ms": h["plan_ms"],
                   "schedule": h["tuning"]},
        "roofline": h["roofline"],
        "fft_stages": h["fft_stages"],
        "hbm_stages": h["hbm_stages"],
        "stages_ms_per_step": h["stages"],
        "fp64": summ["fp64"],
        "mixed": summ["mixed"],
    }
    if variants is not None:
        out["variants"] = variants
    if secondary:
        out["secondary"] = secondary
    if "cpu" in res:
        out["cpu_baseline"] = res["cpu"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
