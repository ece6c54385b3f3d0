"""The benchmark configurations at full size against the oracle, in the launch
configuration the benchmark times (default plans, fl_invert through the C
ABI).

The oracle cannot invert the 256x256x128 seven-frequency grid whole in a
test's time, so there every frequency is checked on sampled systems: the
oracle's own data (Born data by its z-convolution data operator, seeded
noise), its own transform W^ and table, and its own discrepancy-chosen
Tikhonov solve of each sampled (frequency, wavenumber) system; the GPU's
v^, alpha and branch of the same systems (stage taps) must match: branches
exactly, alpha and v^ within 1e-10 (FP64) and v^ within 1e-5 (mixed: v^
is stored in FP32 there). The samples hold, per frequency, systems the
oracle finds active and systems drawn from the whole torus. The same is
done for the two larger instances of the uneven batch; its two smaller
instances and the five-frequency grid are compared with the whole oracle
inversion (xi and every stage).

No value the GPU computed enters the oracle: data, transforms, tables and
solves on the oracle side are the oracle's.
"""
import sys

import numpy as np
import pytest

from oracle import forward, invert, model
from oracle.regularize import tikhonov_dp
from paper_1911_10487_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10
MIXED_TOL = 1e-4


def say(*a):
    print("[gpu-fullsize]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_data(p, delta):
    """Born data of the seeded contrast by the oracle (z-convolution data
    operator), with the seeded noise."""
    xi = synth.contrast(p)
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=True, zconv=True)
    return synth.add_noise(p, W, delta), u0


def gpu_stages(plan, p, precision):
    from paper_1911_10487_amd.flayer import TAP_ALPHA, TAP_BRANCH, TAP_VHAT
    F, N = p.n_omega, p.px * p.py
    cw = np.complex64 if precision == 1 else np.complex128
    return (plan.tap(TAP_VHAT, cw, (F, p.nz, N)), plan.tap(TAP_ALPHA, np.float64, (F, N)),
            plan.tap(TAP_BRANCH, np.int8, (F, N)))


def gpu_run(p, Wd, u0, delta, precision):
    import torch
    from paper_1911_10487_amd.flayer import Plan
    say(f"GPU {p.name} {p.nx}x{p.ny}x{p.nz} F={p.n_omega} precision={precision}")
    plan = Plan.from_problem(p, precision=precision)
    xi = plan.invert(torch.from_numpy(Wd).cuda(), torch.from_numpy(u0).cuda(), delta)
    torch.cuda.synchronize()
    out = (xi.cpu().numpy(), gpu_stages(plan, p, precision), plan.active_systems())
    plan.close()
    torch.cuda.empty_cache()
    return out


def sampled_check(p, Wd, delta, runs, per_f, seed):
    """For every frequency: the oracle's W^, table and solve of per_f
    sampled systems (half among the systems the oracle finds active, half
    uniform), against every GPU run's v^, alpha and branch there."""
    F, N = p.n_omega, p.px * p.py
    rng = np.random.default_rng([seed, 1])
    worst = {k: [0.0, 0.0] for k in runs}
    counts = [0, 0]
    for f in range(F):
        What = np.fft.fft2(Wd[f])
        wsys = What.reshape(p.nd, N).T
        dm = invert.system_noise_level_hat(What, delta, N)
        act = np.flatnonzero(np.linalg.norm(wsys, axis=1) > 1.5 * dm)
        ms = np.unique(np.concatenate([
            rng.choice(act, size=min(per_f // 2, len(act)), replace=False),
            rng.choice(N, size=per_f // 2, replace=False)]))
        tab, idx = model.system_table(p, f)
        A = model.system_matrices(p, f, tab, idx, ms)
        del tab
        v_ref, a_ref, b_ref = tikhonov_dp(A, wsys[ms], dm)
        counts[0] += len(ms)
        counts[1] += int(np.count_nonzero(b_ref))
        for k, (vh, al, br) in runs.items():
            prec = 1 if k == "mixed" else 0
            mism = int(np.count_nonzero(br[f][ms] != b_ref))
            assert mism == 0, f"{k}: frequency {f}: {mism} branch mismatches"
            fin = np.isfinite(a_ref)
            assert np.array_equal(np.isfinite(al[f][ms]), fin)
            ea = float(np.max(np.abs(al[f][ms][fin] - a_ref[fin]) / a_ref[fin])) if fin.any() else 0.0
            v = vh[f][:, ms].T.astype(np.complex128)
            ev = rel(v, v_ref)
            worst[k][0] = max(worst[k][0], ea)
            worst[k][1] = max(worst[k][1], ev)
            assert ea <= TOL, (k, f, ea)
            assert ev <= (1e-5 if prec else TOL), (k, f, ev)
        say(f"frequency {f}: {len(ms)} systems ({int(np.count_nonzero(b_ref))} solved) agree")
    say("sampled", counts[0], "systems,", counts[1], "solved; worst alpha / v^ errors", worst)
    return counts


@pytest.fixture(scope="module")
def large():
    p = synth.workload("large")[0]
    say("large: oracle data", p.nx, p.nz, p.px, p.n_omega)
    Wd, u0 = oracle_data(p, p.deltas[0])
    return p, Wd, u0


@pytest.mark.timeout(900)
def test_large_configuration_sampled_systems_match_oracle(large):
    p, Wd, u0 = large
    delta = p.deltas[0]
    x64, s64, act64 = gpu_run(p, Wd, u0, delta, 0)
    xm, sm, actm = gpu_run(p, Wd, u0, delta, 1)
    assert act64 == actm
    e = rel(xm, x64)
    say("large: active systems", act64, "mixed vs FP64 xi", e)
    assert e <= MIXED_TOL
    n, solved = sampled_check(p, Wd, delta, {"fp64": s64, "mixed": sm}, 2048, 41)
    assert n >= 7 * 1500 and solved >= 7 * 900


@pytest.mark.timeout(600)
def test_large_configuration_twenty_power_iterations(large):
    """20 power iterations on J^T J (the configuration's derivative figure),
    mixed precision: the Rayleigh quotients increase monotonically and the
    last steps agree to 1e-3 (converged), and the FP64 path gives the same
    estimate."""
    import torch
    from paper_1911_10487_amd.autograd import power_iteration
    from paper_1911_10487_amd.flayer import Plan
    p, Wd, u0 = large
    delta = p.deltas[0]
    Wt, ut = torch.from_numpy(Wd).cuda(), torch.from_numpy(u0).cuda()
    est = {}
    for prec in (1, 0):
        say("large power iteration, precision", prec)
        plan = Plan.from_problem(p, precision=prec)
        e, _ = power_iteration(plan, Wt, ut, delta, iters=20, seed=4)
        plan.close()
        torch.cuda.empty_cache()
        say("estimates", e)
        assert all(b >= a * (1 - 1e-9) for a, b in zip(e, e[1:]))
        est[prec] = e
    assert abs(est[1][-1] - est[1][-2]) <= 1e-3 * est[1][-1]
    assert abs(est[1][-1] - est[0][-1]) <= 1e-4 * est[0][-1]


@pytest.mark.timeout(900)
def test_uneven_instances_match_oracle():
    """The four uneven instances inverted together (fl_batch_invert, mixed)
    and each alone in FP64: the two smaller ones against the whole oracle
    inversion, the two larger on sampled systems of every frequency."""
    import torch
    from paper_1911_10487_amd.flayer import Batch, Plan
    insts = synth.workload("uneven")
    data = [oracle_data(p, p.deltas[0]) for p in insts]
    plans = [Plan.from_problem(p, precision=1) for p in insts]
    Ws = [torch.from_numpy(W).cuda() for W, _ in data]
    us = [torch.from_numpy(u).cuda() for _, u in data]
    xis = [torch.empty((p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda") for p in insts]
    b = Batch(plans)
    b.invert(Ws, us, [p.deltas[0] for p in insts], xis)
    torch.cuda.synchronize()
    b.close()
    mixed = [(x.cpu().numpy(), gpu_stages(pl, p, 1)) for x, pl, p in zip(xis, plans, insts)]
    for pl in plans:
        pl.close()
    del Ws, us, xis
    for i, p in enumerate(insts):
        Wd, u0 = data[i]
        d = p.deltas[0]
        x64, s64, _ = gpu_run(p, Wd, u0, d, 0)
        xm, sm = mixed[i]
        e = rel(xm, x64)
        say(p.name, "batched mixed vs FP64 GPU", e)
        assert e <= MIXED_TOL
        if p.nz <= 48:
            ref, st = invert.invert(p, Wd, u0, d, stages=True)
            N = p.px * p.py
            assert np.array_equal(st["branch"], s64[2])
            e64 = {"xi": rel(x64, ref),
                   "Vhat": rel(s64[0], st["Vhat"].reshape(p.n_omega, p.nz, N))}
            em = rel(xm, ref)
            say(p.name, "vs oracle: FP64", e64, "mixed xi", em)
            assert max(e64.values()) <= TOL and em <= MIXED_TOL
        else:
            sampled_check(p, Wd, d, {"fp64": s64, "mixed": sm}, 1024, 50 + i)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("delta", [0.005, 0.02])
def test_five_frequency_configuration_matches_oracle(delta):
    """The 5-frequency 128x128x64 grid at both of its noise levels, whole:
    every stage and xi against the oracle (FP64), xi within 1e-4 (mixed)."""
    p = synth.workload("multi5")[0]
    Wd, u0 = oracle_data(p, delta)
    ref_xi, ref = invert.invert(p, Wd, u0, delta, stages=True)
    F, N = p.n_omega, p.px * p.py
    x64, s64, act = gpu_run(p, Wd, u0, delta, 0)
    assert act == int(np.count_nonzero(ref["branch"]))
    assert np.array_equal(ref["branch"].reshape(F, N), s64[2])
    fin = np.isfinite(ref["alpha"].reshape(F, N))
    ea = rel(s64[1][fin], ref["alpha"].reshape(F, N)[fin])
    ev = rel(s64[0], ref["Vhat"].reshape(F, p.nz, N))
    e = rel(x64, ref_xi)
    xm, _, _ = gpu_run(p, Wd, u0, delta, 1)
    em = rel(xm, ref_xi)
    say("multi5 delta", delta, "active", act, "FP64 alpha / Vhat / xi", ea, ev, e, "mixed xi", em)
    assert max(ea, ev, e) <= TOL and em <= MIXED_TOL
