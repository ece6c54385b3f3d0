"""fl_invert_vjp_noalloc (derivative workspaces in the library's static
device array) called through the C ABI against fl_invert_vjp on the same
plan: two calls in a row on different plans, the second smaller, each
matching the allocating entry point (the same kernels, so bitwise); a plan
whose workspace exceeds the array is refused before any kernel runs."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import forward
from paper_1911_10487_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


def _case(name, nx, ny, nz, omegas, px, py, seed):
    p = synth.make_problem(name, nx, ny, nz, omegas, 3, (seed, 0), (0.02,), px=px, py=py)
    xi = synth.contrast(p) + 0.02
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=True)
    return p, synth.add_noise(p, W, 0.02), u0


def _vjp_c(fn, plan, W, u0, g, gW, gu):
    import torch
    st = fn(plan._h, ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(u0.data_ptr()), 0.02,
            ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(gW.data_ptr()),
            ctypes.c_void_p(gu.data_ptr()))
    torch.cuda.synchronize()
    return st


def test_noalloc_vjp_matches_allocating_vjp():
    import torch
    from paper_1911_10487_amd.flayer import FL_OK, Plan, lib
    assert torch.cuda.is_available()
    L = lib()
    cases = [_case("noalloc-a", 20, 12, 16, [2 * np.pi, 3 * np.pi], 40, 30, 81),
             _case("noalloc-b", 16, 16, 16, [2 * np.pi], 32, 32, 82)]
    for p, W, u0 in cases:
        for prec in (0, 1):
            say("case", p.name, p.nx, p.ny, p.nz, "F", p.n_omega, "precision", prec)
            plan = Plan.from_problem(p, precision=prec)
            Wt, ut = torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda()
            g = torch.from_numpy(synth.random_field((p.nz, p.ny, p.nx), (83,))).cuda()
            outs = []
            for fn in (L.fl_invert_vjp_noalloc, L.fl_invert_vjp):
                gW = torch.full(W.shape, np.nan, dtype=torch.complex128, device="cuda")
                gu = torch.full(u0.shape, np.nan, dtype=torch.complex128, device="cuda")
                assert _vjp_c(fn, plan, Wt, ut, g, gW, gu) == FL_OK, L.fl_last_error()
                outs.append((gW.cpu().numpy(), gu.cpu().numpy()))
            plan.close()
            for a, b in zip(*outs):
                assert np.all(np.isfinite(a))
                err = np.linalg.norm(a - b) / np.linalg.norm(b)
                say("noalloc vs vjp", err)
                assert err <= 1e-10
                assert np.array_equal(a, b)


def test_noalloc_refuses_a_plan_beyond_the_array():
    import torch
    from paper_1911_10487_amd.flayer import FL_EINVAL, Plan, lib
    L = lib()
    # (4 F nx ny nz + 2 F nz px py) complex128 = 75 MiB > 64 MiB
    p = synth.make_problem("noalloc-big", 64, 64, 32, [2 * np.pi] * 3, 2, (84, 0), (0.02,))
    plan = Plan.from_problem(p)
    W = torch.zeros((p.n_omega, p.nd, p.py, p.px), dtype=torch.complex128, device="cuda")
    u0 = torch.zeros((p.n_omega, p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda")
    g = torch.zeros((p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda")
    gW, gu = torch.zeros_like(W), torch.zeros_like(u0)
    st = _vjp_c(L.fl_invert_vjp_noalloc, plan, W, u0, g, gW, gu)
    msg = L.fl_last_error().decode()
    say("refused:", msg)
    assert st == FL_EINVAL and "FL_NOALLOC_SCRATCH_MB" in msg
    plan.close()
