"""GPU derivatives (fl_invert_vjp / fl_invert_jvp through the C ABI) against
the oracle's hand-derived VJP / JVP, plus the dot-product identity and
central finite differences on the GPU itself. FP64 path: relative L2
<= 1e-10 for noisy data, as for the forward map."""
import sys

import numpy as np
import pytest

from oracle import adjoint, forward
from paper_1911_10487_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print("[gpu-adjoint]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def case():
    import torch
    assert torch.cuda.is_available()
    p = synth.make_problem("adjgpu", 20, 12, 16, [2 * np.pi, 3 * np.pi], 3, (23, 0), (0.02,),
                           px=40, py=30)
    xi = synth.contrast(p) + 0.02
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=True)
    Wd = synth.add_noise(p, W, 0.02)
    return p, Wd, u0, 0.02


def _plan(p, **kw):
    from paper_1911_10487_amd.flayer import Plan
    return Plan.from_problem(p, **kw)


def test_vjp_matches_oracle(case):
    import torch
    p, W, u0, d = case
    g = synth.random_field((p.nz, p.ny, p.nx), (40,))
    say("vjp", p.nx, p.ny, p.nz)
    plan = _plan(p)
    gW, gu = plan.vjp(torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda(), d,
                      torch.from_numpy(g).cuda(), want_u0=True)
    torch.cuda.synchronize()
    gW, gu = gW.cpu().numpy(), gu.cpu().numpy()
    plan.close()
    rW, ru = adjoint.vjp(p, W, u0, d, g)
    say("vjp rel err W", rel(gW, rW), "u0", rel(gu, ru))
    assert rel(gW, rW) <= TOL and rel(gu, ru) <= TOL


def test_jvp_matches_oracle_and_dot_product_identity(case):
    import torch
    p, W, u0, d = case
    dW = synth.random_field(W.shape, (41,))
    g = synth.random_field((p.nz, p.ny, p.nx), (42,))
    plan = _plan(p)
    Wt, ut = torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda()
    jv = plan.jvp(Wt, ut, d, torch.from_numpy(dW).cuda()).cpu().numpy()
    gW, _ = plan.vjp(Wt, ut, d, torch.from_numpy(g).cuda())
    gW = gW.cpu().numpy()
    plan.close()
    ref = adjoint.jvp(p, W, u0, d, dW)
    say("jvp rel err", rel(jv, ref))
    assert rel(jv, ref) <= TOL
    lhs = np.real(np.vdot(g, jv))
    rhs = np.real(np.vdot(gW, dW))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_jvp_matches_gpu_central_differences(case):
    import torch
    p, W, u0, d = case
    dW = synth.random_field(W.shape, (43,))
    dW *= np.linalg.norm(W) / np.linalg.norm(dW)
    h = 1e-6
    plan = _plan(p)
    ut = torch.from_numpy(u0).cuda()
    xp = plan.invert(torch.from_numpy(W + h * dW).cuda(), ut, d).cpu().numpy()
    xm = plan.invert(torch.from_numpy(W - h * dW).cuda(), ut, d).cpu().numpy()
    jv = plan.jvp(torch.from_numpy(W).cuda(), ut, d, torch.from_numpy(dW).cuda()).cpu().numpy()
    plan.close()
    fd = (xp - xm) / (2 * h)
    say("fd rel err", rel(fd, jv))
    assert rel(fd, jv) <= 1e-5


def test_autograd_function_gradient(case):
    import torch
    from paper_1911_10487_amd.autograd import invert as finvert
    p, W, u0, d = case
    plan = _plan(p)
    Wt = torch.from_numpy(W).cuda().requires_grad_(True)
    ut = torch.from_numpy(u0).cuda()
    xi = finvert(Wt, ut, d, plan)
    loss = (xi.real ** 2).sum()
    loss.backward()
    g = (2 * xi.real).detach().to(torch.complex128)
    gW, _ = plan.vjp(Wt.detach(), ut, d, g)
    assert torch.allclose(Wt.grad, gW, rtol=0, atol=0)
    plan.close()


def test_power_iteration_matches_oracle(case):
    import torch
    from paper_1911_10487_amd.autograd import power_iteration
    p, W, u0, d = case
    plan = _plan(p)
    est, x = power_iteration(plan, torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda(), d,
                             iters=20, seed=3)
    plan.close()
    # monotone Rayleigh quotients, and the same estimate as the oracle's
    # iteration started from the same direction converges to
    assert all(b >= a * (1 - 1e-9) for a, b in zip(est, est[1:]))
    x0 = x.cpu().numpy()
    y = adjoint.jvp(p, W, u0, d, x0)
    z, _ = adjoint.vjp(p, W, u0, d, y)
    sig = np.sqrt(np.real(np.vdot(x0, z)))
    say("power iteration", est[-1], sig)
    assert abs(est[-1] - sig) <= 1e-3 * sig


def test_mixed_precision_derivatives(case):
    """Mixed precision (FP32 stage (c) transforms): VJP and JVP against the
    oracle within 1e-4, and the dot-product identity of the two GPU maps
    within the same bound."""
    import torch
    p, W, u0, d = case
    g = synth.random_field((p.nz, p.ny, p.nx), (44,))
    dW = synth.random_field(W.shape, (45,))
    plan = _plan(p, precision=1)
    Wt, ut = torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda()
    gW, _ = plan.vjp(Wt, ut, d, torch.from_numpy(g).cuda())
    gW = gW.cpu().numpy()
    jv = plan.jvp(Wt, ut, d, torch.from_numpy(dW).cuda()).cpu().numpy()
    plan.close()
    rW, _ = adjoint.vjp(p, W, u0, d, g)
    rj = adjoint.jvp(p, W, u0, d, dW)
    say("mixed vjp rel err", rel(gW, rW), "jvp", rel(jv, rj))
    assert rel(gW, rW) <= 1e-4 and rel(jv, rj) <= 1e-4
    lhs = np.real(np.vdot(g, jv))
    rhs = np.real(np.vdot(gW, dW))
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


@pytest.mark.parametrize("precision", [0, 1])
def test_chunked_factorization_matches_resident(case, precision):
    """A plan whose solver workspace holds a few dozen systems (so that the
    derivative passes re-factorize chunk by chunk) gives bitwise the same
    xi, VJP and JVP as a plan holding every system at once (one
    factorization per system in both, as the derivative calls use)."""
    import torch
    p, W, u0, d = case
    g = synth.random_field((p.nz, p.ny, p.nx), (45,))
    dW = synth.random_field(W.shape, (46,))
    Wt, ut = torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda()
    gt, dWt = torch.from_numpy(g).cuda(), torch.from_numpy(dW).cuda()
    outs = []
    for mc in (0, 37):
        say("chunk", mc, "precision", precision)
        plan = _plan(p, precision=precision, max_chunk=mc, factor_per_system=1)
        xi = plan.invert(Wt, ut, d).cpu().numpy()
        n_act = plan.active_systems()
        gW, gu = plan.vjp(Wt, ut, d, gt, want_u0=True)
        jv = plan.jvp(Wt, ut, d, dWt)
        torch.cuda.synchronize()
        outs.append((xi, gW.cpu().numpy(), gu.cpu().numpy(), jv.cpu().numpy()))
        plan.close()
    assert n_act > 2 * 37, n_act
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", [0, 1])
def test_orbit_chunks_match_resident(case, precision):
    """Shared (per-orbit) factorizations taken a few dozen orbits at a time
    (max_chunk: the forward factorizes chunk after chunk, the derivative
    passes re-factorize every chunk but the one still in the workspace) give
    bitwise the xi, VJP and JVP of a plan holding every active orbit at
    once, and the oracle's xi."""
    import torch
    from oracle import invert
    p, W, u0, d = case
    g = synth.random_field((p.nz, p.ny, p.nx), (49,))
    dW = synth.random_field(W.shape, (50,))
    Wt, ut = torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda()
    gt, dWt = torch.from_numpy(g).cuda(), torch.from_numpy(dW).cuda()
    outs = []
    for mc in (0, 23):
        say("orbit chunk", mc, "precision", precision)
        plan = _plan(p, precision=precision, max_chunk=mc)
        xi = plan.invert(Wt, ut, d).cpu().numpy()
        n_orb = plan.factorized_systems()
        gW, gu = plan.vjp(Wt, ut, d, gt, want_u0=True)
        jv = plan.jvp(Wt, ut, d, dWt)
        xi2 = plan.invert(Wt, ut, d).cpu().numpy()
        torch.cuda.synchronize()
        outs.append((xi, gW.cpu().numpy(), gu.cpu().numpy(), jv.cpu().numpy(), xi2))
        plan.close()
    assert n_orb > 3 * 23, n_orb
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    if precision == 0:
        ref = invert.invert(p, W, u0, d)
        say("orbit chunks vs oracle", rel(outs[1][0], ref))
        assert rel(outs[1][0], ref) <= TOL


def test_weighted_derivatives_match_oracle(case):
    import torch
    p, W, u0, d = case
    g = synth.random_field((p.nz, p.ny, p.nx), (47,))
    dW = synth.random_field(W.shape, (48,))
    wt = [0.3, 1.7]
    plan = _plan(p)
    plan.set_frequency_weights(wt)
    Wt, ut = torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda()
    gW, _ = plan.vjp(Wt, ut, d, torch.from_numpy(g).cuda())
    jv = plan.jvp(Wt, ut, d, torch.from_numpy(dW).cuda())
    gW, jv = gW.cpu().numpy(), jv.cpu().numpy()
    plan.close()
    rW, _ = adjoint.vjp(p, W, u0, d, g, weights=wt)
    rj = adjoint.jvp(p, W, u0, d, dW, weights=wt)
    say("weighted vjp", rel(gW, rW), "jvp", rel(jv, rj))
    assert rel(gW, rW) <= TOL and rel(jv, rj) <= TOL
