"""HIP-graph replay and the uneven batch (through the C ABI).

Graph replays are checked against eager runs bitwise, several times in a
row, with the input buffers rewritten between replays (a captured inversion
contains no memset nodes; its zero fills are kernels). The batch of uneven
grids is checked bitwise against per-plan eager inversions, and its
smallest instance against the oracle."""
import sys

import numpy as np
import pytest

from oracle import forward, invert
from paper_1911_10487_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-graph]", *a, flush=True)
    sys.stdout.flush()


def _data(p, delta, born=True):
    xi = synth.contrast(p)
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=born)
    return synth.add_noise(p, W, delta), u0


@pytest.mark.parametrize("precision,regularizer", [(0, 0), (1, 0), (0, 1)])
def test_graph_replays_match_eager(precision, regularizer):
    # regularizer 1: the truncated SVD's kernels captured as well
    import torch
    from paper_1911_10487_amd.flayer import Graph, Plan
    p = synth.make_problem("graph", 24, 20, 32, [2 * np.pi, 3 * np.pi], 3, (24, 0), (0.01,),
                           px=48, py=40)
    plan = Plan.from_problem(p, precision=precision, regularizer=regularizer)
    W1, u0 = _data(p, 0.01)
    W2 = synth.add_noise(p, W1, 0.02)
    ut = torch.from_numpy(u0).cuda()
    Wb = torch.from_numpy(W1).cuda()
    xi_g = torch.zeros((p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda")
    eager1 = plan.invert(torch.from_numpy(W1).cuda(), ut, 0.01).cpu().numpy()
    eager2 = plan.invert(torch.from_numpy(W2).cuda(), ut, 0.01).cpu().numpy()
    say("capture", precision, regularizer)
    g = Graph(plan, Wb, ut, 0.01, xi_g)
    for rep in range(3):
        for Wn, ref in ((W1, eager1), (W2, eager2)):
            Wb.copy_(torch.from_numpy(Wn).cuda())
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            got = xi_g.cpu().numpy()
            assert np.array_equal(got, ref), f"replay {rep} differs"
            # eager work between replays
            plan.invert(torch.from_numpy(W1).cuda(), ut, 0.01)
            torch.cuda.synchronize()
    g.close()
    plan.close()


def test_graph_replays_see_later_frequency_weights():
    """Weights set after the capture apply on replay (the kernels read them
    from device memory): a weight-0 frequency drops out of the replayed xi
    exactly as in an eager inversion with those weights."""
    import torch
    from paper_1911_10487_amd.flayer import Graph, Plan
    p = synth.make_problem("graphw", 24, 20, 32, [2 * np.pi, 3 * np.pi], 3, (25, 0), (0.01,),
                           px=48, py=40)
    plan = Plan.from_problem(p)
    W, u0 = _data(p, 0.01)
    Wb, ut = torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda()
    xi_g = torch.zeros((p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda")
    g = Graph(plan, Wb, ut, 0.01, xi_g)
    for wt in ([1.0, 0.0], [0.3, 1.7], None):
        plan.set_frequency_weights(wt)
        eager = plan.invert(Wb, ut, 0.01).cpu().numpy()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(xi_g.cpu().numpy(), eager), wt
        ref = invert.invert(p, W, u0, 0.01, weights=wt)
        say("graph weights", wt, np.linalg.norm(eager - ref) / np.linalg.norm(ref))
        assert np.linalg.norm(eager - ref) <= 1e-10 * np.linalg.norm(ref)
    g.close()
    plan.close()


def test_uneven_batch_matches_eager_and_oracle():
    import torch
    from paper_1911_10487_amd.flayer import Batch, Plan
    insts = synth.workload("uneven")
    plans, Ws, us, ds, eager = [], [], [], [], []
    for p in insts:
        say("instance", p.name, p.nx, p.nz, "delta", p.deltas[0])
        plan = Plan.from_problem(p, precision=1)
        xi_t = torch.from_numpy(synth.contrast(p)).cuda()
        u0 = torch.from_numpy(synth.incident_field(p)).cuda()
        W = plan.forward(xi_t, u0)
        torch.cuda.synchronize()
        Wd = torch.from_numpy(synth.add_noise(p, W.cpu().numpy(), p.deltas[0])).cuda()
        plans.append(plan)
        Ws.append(Wd)
        us.append(u0)
        ds.append(p.deltas[0])
        eager.append(plan.invert(Wd, u0, p.deltas[0]).cpu().numpy())
    b = Batch(plans)
    xis = [torch.empty((p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda") for p in insts]
    for rep in range(2):
        b.invert(Ws, us, ds, xis)
        torch.cuda.synchronize()
        for x, e in zip(xis, eager):
            assert np.array_equal(x.cpu().numpy(), e)
    b.close()
    # the smallest instance against the oracle (mixed gate 1e-4)
    p = insts[0]
    ref = invert.invert(p, Ws[0].cpu().numpy(), us[0].cpu().numpy(), ds[0])
    err = np.linalg.norm(eager[0] - ref) / np.linalg.norm(ref)
    say("uneven[0] mixed vs oracle", err)
    assert err <= 1e-4
    for pl in plans:
        pl.close()
