"""The Python binding refuses arrays that do not match the plan before any
kernel runs: a wrong shape, dtype or device would otherwise make the
kernels read or write past the tensors."""
import sys

import numpy as np
import pytest

from paper_1911_10487_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-binding]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def plan_and_inputs():
    import torch
    from paper_1911_10487_amd.flayer import Plan
    assert torch.cuda.is_available()
    p = synth.make_problem("bind", 16, 16, 16, [2 * np.pi, 3 * np.pi], 2, (61, 0), (0.01,))
    plan = Plan.from_problem(p)
    W = torch.zeros((p.n_omega, p.nd, p.py, p.px), dtype=torch.complex128, device="cuda")
    u0 = torch.zeros((p.n_omega, p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda")
    yield p, plan, W, u0
    plan.close()


def test_invert_refuses_mismatched_arrays(plan_and_inputs):
    import torch
    p, plan, W, u0 = plan_and_inputs
    say("binding checks", p.nx, p.ny, p.nz)
    bad = [
        (W[:, :-1].contiguous(), u0),                      # one data plane short
        (W.to(torch.complex64), u0),                       # complex64 on a complex128 plan
        (W, u0[:1].contiguous()),                          # one frequency short
        (W.cpu(), u0),                                     # host memory
        (W.transpose(2, 3), u0),                           # not contiguous
    ]
    for Wb, ub in bad:
        with pytest.raises(ValueError):
            plan.invert(Wb, ub, 0.01)
    with pytest.raises(ValueError):
        plan.invert(W, u0, 0.01, torch.empty((p.nz, p.ny, p.nx + 1), dtype=torch.complex128,
                                             device="cuda"))
    with pytest.raises(ValueError):
        plan.invert(W, u0, 0.01, torch.empty((p.nz, p.ny, p.nx), dtype=torch.complex64,
                                             device="cuda"))


def test_derivatives_and_forward_refuse_mismatched_arrays(plan_and_inputs):
    import torch
    from paper_1911_10487_amd.flayer import Batch, Graph
    p, plan, W, u0 = plan_and_inputs
    with pytest.raises(ValueError):
        plan.vjp(W, u0, 0.01, torch.zeros((p.nz, p.ny), dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError):
        plan.jvp(W, u0, 0.01, W[:1])
    xi = torch.zeros((p.nz, p.ny, p.nx), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        plan.forward(xi.to(torch.complex128), u0)   # xi is real
    with pytest.raises(ValueError):
        plan.forward(xi[:-1].contiguous(), u0)
    with pytest.raises(ValueError):
        Graph(plan, W, u0, 0.01, torch.zeros((1,), dtype=torch.complex128, device="cuda"))
    b = Batch([plan])
    with pytest.raises(ValueError):
        b.invert([W[:, :-1].contiguous()], [u0], [0.01],
                 [torch.zeros((p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda")])
    with pytest.raises(ValueError):
        b.invert([W, W], [u0], [0.01], [xi])
    b.close()
