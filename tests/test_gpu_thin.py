"""Thin data layer on the GPU (nd = 2 planes 0.01 apart, off X's z-lattice,
wide systems) against the oracle: tables and data operator, the inversion
in both precisions and both kernel tables, element by element."""
import sys

import numpy as np
import pytest

from oracle import forward, invert
from paper_1911_10487_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print("[gpu-thin]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def thin():
    import torch
    assert torch.cuda.is_available()
    p = synth.thin_problem("thin", 20, 12, 16, [2 * np.pi, 1.5 * 2 * np.pi], 3, (9, 2),
                           gap=0.3, spacing=0.01, px=40, py=30)
    xi = synth.contrast(p)
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=True)
    return p, xi, u0, W


def _run(p, W, u0, delta, **kw):
    import torch
    from paper_1911_10487_amd.flayer import (Plan, TAP_ALPHA, TAP_BRANCH, TAP_U, TAP_V,
                                             TAP_VHAT)
    say("plan", p.nx, p.ny, p.nz, "nd", p.nd, "delta", delta, kw)
    plan = Plan.from_problem(p, **kw)
    xi = plan.invert(torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda(), delta)
    F, N = p.n_omega, p.px * p.py
    cw = np.complex64 if kw.get("precision", 0) == 1 else np.complex128
    st = {"Vhat": plan.tap(TAP_VHAT, cw, (F, p.nz, p.py, p.px)),
          "v": plan.tap(TAP_V, np.complex128, (F, p.nz, p.ny, p.nx)),
          "u": plan.tap(TAP_U, np.complex128, (F, p.nz, p.ny, p.nx)),
          "alpha": plan.tap(TAP_ALPHA, np.float64, (F, N)),
          "branch": plan.tap(TAP_BRANCH, np.int8, (F, N))}
    out = xi.cpu().numpy()
    plan.close()
    return out, st


def test_thin_forward_data_matches_oracle(thin):
    import torch
    from paper_1911_10487_amd.flayer import Plan
    p, xi, u0, W = thin
    plan = Plan.from_problem(p)
    got = plan.forward(torch.from_numpy(xi).cuda(), torch.from_numpy(u0).cuda()).cpu().numpy()
    plan.close()
    say("thin Born data", rel(got, W))
    assert rel(got, W) <= 1e-12


@pytest.mark.parametrize("delta", [0.01, 0.0])
def test_thin_inversion_matches_oracle(thin, delta):
    # delta = 0 solves every system at the floor alpha; the gate is the same
    # 1e3 u eta^-1/2 as for the thick layer (rounding of the FFT tables,
    # amplified by the floor's conditioning)
    p, xi, u0, W = thin
    Wd = synth.add_noise(p, W, delta)
    ref_xi, ref = invert.invert(p, Wd, u0, delta, stages=True)
    got, st = _run(p, Wd, u0, delta)
    tol = TOL if delta > 0 else 1e3 * 2.0 ** -53 * 1e5
    br = ref["branch"].reshape(st["branch"].shape)
    assert np.array_equal(br, st["branch"])
    fin = np.isfinite(ref["alpha"].reshape(st["alpha"].shape))
    a_ref = ref["alpha"].reshape(st["alpha"].shape)
    ra = np.max(np.abs(st["alpha"][fin] - a_ref[fin]) / a_ref[fin])
    say("thin delta", delta, "alpha", ra, "Vhat", rel(st["Vhat"], ref["Vhat"]), "xi",
        rel(got, ref_xi), "branches", np.unique(br, return_counts=True))
    assert ra <= tol
    assert rel(st["Vhat"], ref["Vhat"]) <= tol
    assert rel(st["u"], ref["u"]) <= tol
    assert rel(got, ref_xi) <= tol


def test_thin_mixed_and_closed_form(thin):
    p, xi, u0, W = thin
    Wd = synth.add_noise(p, W, 0.01)
    ref_xi = invert.invert(p, Wd, u0, 0.01)
    got, _ = _run(p, Wd, u0, 0.01, precision=1)
    say("thin mixed", rel(got, ref_xi))
    assert rel(got, ref_xi) <= 1e-4
    kw = dict(kernel_mode=1, damping=0.02, eta=1e-4)
    ref_c = invert.invert(p, Wd, u0, 0.01, **kw)
    got_c, _ = _run(p, Wd, u0, 0.01, **kw)
    say("thin closed form", rel(got_c, ref_c))
    assert rel(got_c, ref_c) <= TOL


def test_thin_layer_has_no_derivatives(thin):
    import torch
    from paper_1911_10487_amd.flayer import FlError, FL_EUNSUPPORTED, Plan
    p, xi, u0, W = thin
    plan = Plan.from_problem(p)
    with pytest.raises(FlError) as e:
        plan.vjp(torch.from_numpy(W).cuda(), torch.from_numpy(u0).cuda(), 0.01,
                 torch.ones((p.nz, p.ny, p.nx), dtype=torch.complex128, device="cuda"))
    assert e.value.status == FL_EUNSUPPORTED
    plan.close()


@pytest.mark.parametrize("delta", [0.01, 0.0])
def test_thin_tsvd_matches_oracle(thin, delta):
    # regularizer 1: the truncated SVD with the discrepancy-chosen count of
    # triplets (the paper's best performer), against the oracle's rule "tsvd":
    # the same count for every solved system and the same solution
    p, xi, u0, W = thin
    Wd = synth.add_noise(p, W, delta)
    ref_xi, ref = invert.invert(p, Wd, u0, delta, rule="tsvd", stages=True)
    got, st = _run(p, Wd, u0, delta, regularizer=1)
    k_ref = ref["alpha"].reshape(st["alpha"].shape)
    act = np.isfinite(st["alpha"])
    assert np.array_equal(st["alpha"][act], k_ref[act])
    assert not np.any(k_ref[~act])
    say("thin tsvd delta", delta, "counts", np.unique(k_ref, return_counts=True), "Vhat",
        rel(st["Vhat"], ref["Vhat"]), "xi", rel(got, ref_xi))
    tol = TOL if delta > 0 else 1e3 * 2.0 ** -53 * 1e5
    assert rel(st["Vhat"], ref["Vhat"]) <= tol
    assert rel(got, ref_xi) <= tol
