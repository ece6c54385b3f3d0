"""Pins of the oracle's VJP / JVP of W -> xi (no GPU)."""
import numpy as np
import pytest

from oracle import adjoint, forward, invert, model
from paper_1911_10487_amd import synth


def rdot(a, b):
    return float(np.real(np.vdot(a, b)))


@pytest.fixture(scope="module")
def prob():
    p = synth.make_problem("adj", 6, 5, 4, [2 * np.pi, 3 * np.pi], 2, (21, 0), (0.02,),
                           px=12, py=10)
    xi = synth.contrast(p) + 0.05
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0)
    Wd = synth.add_noise(p, W, 0.02)
    return p, Wd, u0, 0.02


def test_branches_cover_root_floor_and_zero(prob):
    p, W, u0, d = prob
    _, st = invert.invert(p, W, u0, d, stages=True)
    b = st["branch"].ravel()
    assert (b == 2).sum() > 5 and (b == 0).sum() > 5


def test_dot_product_identity(prob):
    p, W, u0, d = prob
    g = synth.random_field((p.nz, p.ny, p.nx), (30,))
    dW = synth.random_field(W.shape, (31,))
    Wbar, _ = adjoint.vjp(p, W, u0, d, g)
    lhs = rdot(g, adjoint.jvp(p, W, u0, d, dW))
    rhs = rdot(Wbar, dW)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def _xi(p, W, u0, d):
    return invert.invert(p, W, u0, d)


def test_jvp_matches_central_differences(prob):
    p, W, u0, d = prob
    dW = synth.random_field(W.shape, (32,))
    dW *= np.linalg.norm(W) / np.linalg.norm(dW)
    h = 1e-6
    _, s0 = invert.invert(p, W, u0, d, stages=True)
    _, sp = invert.invert(p, W + h * dW, u0, d, stages=True)
    _, sm = invert.invert(p, W - h * dW, u0, d, stages=True)
    assert np.array_equal(s0["branch"], sp["branch"]) and np.array_equal(s0["branch"], sm["branch"])
    fd = (_xi(p, W + h * dW, u0, d) - _xi(p, W - h * dW, u0, d)) / (2 * h)
    jv = adjoint.jvp(p, W, u0, d, dW)
    assert np.linalg.norm(fd - jv) <= 1e-6 * np.linalg.norm(jv)


def test_u0_cotangent_matches_central_differences(prob):
    p, W, u0, d = prob
    g = synth.random_field((p.nz, p.ny, p.nx), (33,))
    du = synth.random_field(u0.shape, (34,))
    du *= np.linalg.norm(u0) / np.linalg.norm(du)
    h = 1e-6
    fd = (_xi(p, W, u0 + h * du, d) - _xi(p, W, u0 - h * du, d)) / (2 * h)
    _, u0bar = adjoint.vjp(p, W, u0, d, g)
    assert abs(rdot(g, fd) - rdot(u0bar, du)) <= 1e-6 * abs(rdot(g, fd))


def test_noise_free_map_derivatives(prob):
    # delta = 0: every system at the floor, so the map is linear in W
    p, W, u0, d = prob
    g = synth.random_field((p.nz, p.ny, p.nx), (35,))
    dW = synth.random_field(W.shape, (36,))
    Wbar, _ = adjoint.vjp(p, W, u0, 0.0, g)
    assert abs(rdot(g, adjoint.jvp(p, W, u0, 0.0, dW)) - rdot(Wbar, dW)) <= 1e-11 * np.linalg.norm(Wbar) * np.linalg.norm(dW)


def test_linear_stage_adjoints():
    p = synth.tiny_problem(nx=3, ny=4, nz=3, px=8, py=8)
    x = synth.random_field((p.nz, p.ny, p.nx), (37,))
    y = synth.random_field((p.nz, p.ny, p.nx), (38,))
    # volume potential: <y, K x> = <K^H y, x>
    assert abs(np.vdot(y, model.volume_potential(p, 0, x))
               - np.vdot(adjoint._volume_adjoint(p, 0, y), x)) < 1e-13 * np.linalg.norm(x) * np.linalg.norm(y)
    # crop(IFFT2(.)) and FFT2(pad(.)) / N
    V = synth.random_field((p.nz, p.py, p.px), (39,))
    N = p.px * p.py
    lhs = np.vdot(y, model.crop(p, np.fft.ifft2(V)))
    rhs = np.vdot(np.fft.fft2(model.embed(p, y)) / N, V)
    assert abs(lhs - rhs) < 1e-14 * np.linalg.norm(V) * np.linalg.norm(y)


def test_power_iteration_finds_the_largest_singular_value():
    # tiny grid: J is small enough to build column by column from the JVP
    p = synth.make_problem("pw", 3, 3, 3, [2 * np.pi], 1, (22, 0), (0.05,), px=6, py=6)
    xi = synth.contrast(p) + 0.05
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0)
    W = synth.add_noise(p, W, 0.05)
    n = W.size
    cols = []
    for k in range(2 * n):
        e = np.zeros(n, np.complex128)
        e[k % n] = 1.0 if k < n else 1j
        jv = adjoint.jvp(p, W, u0, 0.05, e.reshape(W.shape)).ravel()
        cols.append(np.concatenate([jv.real, jv.imag]))
    J = np.stack(cols, axis=1)
    smax = np.linalg.svd(J, compute_uv=False)[0]
    est, _ = adjoint.power_iteration(p, W, u0, 0.05, iters=30)
    assert np.all(np.diff(est) >= -1e-12 * est[-1])
    assert abs(est[-1] - smax) <= 1e-3 * smax
