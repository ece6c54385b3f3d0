"""Reverse (VJP) and tangent (JVP) derivatives of the inversion map W -> xi
(oracle; test infrastructure only).

Conventions: complex arrays carry the real inner product
<a, b> = Re sum conj(a) b; a cotangent g of xi is what PyTorch stores as the
gradient of a real loss (dL/dRe + i dL/dIm), and the VJP returns the W (and
u0) cotangents in the same convention, so <vjp(g), dW> = <g, jvp(dW)>.

Derivation, stage by stage (the forward is Algorithm 2 as in invert.py):

(d) xi = num / den, num = sum_f conj(u_f) v_f, den = sum_f |u_f|^2:
    vbar_f = g u_f / den, ubar_f = (conj(g) (v_f - xi u_f) - g conj(xi) u_f) / den.
(c) u_f = u0_f + K_f v_f with K_f = omega^2 (kappa *), kappa even, so
    K_f^H y = conj(K_f conj(y)); v_f = crop(IFFT2(V^_f)) so
    V^bar_f = FFT2(pad(vbar_f)) / N.
(b) per solved system, M = A^H A + alpha I, v^ = M^-1 A^H w:
    w^bar = A M^-1 v^bar, and when alpha is the discrepancy root
    (phi(alpha, w) = T, phi = ||A v^ - w||^2) the implicit derivative
    d alpha = (dT - <q, dw>) / phi_a with phi_a = 2 alpha v^H M^-1 v^ and
    q = 2 (-alpha A M^-1 v^ - r), r = A v^ - w, adds
    w^bar -= (s / phi_a) q and Tbar_f += s / phi_a, s = -Re(v^bar^H M^-1 v^).
    The floor and zero branches are locally constant in alpha / v^.
(a) W^ = FFT2(W) unnormalized: Wbar = N IFFT2(W^bar); the threshold
    T_f = tau^2 delta^2 ||W_f||^2 adds 2 tau^2 delta^2 Tbar_f W_f.

Parity: pinned by tests/test_oracle_adjoint.py (the dot-product identity
between the two maps, central finite differences, adjointness of the linear
stages).
"""
from __future__ import annotations

import numpy as np

from . import model
from .invert import invert
from .regularize import ETA, TAU, ROOT


def _volume_adjoint(p, f, y):
    return np.conj(model.volume_potential(p, f, np.conj(y)))


def _systems(p, f, What_f, Vhat_f, alpha, branch):
    """Per active system: (indices, A, w, v, alpha, branch, Minv) with Minv
    a function applying (A^H A + alpha I)^-1 to a batch of vectors."""
    tab, idx = model.system_table(p, f)
    N = p.px * p.py
    act = np.nonzero(branch != 0)[0]
    A = model.system_matrices(p, f, tab, idx, act)
    w = What_f.reshape(p.nd, N).T[act]
    v = Vhat_f.reshape(p.nz, N).T[act]
    al = alpha[act]
    U, s, Vh = np.linalg.svd(A, full_matrices=True)
    lam = np.zeros((len(act), p.nz))
    r = min(p.nd, p.nz)
    lam[:, :r] = s[:, :r] ** 2

    def Minv(x):
        c = np.einsum("sij,sj->si", Vh, x) / (lam + al[:, None])
        return np.einsum("sji,sj->si", Vh.conj(), c)

    return act, A, w, v, al, branch[act], Minv


def vjp(p, W, u0, delta, g_xi, tau=TAU, eta=ETA, weights=None):
    """Cotangents (Wbar, u0bar) of xi = invert(W, u0) for the xi cotangent
    g_xi (shape of xi; combine = least squares, optionally weighted: every
    frequency's terms carry its weight)."""
    W = np.asarray(W, np.complex128)
    xi, st = invert(p, W, u0, delta, tau, eta, stages=True, weights=weights)
    u, v = st["u"], st["v"]
    wt = np.ones(p.n_omega) if weights is None else np.asarray(weights, np.float64)
    den = np.sum(wt[:, None, None, None] * np.abs(u) ** 2, axis=0)
    inv = np.where(den > 0, 1.0 / np.where(den > 0, den, 1.0), 0.0)
    N = p.px * p.py
    Wbar = np.zeros_like(W)
    u0bar = np.zeros_like(u)
    for f in range(p.n_omega):
        vbar = wt[f] * g_xi * u[f] * inv
        ubar = wt[f] * (np.conj(g_xi) * (v[f] - xi * u[f]) - g_xi * np.conj(xi) * u[f]) * inv
        u0bar[f] = ubar
        vbar = vbar + _volume_adjoint(p, f, ubar)
        Vbar = np.fft.fft2(model.embed(p, vbar)) / N
        act, A, w, vh, al, br, Minv = _systems(p, f, st["What"][f], st["Vhat"][f],
                                              st["alpha"][f], st["branch"][f])
        vb = Vbar.reshape(p.nz, N).T[act]
        x1 = Minv(vb)
        wbar = np.einsum("sjl,sl->sj", A, x1)
        Tbar = 0.0
        root = br == ROOT
        if np.any(root):
            x2 = Minv(vh)
            r = np.einsum("sjl,sl->sj", A, vh) - w
            s = -np.real(np.sum(np.conj(vb) * x2, axis=1))
            phia = 2.0 * al * np.real(np.sum(np.conj(vh) * x2, axis=1))
            q = 2.0 * (-al[:, None] * np.einsum("sjl,sl->sj", A, x2) - r)
            c = np.where(root, s / np.where(root, phia, 1.0), 0.0)
            wbar = wbar - c[:, None] * q
            Tbar = float(np.sum(c))
        What_bar = np.zeros((N, p.nd), np.complex128)
        What_bar[act] = wbar
        What_bar = What_bar.T.reshape(p.nd, p.py, p.px)
        Wbar[f] = N * np.fft.ifft2(What_bar) + 2.0 * (tau * delta) ** 2 * Tbar * W[f]
    return Wbar, u0bar


def jvp(p, W, u0, delta, dW, tau=TAU, eta=ETA, weights=None):
    """Tangent of xi for a W tangent dW (u0 held fixed)."""
    W = np.asarray(W, np.complex128)
    xi, st = invert(p, W, u0, delta, tau, eta, stages=True, weights=weights)
    u, v = st["u"], st["v"]
    wt = np.ones(p.n_omega) if weights is None else np.asarray(weights, np.float64)
    den = np.sum(wt[:, None, None, None] * np.abs(u) ** 2, axis=0)
    inv = np.where(den > 0, 1.0 / np.where(den > 0, den, 1.0), 0.0)
    N = p.px * p.py
    acc = np.zeros_like(xi)
    for f in range(p.n_omega):
        dWh = np.fft.fft2(dW[f])
        dT = 2.0 * (tau * delta) ** 2 * np.real(np.vdot(W[f], dW[f]))
        act, A, w, vh, al, br, Minv = _systems(p, f, st["What"][f], st["Vhat"][f],
                                              st["alpha"][f], st["branch"][f])
        dw = dWh.reshape(p.nd, N).T[act]
        b = np.einsum("sjl,sj->sl", A.conj(), dw)
        root = br == ROOT
        if np.any(root):
            x2 = Minv(vh)
            r = np.einsum("sjl,sl->sj", A, vh) - w
            phia = 2.0 * al * np.real(np.sum(np.conj(vh) * x2, axis=1))
            q = 2.0 * (-al[:, None] * np.einsum("sjl,sl->sj", A, x2) - r)
            da = np.where(root, (dT - np.real(np.sum(np.conj(q) * dw, axis=1)))
                          / np.where(root, phia, 1.0), 0.0)
            b = b - da[:, None] * vh
        dvh = Minv(b)
        dV = np.zeros((N, p.nz), np.complex128)
        dV[act] = dvh
        dV = dV.T.reshape(p.nz, p.py, p.px)
        dv = model.crop(p, np.fft.ifft2(dV))
        du = model.volume_potential(p, f, dv)
        acc += wt[f] * (np.conj(u[f]) * dv + np.conj(du) * (v[f] - xi * u[f])
                        - xi * np.conj(u[f]) * du)
    return acc * inv


def power_iteration(p, W, u0, delta, iters=20, seed=(5, 5)):
    """Largest singular value of J = d xi / d W (real-linear) by power
    iteration on J^T J; returns (sigma estimates per iteration, final
    direction)."""
    rng = np.random.default_rng(list(seed))
    x = rng.standard_normal(W.shape) + 1j * rng.standard_normal(W.shape)
    x /= np.linalg.norm(x)
    est = []
    for _ in range(iters):
        y = jvp(p, W, u0, delta, x)
        z, _ = vjp(p, W, u0, delta, y)
        lam = float(np.real(np.vdot(x, z)))
        est.append(np.sqrt(max(lam, 0.0)))
        x = z / np.linalg.norm(z)
    return np.array(est), x
