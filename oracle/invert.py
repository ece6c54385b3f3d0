"""Algorithm 2 end to end on the CPU (oracle; test infrastructure only).

Algorithm 2 (Section 4):
  item 1  for every frequency and horizontal wavenumber, solve the first-kind
          system of eq. (8) by a regularizing algorithm  -> V^(z', omega, Omega)
  item 2  V = F^-1[V^] on X, and U from eq. (9); this build evaluates eq. (9)
          in X as the linear convolution of v with the volume kernel (the
          in-X form of eq. 4), zero-padded in all three directions
  item 3  xi from u xi = V: v/u for one frequency, least squares over the
          frequencies otherwise (Section 5.2, last paragraph):
          xi = sum_f conj(u_f) v_f / sum_f |u_f|^2, xi = 0 where the
          denominator vanishes.

Shapes: W (n_omega, nd, py, px); u0 (n_omega, nz, ny, nx); xi (nz, ny, nx),
complex (the physical contrast is its real part).

Parity: pinned by tests/test_oracle_invert.py (consistency with the forward
model, the sign-flip invariance of the 2D transform, single-frequency and
duplicated-frequency reductions, Parseval for the noise level).
"""
from __future__ import annotations

import numpy as np

from . import model
from .regularize import TAU, ETA, tikhonov_dp, tsvd_dp


def system_noise_level(W_f: np.ndarray, delta: float) -> float:
    """delta_m = delta * ||W^delta_f||_2 over all nd*py*px samples."""
    return float(delta) * float(np.linalg.norm(W_f))


def solve_systems(p, f, What_f, delta, tau=TAU, eta=ETA, rule="tikhonov",
                  chunk=2048, tab=None, idx=None, kernel_mode=0, damping=0.0):
    """Algorithm 2 item 1 for one frequency. What_f: (nd, py, px) transformed
    data. Returns (Vhat (nz, py, px), alpha (py*px,), branch (py*px,))."""
    if tab is None:
        tab, idx = model.system_table(p, f, kernel_mode, damping)
    N = p.px * p.py
    wsys = What_f.reshape(p.nd, N).T                      # (N, nd)
    dm = system_noise_level_hat(What_f, delta, N)
    V = np.zeros((N, p.nz), np.complex128)
    alpha = np.full(N, np.inf)
    branch = np.zeros(N, np.int8)
    for s0 in range(0, N, chunk):
        ms = np.arange(s0, min(N, s0 + chunk))
        A = model.system_matrices(p, f, tab, idx, ms)
        if rule == "tikhonov":
            V[ms], alpha[ms], branch[ms] = tikhonov_dp(A, wsys[ms], dm, tau, eta)
        elif rule == "tsvd":
            V[ms], k = tsvd_dp(A, wsys[ms], dm, tau, eta)
            alpha[ms] = k
        else:
            raise ValueError(rule)
    return V.T.reshape(p.nz, p.py, p.px), alpha, branch


def system_noise_level_hat(What_f, delta, N):
    """The same delta_m computed from the transformed data via Parseval:
    ||W||^2 = ||W^||^2 / N."""
    return float(delta) * float(np.linalg.norm(What_f)) / np.sqrt(N)


def invert(p, W, u0, delta, tau=TAU, eta=ETA, combine="lsq", rule="tikhonov",
           stages=False, kernel_mode=0, damping=0.0):
    """W -> xi. With stages=True also returns a dict of per-frequency
    intermediates (What, Vhat, v, u, alpha, branch). kernel_mode / damping
    select the table of A (model.system_table)."""
    W = np.asarray(W, np.complex128)
    u0 = np.asarray(u0, np.complex128)
    nf = p.n_omega
    num = np.zeros((p.nz, p.ny, p.nx), np.complex128)
    den = np.zeros((p.nz, p.ny, p.nx), np.float64)
    per_f = []
    keep = {k: [] for k in ("What", "Vhat", "v", "u", "alpha", "branch")}
    for f in range(nf):
        What = np.fft.fft2(W[f])                                  # item 1 input
        Vhat, alpha, branch = solve_systems(p, f, What, delta, tau, eta, rule,
                                            kernel_mode=kernel_mode, damping=damping)
        v = model.crop(p, np.fft.ifft2(Vhat))                      # item 2
        u = u0[f] + model.volume_potential(p, f, v)
        num += np.conj(u) * v                                      # item 3
        den += np.abs(u) ** 2
        if combine == "per_frequency":
            per_f.append(_divide(np.conj(u) * v, np.abs(u) ** 2))
        if stages:
            for k, val in (("What", What), ("Vhat", Vhat), ("v", v), ("u", u),
                           ("alpha", alpha), ("branch", branch)):
                keep[k].append(val)
    xi = np.stack(per_f) if combine == "per_frequency" else _divide(num, den)
    if stages:
        return xi, {k: np.stack(val) for k, val in keep.items()}
    return xi


def _divide(num, den):
    out = np.zeros_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return out


def combine_lsq(u, v):
    """Item 3 on given stacks u, v (n_omega, ...)."""
    return _divide(np.sum(np.conj(u) * v, axis=0), np.sum(np.abs(u) ** 2, axis=0))
