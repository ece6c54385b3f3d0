"""Algorithm 2 end to end on the CPU (oracle; test infrastructure only).

Algorithm 2 (Section 4):
  item 1  for every frequency and horizontal wavenumber, solve the first-kind
          system of eq. (8) by a regularizing algorithm  -> V^(z', omega, Omega)
  item 2  V = F^-1[V^] on X, and U from eq. (9); the oracle evaluates eq. (9)
          in X as the linear convolution of v with the volume kernel (the
          in-X form of eq. 4), zero-padded in all three directions
  item 3  xi from u xi = V: v/u for one frequency, least squares over the
          frequencies otherwise (Section 5.2, last paragraph):
          xi = sum_f conj(u_f) v_f / sum_f |u_f|^2, xi = 0 where the
          denominator vanishes. Section 5 notes that the frequencies give
          reconstructions of different accuracy; optional weights w_f >= 0
          (frequency selection when 0/1) make it the weighted least squares
          sum_f w_f conj(u_f) v_f / sum_f w_f |u_f|^2, and a frequency of
          weight 0 is not solved at all.

Shapes: W (n_omega, nd, py, px); u0 (n_omega, nz, ny, nx); xi (nz, ny, nx),
complex (the physical contrast is its real part).

Parity: pinned by tests/test_oracle_invert.py (consistency with the forward
model, the sign-flip invariance of the 2D transform, single-frequency and
duplicated-frequency reductions, Parseval for the noise level).
"""
from __future__ import annotations

import numpy as np

from . import model
from .regularize import TAU, ETA, FLOOR, ROOT, tikhonov_dp, tikhonov_fixed, tsvd_dp


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
    if rule == "global":
        V, alpha, branch = _solve_global(p, f, tab, idx, wsys, dm, tau, eta, chunk)
        return V.T.reshape(p.nz, p.py, p.px), alpha, branch
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


def _solve_global(p, f, tab, idx, wsys, dm, tau, eta, chunk, bisect_steps=240):
    """One alpha for every system of the frequency (the paper's single noise
    level delta for the whole data set): the total discrepancy
    sum_m ||A_m v_m(alpha) - w_m||^2 = tau^2 N delta_m^2 (= tau^2 times the
    noise energy of all N transformed systems, Parseval), solved by bisection
    on log(alpha); alpha >= eta max_m ||A_m||_F^2, which is also the value for
    noise-free data. Systems with w_m = 0 get v_m = 0 (branch zero), and so
    do all systems when sum_m ||w_m||^2 <= tau^2 N delta_m^2 (v = 0 already
    meets the total discrepancy: the per-system rule's zero branch)."""
    N = wsys.shape[0]
    live = np.linalg.norm(wsys, axis=1) > 0
    ms_live = np.nonzero(live)[0]
    s2s, b2s, rho2s, fro = [], [], [], []
    for s0 in range(0, len(ms_live), chunk):
        ms = ms_live[s0:s0 + chunk]
        A = model.system_matrices(p, f, tab, idx, ms)
        U, s, _ = np.linalg.svd(A, full_matrices=False)
        b = np.einsum("sji,sj->si", U.conj(), wsys[ms])
        rho2s.append(np.sum(np.abs(wsys[ms] - np.einsum("sji,si->sj", U, b)) ** 2, axis=1))
        s2s.append(s * s)
        b2s.append(np.abs(b) ** 2)
        fro.append(np.sum(np.abs(A) ** 2, axis=(1, 2)))
    V = np.zeros((N, p.nz), np.complex128)
    alpha = np.full(N, np.inf)
    branch = np.zeros(N, np.int8)
    if len(ms_live) == 0:
        return V, alpha, branch
    s2, b2 = np.concatenate(s2s), np.concatenate(b2s)
    rho2 = np.concatenate(rho2s)
    amin = eta * float(np.max(np.concatenate(fro)))

    def total(a):
        t = a / (s2 + a)
        return float(np.sum(t * t * b2) + np.sum(rho2))

    target = tau * tau * N * dm * dm
    if dm > 0 and np.sum(np.abs(wsys[live]) ** 2) <= target:
        return V, alpha, branch
    if dm > 0 and total(amin) < target:
        lo, hi = np.log(amin), np.log(float(np.max(s2))) + 1.0
        while total(np.exp(hi)) < target:
            hi += 4.0
        for _ in range(bisect_steps):
            mid = 0.5 * (lo + hi)
            if total(np.exp(mid)) >= target:
                hi = mid
            else:
                lo = mid
        al, br = float(np.exp(0.5 * (lo + hi))), ROOT
    else:
        al, br = amin, FLOOR
    for s0 in range(0, len(ms_live), chunk):
        ms = ms_live[s0:s0 + chunk]
        V[ms] = tikhonov_fixed(model.system_matrices(p, f, tab, idx, ms), wsys[ms], al)
    alpha[ms_live] = al
    branch[ms_live] = br
    return V, alpha, branch


def solve_sampled(p, f, W_f, delta, ms, tau=TAU, eta=ETA):
    """Algorithm 2 item 1 for the sampled wavenumbers ms of frequency f only:
    w_m by the 2D DFT at ms, delta_m from the whole data array of the
    frequency, A_m from the sampled table; then the same regularized solve
    as solve_systems. For checking full-size grids where the full tables
    and transforms are too costly. Returns (Vhat (len(ms), nz), alpha, branch)."""
    W_f = np.asarray(W_f, np.complex128)
    wsys = model.dft2_at(W_f, ms, p.px, p.py).T                   # (S, nd)
    dm = system_noise_level(W_f, delta)
    tab, idx = model.system_table_at(p, f, ms)
    A = model.system_matrices(p, f, tab, idx, None)
    return tikhonov_dp(A, wsys, dm, tau, eta)


def solve_joint(p, Whats, delta, tau=TAU, eta=ETA, selected=None, chunk=512,
                bisect_steps=240, kernel_mode=0, damping=0.0):
    """Algorithm 2 item 1 with the equations of all frequencies solved as one
    system (Section 4, comment c: item 1 by least squares over the
    frequencies). For a wavenumber m the frequencies' systems form the
    block-diagonal system diag(A_1m, ..., A_Fm) [v_1; ...; v_F] =
    [w_1m; ...; w_Fm]; it is regularized as one system: one Tikhonov
    parameter alpha_m, chosen by the discrepancy principle for the stacked
    data,
        sum_f ||A_fm v_f - w_fm||^2 = tau^2 sum_f delta_fm^2,
    with alpha_m >= eta sum_f ||A_fm||_F^2 (the stacked matrix's floor, also
    the value for noise-free data), and v = 0 at every frequency when
    sum_f ||w_fm||^2 <= tau^2 sum_f delta_fm^2. The system being block
    diagonal, v_f is frequency f's Tikhonov solution at alpha_m.
    Whats: (n_omega, nd, py, px); selected: frequencies taking part (all by
    default; the others get v = 0). Returns (Vhat (F, nz, py, px), alpha
    (F, N), branch (F, N)), alpha and branch the same at every selected
    frequency of a wavenumber."""
    F, N = p.n_omega, p.px * p.py
    sel = [f for f in range(F) if selected is None or selected[f]]
    V = np.zeros((F, N, p.nz), np.complex128)
    alpha = np.full((F, N), np.inf)
    branch = np.zeros((F, N), np.int8)
    if not sel:
        return V.transpose(0, 2, 1).reshape(F, p.nz, p.py, p.px), alpha, branch
    tabs = [model.system_table(p, f, kernel_mode, damping) for f in sel]
    wsys = [Whats[f].reshape(p.nd, N).T for f in sel]
    dms = np.array([system_noise_level_hat(Whats[f], delta, N) for f in sel])
    target = tau * tau * float(np.sum(dms * dms))
    for s0 in range(0, N, chunk):
        ms = np.arange(s0, min(N, s0 + chunk))
        S = len(ms)
        wn2 = sum(np.sum(np.abs(w[ms]) ** 2, axis=1) for w in wsys)
        live = wn2 > 0 if target == 0 else wn2 > target
        if not np.any(live):
            continue
        ml = ms[live]
        svd, fro = [], np.zeros(len(ml))
        for k, f in enumerate(sel):
            A = model.system_matrices(p, f, tabs[k][0], tabs[k][1], ml)
            U, sv, Vh = np.linalg.svd(A, full_matrices=False)
            b = np.einsum("sji,sj->si", U.conj(), wsys[k][ml])
            rho2 = np.sum(np.abs(wsys[k][ml] - np.einsum("sji,si->sj", U, b)) ** 2, axis=1)
            svd.append((sv, b, rho2, Vh))
            fro += np.sum(np.abs(A) ** 2, axis=(1, 2))

        def phi(a):
            tot = np.zeros(len(a))
            for sv, b, rho2, _ in svd:
                t = a[:, None] / (sv * sv + a[:, None])
                tot += np.sum(t * t * np.abs(b) ** 2, axis=1) + rho2
            return tot

        amin = eta * fro
        al = amin.copy()
        br = np.full(len(ml), FLOOR, np.int8)
        need = (target > 0) & (phi(amin) < target)
        if np.any(need):
            i = np.nonzero(need)[0]
            lo = np.log(amin[i])
            smax = np.max([sv[i, 0] for sv, _, _, _ in svd], axis=0)
            hi = np.log(smax * smax) + 1.0
            for _ in range(2000):
                bad = phi(np.exp(hi)) < target
                if not np.any(bad):
                    break
                hi = np.where(bad, hi + 4.0, hi)
            for _ in range(bisect_steps):
                mid = 0.5 * (lo + hi)
                up = phi(np.exp(mid)) >= target
                hi = np.where(up, mid, hi)
                lo = np.where(up, lo, mid)
            al[i] = np.exp(0.5 * (lo + hi))
            br[i] = ROOT
        for k, f in enumerate(sel):
            sv, b, _, Vh = svd[k]
            coef = sv * b / (sv * sv + al[:, None])
            V[f, ml] = np.einsum("sij,si->sj", Vh.conj(), coef)
            alpha[f, ml] = al
            branch[f, ml] = br
    return V.transpose(0, 2, 1).reshape(F, p.nz, p.py, p.px), alpha, branch


def system_noise_level_hat(What_f, delta, N):
    """The same delta_m computed from the transformed data via Parseval:
    ||W||^2 = ||W^||^2 / N."""
    return float(delta) * float(np.linalg.norm(What_f)) / np.sqrt(N)


def invert(p, W, u0, delta, tau=TAU, eta=ETA, combine="lsq", rule="tikhonov",
           stages=False, kernel_mode=0, damping=0.0, weights=None):
    """W -> xi. With stages=True also returns a dict of per-frequency
    intermediates (What, Vhat, v, u, alpha, branch). kernel_mode / damping
    select the table of A (model.system_table); weights (n_omega,) the
    weighted least squares of item 3 (combine "lsq" only)."""
    W = np.asarray(W, np.complex128)
    u0 = np.asarray(u0, np.complex128)
    nf = p.n_omega
    wt = np.ones(nf) if weights is None or combine != "lsq" else np.asarray(weights, np.float64)
    num = np.zeros((p.nz, p.ny, p.nx), np.complex128)
    den = np.zeros((p.nz, p.ny, p.nx), np.float64)
    per_f = []
    keep = {k: [] for k in ("What", "Vhat", "v", "u", "alpha", "branch")}
    joint = None
    if rule == "joint":
        # item 1 for all frequencies at once (one system per wavenumber)
        joint = solve_joint(p, np.fft.fft2(W), delta, tau, eta, selected=wt > 0,
                            kernel_mode=kernel_mode, damping=damping)
    for f in range(nf):
        What = np.fft.fft2(W[f])                                  # item 1 input
        if joint is not None:
            Vhat, alpha, branch = joint[0][f], joint[1][f], joint[2][f]
        elif wt[f] == 0:
            # not selected: no solve, v = 0
            N = p.px * p.py
            Vhat = np.zeros((p.nz, p.py, p.px), np.complex128)
            alpha, branch = np.full(N, np.inf), np.zeros(N, np.int8)
        else:
            Vhat, alpha, branch = solve_systems(p, f, What, delta, tau, eta, rule,
                                                kernel_mode=kernel_mode, damping=damping)
        v = model.crop(p, np.fft.ifft2(Vhat))                      # item 2
        u = u0[f] + model.volume_potential(p, f, v)
        num += wt[f] * np.conj(u) * v                              # item 3
        den += wt[f] * np.abs(u) ** 2
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
