"""Regularized solution of the first-kind systems A_m v_m = w_m (oracle).

Algorithm 2, item 1 asks for a regularizing algorithm that yields the normal
(minimum-norm) solution (Section 4, comment b; Section 5.2 names Tikhonov
regularization and TSVD). The paper does not say how the parameter is chosen;
the reading taken here:

* Tikhonov: v(alpha) = (A^H A + alpha I)^{-1} A^H w.
* Discrepancy principle per system: alpha solves
  ||A v(alpha) - w||^2 = tau^2 delta_m^2, with delta_m = delta * ||W^delta||
  (the l2 norm of frequency f's whole data array; by Parseval this is the
  expected noise norm of every system in unnormalized DFT units) and
  tau = 1.5.
* alpha is bounded below by alpha_min = eta * ||A||_F^2 (eta = 1e-10): noise
  free data (delta = 0) use alpha_min, and so does a system whose residual
  already exceeds tau*delta_m at alpha_min. A system with
  ||w|| <= tau*delta_m gets v = 0 (alpha = infinity).
* TSVD (the paper's best performer) keeps the k leading singular triplets,
  k the smallest count whose residual meets tau*delta_m.

The oracle computes everything from LAPACK's SVD (numpy.linalg.svd) and
finds alpha by bisection on log(alpha) of the monotone function
phi(alpha) = sum_i (alpha/(s_i^2+alpha))^2 |b_i|^2 + rho_perp^2, b = U^H w.

Branch codes: 0 = zero (alpha = inf), 1 = floor (alpha = alpha_min),
2 = discrepancy root.

Parity: pinned by tests/test_oracle_regularize.py (augmented least squares,
closed-form rank-one systems, unitary invariance, direct residuals).
"""
from __future__ import annotations

import numpy as np

TAU = 1.5
ETA = 1e-10

ZERO, FLOOR, ROOT = 0, 1, 2


def _phi(alpha, s2, b2, rho2):
    """phi(alpha) for a batch: alpha (S,), s2 and b2 (S, r), rho2 (S,)."""
    t = alpha[:, None] / (s2 + alpha[:, None])
    return np.sum(t * t * b2, axis=1) + rho2


def tikhonov_dp(A, w, delta_m, tau=TAU, eta=ETA, bisect_steps=240):
    """Solve a batch of systems. A: (S, nd, nz), w: (S, nd), delta_m scalar
    (or (S,)). Returns (v (S, nz), alpha (S,), branch (S,))."""
    A = np.asarray(A, np.complex128)
    w = np.asarray(w, np.complex128)
    S = A.shape[0]
    nz = A.shape[2]
    dm = np.broadcast_to(np.asarray(delta_m, np.float64), (S,))
    v = np.zeros((S, nz), np.complex128)
    alpha = np.full(S, np.inf)
    branch = np.full(S, ZERO, np.int8)

    wn = np.linalg.norm(w, axis=1)
    noisy = dm > 0
    live = ~(noisy & (wn <= tau * dm)) & (wn > 0)
    live &= np.abs(A).reshape(S, -1).max(axis=1) > 0
    if not np.any(live):
        return v, alpha, branch
    Al, wl, dl = A[live], w[live], dm[live]
    U, s, Vh = np.linalg.svd(Al, full_matrices=False)
    b = np.einsum("sji,sj->si", U.conj(), wl)
    rho2 = np.sum(np.abs(wl - np.einsum("sji,si->sj", U, b)) ** 2, axis=1)
    s2 = s * s
    b2 = np.abs(b) ** 2
    amin = eta * np.sum(np.abs(Al) ** 2, axis=(1, 2))
    target = (tau * dl) ** 2

    al = amin.copy()
    br = np.full(len(al), FLOOR, np.int8)
    need = (dl > 0) & (_phi(amin, s2, b2, rho2) < target)
    if np.any(need):
        i = np.nonzero(need)[0]
        lo = np.log(amin[i])
        hi = np.log(s2[i, 0]) + 1.0
        # grow the upper end until phi exceeds the target (phi(inf) = ||w||^2)
        for _ in range(2000):
            bad = _phi(np.exp(hi), s2[i], b2[i], rho2[i]) < target[i]
            if not np.any(bad):
                break
            hi = np.where(bad, hi + 4.0, hi)
        for _ in range(bisect_steps):
            mid = 0.5 * (lo + hi)
            up = _phi(np.exp(mid), s2[i], b2[i], rho2[i]) >= target[i]
            hi = np.where(up, mid, hi)
            lo = np.where(up, lo, mid)
        al[i] = np.exp(0.5 * (lo + hi))
        br[i] = ROOT
    coef = s * b / (s2 + al[:, None])
    v[live] = np.einsum("sij,si->sj", Vh.conj(), coef)
    alpha[live] = al
    branch[live] = br
    return v, alpha, branch


def tikhonov_fixed(A, w, alpha):
    """Tikhonov solution at a given alpha (batch), from the SVD."""
    U, s, Vh = np.linalg.svd(np.asarray(A, np.complex128), full_matrices=False)
    b = np.einsum("sji,sj->si", U.conj(), w)
    alpha = np.broadcast_to(np.asarray(alpha, np.float64), (A.shape[0],))
    coef = s * b / (s * s + alpha[:, None])
    return np.einsum("sij,si->sj", Vh.conj(), coef)


def tsvd_dp(A, w, delta_m, tau=TAU, eta=ETA):
    """Truncated SVD with the truncation index chosen by the discrepancy
    principle: keep the fewest leading triplets (with s_i^2 > eta ||A||_F^2) whose
    residual is <= tau*delta_m. Returns (v, k)."""
    A = np.asarray(A, np.complex128)
    S, nd, nz = A.shape
    dm = np.broadcast_to(np.asarray(delta_m, np.float64), (S,))
    U, s, Vh = np.linalg.svd(A, full_matrices=False)
    b = np.einsum("sji,sj->si", U.conj(), w)
    rho2 = np.sum(np.abs(w - np.einsum("sji,si->sj", U, b)) ** 2, axis=1)
    b2 = np.abs(b) ** 2
    r = s.shape[1]
    # residual after keeping k triplets: rho2 + sum_{i >= k} |b_i|^2
    tail = np.concatenate([np.cumsum(b2[:, ::-1], axis=1)[:, ::-1],
                           np.zeros((S, 1))], axis=1) + rho2[:, None]
    allowed = (s * s > eta * np.sum(np.abs(A) ** 2, axis=(1, 2))[:, None])
    kmax = allowed.sum(axis=1)
    ok = tail <= (tau * dm)[:, None] ** 2
    k = np.where(ok.any(axis=1), np.argmax(ok, axis=1), r)
    k = np.minimum(k, kmax)
    keep = np.arange(r)[None, :] < k[:, None]
    coef = np.where(keep, b / np.where(s > 0, s, 1.0), 0.0)
    v = np.einsum("sij,si->sj", Vh.conj(), coef)
    return v, k
