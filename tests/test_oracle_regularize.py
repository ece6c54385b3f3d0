"""Pins of the oracle's regularized first-kind solver (no GPU)."""
import numpy as np
import pytest

from oracle import regularize as rg
from paper_1911_10487_amd import synth


def _graded(S, nd, nz, decay, seed):
    """Batch of complex matrices with singular values decay**i."""
    rng = np.random.default_rng(seed)
    r = min(nd, nz)
    out = np.empty((S, nd, nz), complex)
    for s in range(S):
        U, _ = np.linalg.qr(rng.standard_normal((nd, nd)) + 1j * rng.standard_normal((nd, nd)))
        V, _ = np.linalg.qr(rng.standard_normal((nz, nz)) + 1j * rng.standard_normal((nz, nz)))
        sv = decay ** np.arange(r)
        out[s] = (U[:, :r] * sv) @ V[:, :r].conj().T
    return out


@pytest.mark.parametrize("nd,nz", [(6, 6), (8, 5), (4, 7)])
def test_tikhonov_equals_augmented_least_squares(nd, nz):
    A = _graded(5, nd, nz, 0.3, (1, nd, nz))
    w = synth.random_field((5, nd), (2, nd, nz))
    for alpha in (1e-6, 1e-2, 3.0):
        v = rg.tikhonov_fixed(A, w, alpha)
        for s in range(5):
            M = np.vstack([A[s], np.sqrt(alpha) * np.eye(nz)])
            rhs = np.concatenate([w[s], np.zeros(nz)])
            ref = np.linalg.lstsq(M, rhs, rcond=None)[0]
            assert np.linalg.norm(v[s] - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("nd,nz", [(7, 7), (9, 4)])
def test_rank_one_system_has_the_closed_form_root(nd, nz):
    # A = s a b^T: v(alpha) = conj(s) (a^H w) conj(b) / (sigma1^2 + alpha), and the
    # discrepancy root is alpha = sigma1^2 r / (1 - r) with
    # r^2 = (T - ||P_perp w||^2) / (|a^H w|^2 / ||a||^2).
    rng = np.random.default_rng(7)
    s = 0.7 - 1.3j
    a = rng.standard_normal(nd) + 1j * rng.standard_normal(nd)
    b = rng.standard_normal(nz) + 1j * rng.standard_normal(nz)
    A = (s * np.outer(a, b))[None]
    w = (3.0 * a + 0.05 * (rng.standard_normal(nd) + 1j * rng.standard_normal(nd)))[None]
    sig1 = abs(s) * np.linalg.norm(a) * np.linalg.norm(b)
    aw = np.vdot(a, w[0])
    perp2 = np.linalg.norm(w[0]) ** 2 - abs(aw) ** 2 / np.linalg.norm(a) ** 2
    tau = rg.TAU
    dm = 0.3 * np.linalg.norm(w[0]) / tau  # tau * delta_m = 0.3 ||w||
    T = (tau * dm) ** 2
    r = np.sqrt((T - perp2) / (abs(aw) ** 2 / np.linalg.norm(a) ** 2))
    alpha_ref = sig1 ** 2 * r / (1 - r)
    v, alpha, br = rg.tikhonov_dp(A, w, dm)
    assert br[0] == rg.ROOT
    assert abs(alpha[0] - alpha_ref) <= 1e-12 * alpha_ref
    v_ref = np.conj(s) * aw * np.conj(b) / (sig1 ** 2 + alpha_ref)
    assert np.linalg.norm(v[0] - v_ref) <= 1e-12 * np.linalg.norm(v_ref)


def test_discrepancy_root_meets_the_residual_exactly():
    A = _graded(20, 10, 10, 0.2, (3,))
    v0 = synth.random_field((20, 10), (4,))
    w = np.einsum("sjl,sl->sj", A, v0) + 1e-3 * synth.random_field((20, 10), (5,))
    dm = 2e-3
    v, alpha, br = rg.tikhonov_dp(A, w, dm)
    res = np.linalg.norm(np.einsum("sjl,sl->sj", A, v) - w, axis=1)
    root = br == rg.ROOT
    assert root.sum() > 10
    assert np.all(abs(res[root] - rg.TAU * dm) <= 1e-12 * rg.TAU * dm)
    # v is the Tikhonov solution at the returned alpha
    vf = rg.tikhonov_fixed(A[root], w[root], alpha[root])
    assert np.linalg.norm(vf - v[root]) <= 1e-12 * np.linalg.norm(v[root])


def test_branches():
    A = _graded(3, 6, 6, 0.3, (8,))
    w = synth.random_field((3, 6), (9,))
    wn = np.linalg.norm(w, axis=1)
    # zero branch: ||w|| <= tau delta_m
    v, alpha, br = rg.tikhonov_dp(A, w, wn.max() / rg.TAU * 1.0001)
    assert np.all(br == rg.ZERO) and np.all(v == 0) and np.all(np.isinf(alpha))
    # noise-free data: alpha = eta ||A||_F^2
    v, alpha, br = rg.tikhonov_dp(A, w, 0.0)
    fro2 = np.sum(abs(A) ** 2, axis=(1, 2))
    assert np.all(br == rg.FLOOR)
    assert np.allclose(alpha, rg.ETA * fro2, rtol=1e-15, atol=0)
    # a residual above tau delta_m already at the floor: tiny noise level on a
    # system whose data leave the range of A (nd > nz)
    A2 = _graded(2, 8, 3, 0.5, (10,))
    w2 = synth.random_field((2, 8), (11,))
    v, alpha, br = rg.tikhonov_dp(A2, w2, 1e-8)
    assert np.all(br == rg.FLOOR)


def test_unitary_invariance():
    # v(QA, Qw) = v(A, w) and v(AZ, w) = Z^H v(A, w) for unitary Q, Z
    rng = np.random.default_rng(12)
    A = _graded(4, 7, 7, 0.25, (13,))
    w = np.einsum("sjl,sl->sj", A, synth.random_field((4, 7), (14,))) \
        + 1e-2 * synth.random_field((4, 7), (15,))
    dm = 5e-3
    v, alpha, br = rg.tikhonov_dp(A, w, dm)
    Q, _ = np.linalg.qr(rng.standard_normal((7, 7)) + 1j * rng.standard_normal((7, 7)))
    Z, _ = np.linalg.qr(rng.standard_normal((7, 7)) + 1j * rng.standard_normal((7, 7)))
    vq, aq, _ = rg.tikhonov_dp(Q @ A, w @ Q.T, dm)
    assert np.linalg.norm(vq - v) <= 1e-11 * np.linalg.norm(v)
    vz, az, _ = rg.tikhonov_dp(A @ Z, w, dm)
    assert np.linalg.norm(vz - v @ Z.conj()) <= 1e-11 * np.linalg.norm(v)
    assert np.allclose(aq, alpha, rtol=1e-11) and np.allclose(az, alpha, rtol=1e-11)


def test_noise_free_consistent_data_are_recovered():
    # w = A v0 with v0 in the range of A^H: as alpha -> 0 the Tikhonov solution
    # tends to v0 = lstsq(A, w) (the normal solution)
    A = _graded(3, 6, 9, 0.6, (16,))
    y = synth.random_field((3, 6), (17,))
    v0 = np.einsum("sjl,sj->sl", A.conj(), y)
    w = np.einsum("sjl,sl->sj", A, v0)
    v, alpha, br = rg.tikhonov_dp(A, w, 0.0, eta=1e-28)
    for s in range(3):
        ref = np.linalg.lstsq(A[s], w[s], rcond=None)[0]
        assert np.linalg.norm(ref - v0[s]) <= 1e-12 * np.linalg.norm(v0[s])
        assert np.linalg.norm(v[s] - v0[s]) <= 1e-11 * np.linalg.norm(v0[s])
    # and at the default floor the bias is of order eta * ||A||_F^2 / sigma_min^2
    v, alpha, br = rg.tikhonov_dp(A, w, 0.0)
    smin2 = 0.6 ** 10
    fro2 = np.sum(0.6 ** (2 * np.arange(6)))
    bound = 3 * rg.ETA * fro2 / smin2
    assert np.linalg.norm(v - v0) <= bound * np.linalg.norm(v0)


def test_tsvd_keeps_the_fewest_triplets_meeting_the_discrepancy():
    A = _graded(10, 8, 8, 0.3, (18,))
    w = np.einsum("sjl,sl->sj", A, synth.random_field((10, 8), (19,))) \
        + 1e-3 * synth.random_field((10, 8), (20,))
    dm = 1e-3
    v, k = rg.tsvd_dp(A, w, dm)
    U, s, Vh = np.linalg.svd(A)
    for i in range(10):
        def resid(kk):
            c = U[i, :, :kk].conj().T @ w[i] / s[i, :kk]
            return np.linalg.norm(A[i] @ (Vh[i, :kk].conj().T @ c) - w[i])
        assert resid(k[i]) <= rg.TAU * dm * (1 + 1e-12)
        if k[i] > 0:
            assert resid(k[i] - 1) > rg.TAU * dm


def test_tsvd_without_noise_is_the_floored_pseudo_inverse():
    # delta = 0: no residual is within a zero threshold, so every triplet above
    # the floor s^2 > eta ||A||_F^2 is kept: the pseudo-inverse whose cut-off
    # relative to s_max is sqrt(eta) ||A||_F / s_max (numpy's pinv)
    A = _graded(6, 9, 9, 0.05, (21,))
    w = synth.random_field((6, 9), (22,))
    v, k = rg.tsvd_dp(A, w, 0.0)
    for i in range(6):
        s = np.linalg.svd(A[i], compute_uv=False)
        fro = np.linalg.norm(A[i])
        floor = np.sqrt(rg.ETA) * fro
        # the graded spectrum keeps no singular value near the cut-off
        assert np.min(np.abs(s - floor)) > 0.1 * floor
        assert k[i] == np.count_nonzero(s > floor) < 9
        ref = np.linalg.pinv(A[i], rcond=floor / s[0]) @ w[i]
        assert np.linalg.norm(v[i] - ref) <= 1e-10 * np.linalg.norm(ref)
