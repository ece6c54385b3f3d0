"""Pins of the oracle's Algorithm 2 pipeline (no GPU)."""
import numpy as np
import pytest

from oracle import forward, invert, model
from paper_1911_10487_amd import synth


@pytest.fixture(scope="module")
def small():
    p = synth.workload("small")[0]
    xi = synth.contrast(p)
    u0 = synth.incident_field(p)
    W, U, V, info = forward.synthesize(p, xi, u0)
    return p, xi, u0, W, U, V


def test_items_2_and_3_return_the_truth_from_the_true_current(small):
    # Fed the exact v = xi * u of the forward solve, eq. (9) rebuilds u and
    # item 3 returns xi (BiCGSTAB tolerance 1e-12).
    p, xi, u0, W, U, V = small
    u = u0[0] + model.volume_potential(p, 0, V[0])
    assert np.linalg.norm(u - U[0]) <= 1e-10 * np.linalg.norm(U[0])
    x = invert.combine_lsq(u[None], V[0][None])
    assert np.linalg.norm(x - xi) <= 1e-10 * np.linalg.norm(xi)


def test_item_1_sees_the_data_operator(small):
    # the transformed data of every wavenumber is A_m applied to V^_m
    p, xi, u0, W, U, V = small
    What = np.fft.fft2(W[0]).reshape(p.nd, -1)
    Vh = np.fft.fft2(model.embed(p, V[0])).reshape(p.nz, -1)
    tab, idx = model.system_table(p, 0)
    ms = np.arange(0, p.px * p.py, 37)
    A = model.system_matrices(p, 0, tab, idx, ms)
    lhs = np.einsum("mjl,lm->jm", A, Vh[:, ms])
    assert np.linalg.norm(lhs - What[:, ms]) <= 1e-12 * np.linalg.norm(What[:, ms])


def test_flipping_the_transform_sign_leaves_xi_unchanged(small, monkeypatch):
    # Section 2 prints exp(+i ...); the oracle and the kernels use exp(-i ...). G is radial,
    # so the two conventions give the same xi.
    p, xi, u0, W, U, V = small
    Wd = synth.add_noise(p, W, 0.01)
    ref = invert.invert(p, Wd, u0, 0.01)
    f2, if2 = np.fft.fft2, np.fft.ifft2
    monkeypatch.setattr(np.fft, "fft2", lambda x, *a, **k: np.conj(f2(np.conj(x), *a, **k)))
    monkeypatch.setattr(np.fft, "ifft2", lambda x, *a, **k: np.conj(if2(np.conj(x), *a, **k)))
    flipped = invert.invert(p, Wd, u0, 0.01)
    assert np.linalg.norm(flipped - ref) <= 1e-12 * np.linalg.norm(ref)


def test_mirror_symmetry(small):
    # Mirroring x about X's centre (data, incident field) mirrors xi.
    p, xi, u0, W, U, V = small
    Wd = synth.add_noise(p, W, 0.01)
    ref = invert.invert(p, Wd, u0, 0.01)
    ox, _ = model.window_offset(p)
    perm = (2 * ox + p.nx - 1 - np.arange(p.px)) % p.px
    Wm = Wd[..., perm]
    um = u0[..., ::-1]
    got = invert.invert(p, Wm, um, 0.01)
    assert np.linalg.norm(got - ref[..., ::-1]) <= 1e-11 * np.linalg.norm(ref)


def test_one_frequency_least_squares_is_the_quotient():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((1, 4, 5)) + 1j * rng.standard_normal((1, 4, 5))
    v = rng.standard_normal((1, 4, 5)) + 1j * rng.standard_normal((1, 4, 5))
    assert np.allclose(invert.combine_lsq(u, v), v[0] / u[0], rtol=1e-15, atol=0)
    u[0, 0, 0] = 0
    assert invert.combine_lsq(u, v)[0, 0] == 0


def test_duplicated_frequency_gives_the_same_xi(small):
    p, xi, u0, W, U, V = small
    Wd = synth.add_noise(p, W, 0.01)
    ref = invert.invert(p, Wd, u0, 0.01)
    p2 = synth.make_problem("dup", p.nx, p.ny, p.nz, [p.omegas[0]] * 2, 3, (0, 0))
    got = invert.invert(p2, np.concatenate([Wd, Wd]), np.concatenate([u0, u0]), 0.01)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)


def test_noise_level_by_parseval(small):
    p, xi, u0, W, U, V = small
    Wd = synth.add_noise(p, W, 0.01)
    What = np.fft.fft2(Wd[0])
    a = invert.system_noise_level(Wd[0], 0.01)
    b = invert.system_noise_level_hat(What, 0.01, p.px * p.py)
    assert abs(a - b) <= 1e-14 * a


def test_reconstruction_is_meaningful(small):
    # Not a parity gate (the problem is severely ill-posed, Section 6): the
    # reconstruction still carries the blobs.
    p, xi, u0, W, U, V = small
    x0, st = invert.invert(p, W, u0, 0.0, stages=True)
    assert np.all(st["branch"] == 1)
    assert np.linalg.norm(x0.real - xi) < 0.5 * np.linalg.norm(xi)
    x1, st = invert.invert(p, synth.add_noise(p, W, 0.01), u0, 0.01, stages=True)
    assert np.linalg.norm(x1.real - xi) < 0.8 * np.linalg.norm(xi)
    assert (st["branch"] == 0).mean() > 0.5


@pytest.mark.parametrize("eta", [1e-10, 1e-8])
def test_noise_free_inversion_is_fft_rounding_limited(small, eta, monkeypatch):
    # delta = 0 solves every system at alpha = eta ||A||_F^2 (condition number
    # up to eta^-1/2). Swapping numpy's FFT for scipy's (rounding differences
    # only) moves v^ far above u but within 1e3 * u * eta^-1/2: the gate that
    # the GPU parity tests use for noise-free data.
    import scipy.fft as sf
    p, xi, u0, W, U, V = small
    x1, s1 = invert.invert(p, W, u0, 0.0, eta=eta, stages=True)
    monkeypatch.setattr(np.fft, "fft2", lambda a, *k, **kw: sf.fft2(a, *k, **kw, workers=1))
    monkeypatch.setattr(np.fft, "ifft2", lambda a, *k, **kw: sf.ifft2(a, *k, **kw, workers=1))
    x2, s2 = invert.invert(p, W, u0, 0.0, eta=eta, stages=True)
    d = np.linalg.norm(s2["Vhat"] - s1["Vhat"]) / np.linalg.norm(s1["Vhat"])
    assert 1e-12 < d < 1e3 * 2.0 ** -53 * eta ** -0.5
    # with noise the zero branch removes the tiny systems: FP64-level agreement
    Wd = synth.add_noise(p, W, 0.01)
    monkeypatch.undo()
    y1 = invert.invert(p, Wd, u0, 0.01)
    monkeypatch.setattr(np.fft, "fft2", lambda a, *k, **kw: sf.fft2(a, *k, **kw, workers=1))
    monkeypatch.setattr(np.fft, "ifft2", lambda a, *k, **kw: sf.ifft2(a, *k, **kw, workers=1))
    y2 = invert.invert(p, Wd, u0, 0.01)
    assert np.linalg.norm(y2 - y1) / np.linalg.norm(y1) < 1e-12


# ------------------------------------------------ one alpha per frequency

def test_global_rule_with_one_nonzero_system_is_the_per_system_rule():
    # data with a single nonzero wavenumber: the only live system sees the
    # same target under both rules once tau_global = tau / sqrt(N)
    p = synth.tiny_problem(nx=6, ny=5, nz=4, px=12, py=10)
    rng = np.random.default_rng([8, 1])
    What = np.zeros((1, p.nd, p.py, p.px), np.complex128)
    What[0, :, 3, 7] = rng.standard_normal(p.nd) + 1j * rng.standard_normal(p.nd)
    W = np.fft.ifft2(What)
    N = p.px * p.py
    tab, idx = model.system_table(p, 0)
    Vs, a_s, b_s = invert.solve_systems(p, 0, What[0], 0.3, tau=1.5, tab=tab, idx=idx)
    Vg, a_g, b_g = invert.solve_systems(p, 0, What[0], 0.3, tau=1.5 / np.sqrt(N), rule="global",
                                        tab=tab, idx=idx)
    m0 = 3 * p.px + 7
    assert b_s[m0] == 2 and b_g[m0] == 2
    assert np.count_nonzero(b_g) == 1 and np.count_nonzero(b_s) == 1
    assert abs(a_g[m0] - a_s[m0]) <= 1e-13 * a_s[m0]
    assert np.linalg.norm(Vg - Vs) <= 1e-13 * np.linalg.norm(Vs)
    assert np.isfinite(W).all()


def test_global_rule_meets_the_total_discrepancy(small):
    # sum_m ||A_m v_m - w_m||^2 at the returned alpha, from the matrices
    # themselves (not the SVD), equals tau^2 N delta_m^2; more noise gives a
    # larger alpha
    p, xi, u0, W, U, V = small
    Wd = synth.add_noise(p, W, 0.02)
    What = np.fft.fft2(Wd[0])
    N = p.px * p.py
    tab, idx = model.system_table(p, 0)
    Vg, a, br = invert.solve_systems(p, 0, What, 0.02, tau=1.0, rule="global", tab=tab, idx=idx)
    live = br > 0
    assert live.sum() == N and np.all(br[live] == 2) and np.ptp(a[live]) == 0
    A = model.system_matrices(p, 0, tab, idx, np.arange(N))
    r = np.einsum("sjl,sl->sj", A, Vg.reshape(p.nz, N).T) - What.reshape(p.nd, N).T
    dm = invert.system_noise_level_hat(What, 0.02, N)
    assert abs(np.sum(np.abs(r) ** 2) / (N * dm * dm) - 1.0) <= 1e-10
    _, a2, _ = invert.solve_systems(p, 0, What, 0.04, tau=1.0, rule="global", tab=tab, idx=idx)
    assert a2[0] > a[0]


def test_global_rule_data_inside_the_noise_level_give_zero(small):
    # tau delta >= 1: v = 0 meets the total discrepancy (sum_m ||w_m||^2 =
    # N ||W||^2 by Parseval); just below, a root with a large alpha
    p, xi, u0, W, U, V = small
    What = np.fft.fft2(W[0])
    tab, idx = model.system_table(p, 0)
    Vg, a, br = invert.solve_systems(p, 0, What, 1.0, tau=1.0 + 1e-9, rule="global", tab=tab,
                                     idx=idx)
    assert not Vg.any() and np.all(br == 0) and np.all(np.isinf(a))
    Vg, a, br = invert.solve_systems(p, 0, What, 0.9, tau=1.0, rule="global", tab=tab, idx=idx)
    assert np.all(br == 2) and Vg.any()


# ------------------------------------------------ weighted frequencies

@pytest.fixture(scope="module")
def two_freq():
    p = synth.make_problem("w2", 12, 10, 8, [2 * np.pi, 1.5 * 2 * np.pi], 2, (7, 3), (0.02,),
                           px=24, py=20)
    xi = synth.contrast(p)
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=True)
    return p, synth.add_noise(p, W, 0.02), u0


def test_selecting_one_frequency_is_its_quotient(two_freq):
    # weights (1, 0): the least squares reduces to v_0 / u_0, the first
    # frequency's per-frequency result, and the second is not solved
    p, W, u0 = two_freq
    per = invert.invert(p, W, u0, 0.02, combine="per_frequency")
    x, st = invert.invert(p, W, u0, 0.02, weights=[1.0, 0.0], stages=True)
    assert np.linalg.norm(x - per[0]) <= 1e-14 * np.linalg.norm(per[0])
    assert not st["Vhat"][1].any() and np.all(st["branch"][1] == 0)
    x2 = invert.invert(p, W, u0, 0.02, weights=[0.0, 3.0])
    assert np.linalg.norm(x2 - per[1]) <= 1e-14 * np.linalg.norm(per[1])


def test_weights_are_scale_free(two_freq):
    p, W, u0 = two_freq
    ref = invert.invert(p, W, u0, 0.02)
    same = invert.invert(p, W, u0, 0.02, weights=[2.5, 2.5])
    assert np.linalg.norm(same - ref) <= 1e-14 * np.linalg.norm(ref)
    a = invert.invert(p, W, u0, 0.02, weights=[0.3, 1.7])
    b = invert.invert(p, W, u0, 0.02, weights=[0.6, 3.4])
    assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(a)
    assert np.linalg.norm(a - ref) > 1e-6 * np.linalg.norm(ref)


def test_weighted_derivatives_satisfy_the_dot_product_identity(two_freq):
    from oracle import adjoint
    p, W, u0 = two_freq
    g = synth.random_field((p.nz, p.ny, p.nx), (61,))
    dW = synth.random_field(W.shape, (62,))
    dW *= np.linalg.norm(W) / np.linalg.norm(dW)
    wt = [0.3, 1.7]
    gW, _ = adjoint.vjp(p, W, u0, 0.02, g, weights=wt)
    jv = adjoint.jvp(p, W, u0, 0.02, dW, weights=wt)
    lhs = np.real(np.vdot(g, jv))
    rhs = np.real(np.vdot(gW, dW))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    # and the tangent is the derivative: central differences on the oracle
    h = 1e-6
    xp = invert.invert(p, W + h * dW, u0, 0.02, weights=wt)
    xm = invert.invert(p, W - h * dW, u0, 0.02, weights=wt)
    fd = (xp - xm) / (2 * h)
    assert np.linalg.norm(fd - jv) <= 1e-5 * np.linalg.norm(jv)


def test_thin_layer_solutions_are_minimum_norm_and_meet_the_discrepancy():
    # nd = 2 planes, nz = 8: wide systems. Every solved v^_m lies in the row
    # space of A_m (minimum norm) and a root system's residual is tau delta_m
    p = synth.thin_problem("thin", 6, 5, 8, [2 * np.pi], 2, (4, 4), gap=0.3, spacing=0.01,
                           px=12, py=10)
    xi = synth.contrast(p)
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=True)
    Wd = synth.add_noise(p, W, 0.01)
    x, st = invert.invert(p, Wd, u0, 0.01, stages=True)
    assert np.isfinite(x).all()
    N = p.px * p.py
    tab, idx = model.system_table(p, 0)
    A = model.system_matrices(p, 0, tab, idx, np.arange(N))
    V = st["Vhat"][0].reshape(p.nz, N).T
    w = st["What"][0].reshape(p.nd, N).T
    dm = invert.system_noise_level_hat(st["What"][0], 0.01, N)
    br = st["branch"][0]
    assert (br == 2).any()
    for m in np.nonzero(br)[0]:
        # component of v in null(A): v - A^H (A A^H)^-1 A v
        Am = A[m]
        proj = Am.conj().T @ np.linalg.solve(Am @ Am.conj().T, Am @ V[m])
        assert np.linalg.norm(V[m] - proj) <= 1e-8 * np.linalg.norm(V[m])
        if br[m] == 2:
            r = np.linalg.norm(Am @ V[m] - w[m])
            assert abs(r / (1.5 * dm) - 1.0) <= 1e-9


def test_sampled_solve_matches_the_full_solve():
    # the sampled route (DFT and table at a few wavenumbers) reproduces the
    # full inversion's per-system outputs at those wavenumbers
    from oracle import invert as inv
    p = synth.make_problem("samp", 12, 10, 8, [2 * np.pi, 3 * np.pi], 2, (71, 0), (0.02,),
                           px=24, py=20)
    xi = synth.contrast(p)
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=True)
    Wd = synth.add_noise(p, W, 0.02)
    _, st = inv.invert(p, Wd, u0, 0.02, stages=True)
    ms = np.array([0, 1, 13, 100, 241, 479])
    for f in range(p.n_omega):
        V, al, br = inv.solve_sampled(p, f, Wd[f], 0.02, ms)
        Vref = st["Vhat"][f].reshape(p.nz, -1)[:, ms].T
        assert np.array_equal(br, st["branch"][f][ms])
        assert np.linalg.norm(V - Vref) <= 1e-12 * np.linalg.norm(Vref)
        fin = np.isfinite(al)
        assert np.allclose(al[fin], st["alpha"][f][ms][fin], rtol=1e-12, atol=0)


def _joint_case(omegas=(2 * np.pi, 3 * np.pi), seed=(73, 0)):
    p = synth.make_problem("joint", 12, 10, 8, list(omegas), 2, seed, (0.02,), px=24, py=20)
    xi = synth.contrast(p)
    u0 = synth.incident_field(p)
    W, _, _, _ = forward.synthesize(p, xi, u0, born=True)
    return p, synth.add_noise(p, W, 0.02), u0


def test_joint_rule_reduces_to_the_per_system_rule_for_one_frequency():
    p, Wd, u0 = _joint_case(omegas=(2 * np.pi,))
    Wh = np.fft.fft2(Wd)
    Vj, aj, bj = invert.solve_joint(p, Wh, 0.02)
    Vs, as_, bs = invert.solve_systems(p, 0, Wh[0], 0.02)
    assert np.array_equal(bj[0], bs)
    fin = np.isfinite(as_)
    assert np.allclose(aj[0][fin], as_[fin], rtol=1e-12, atol=0)
    assert np.linalg.norm(Vj[0] - Vs) <= 1e-12 * np.linalg.norm(Vs)


def test_joint_rule_on_a_duplicated_frequency_is_the_per_system_rule():
    # two identical frequencies with identical data: the stacked discrepancy
    # and its target both double, so alpha_m is the single system's
    p, Wd, u0 = _joint_case(omegas=(2 * np.pi, 2 * np.pi))
    Wd[1] = Wd[0]
    Wh = np.fft.fft2(Wd)
    Vj, aj, bj = invert.solve_joint(p, Wh, 0.02)
    Vs, as_, bs = invert.solve_systems(p, 0, Wh[0], 0.02)
    for f in range(2):
        assert np.array_equal(bj[f], bs)
        assert np.linalg.norm(Vj[f] - Vs) <= 1e-11 * np.linalg.norm(Vs)


def test_joint_rule_meets_the_stacked_discrepancy_and_is_tikhonov():
    from oracle import model
    p, Wd, u0 = _joint_case()
    Wh = np.fft.fft2(Wd)
    N = p.px * p.py
    Vj, aj, bj = invert.solve_joint(p, Wh, 0.02)
    roots = np.flatnonzero(bj[0] == 2)
    assert len(roots) > 5 and np.array_equal(bj[0], bj[1])
    dms = [invert.system_noise_level_hat(Wh[f], 0.02, N) for f in range(2)]
    target = 1.5 ** 2 * sum(d * d for d in dms)
    tabs = [model.system_table(p, f) for f in range(2)]
    for m in roots[:: max(1, len(roots) // 8)]:
        res, al = 0.0, aj[0][m]
        for f in range(2):
            A = model.system_matrices(p, f, tabs[f][0], tabs[f][1], [m])[0]
            w = Wh[f].reshape(p.nd, N)[:, m]
            v = Vj[f].reshape(p.nz, N)[:, m]
            res += np.linalg.norm(A @ v - w) ** 2
            # Tikhonov at the joint alpha: augmented least squares
            aug = np.vstack([A, np.sqrt(al) * np.eye(p.nz)])
            ref = np.linalg.lstsq(aug, np.concatenate([w, np.zeros(p.nz)]), rcond=None)[0]
            assert np.linalg.norm(v - ref) <= 1e-9 * np.linalg.norm(ref)
        assert abs(res - target) <= 1e-10 * target
    # below the stacked noise level: v = 0 at every frequency
    zero = np.flatnonzero(bj[0] == 0)
    assert len(zero) > 0
    assert not np.any(Vj[:, :, :, :].reshape(2, p.nz, N)[:, :, zero])


def test_joint_rule_end_to_end():
    # invert(rule="joint"): stages consistent with solve_joint, xi finite
    p, Wd, u0 = _joint_case()
    xi, st = invert.invert(p, Wd, u0, 0.02, rule="joint", stages=True)
    Vj, aj, bj = invert.solve_joint(p, np.fft.fft2(Wd), 0.02)
    assert np.array_equal(st["branch"], bj)
    assert np.linalg.norm(st["Vhat"] - Vj) == 0.0
    assert np.all(np.isfinite(xi))
