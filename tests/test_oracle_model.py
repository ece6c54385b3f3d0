"""Pins of the oracle's discrete model against brute force, quadrature and
closed forms (no GPU)."""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import model
from paper_1911_10487_amd import synth


def _brute_data(p, f, vX):
    """W[j, py, px] = omega^2 h^3 sum_{l, window q} G(|x_p,j - x_q,l|) v[l, q]
    with minimum-image horizontal distances: eq. (3) with the midpoint rule,
    written as a direct sum."""
    om = p.omegas[f]
    k0 = om / p.c0
    ox, oy = model.window_offset(p)
    hz = p.h if p.hz is None else p.hz
    zx = (np.arange(p.nz) + 0.5) * hz
    W = np.zeros((p.nd, p.py, p.px), complex)
    for j in range(p.nd):
        for py in range(p.py):
            for px in range(p.px):
                acc = 0j
                for l in range(p.nz):
                    for iy in range(p.ny):
                        for ix in range(p.nx):
                            dx = (px - (ix + ox)) % p.px
                            dy = (py - (iy + oy)) % p.py
                            dx = dx if dx <= p.px // 2 else dx - p.px
                            dy = dy if dy <= p.py // 2 else dy - p.py
                            r = np.sqrt((dx * p.h) ** 2 + (dy * p.h) ** 2
                                        + (p.planes[j] - zx[l]) ** 2)
                            acc += -np.exp(1j * k0 * r) / (4 * np.pi * r) * vX[l, iy, ix]
                W[j, py, px] = om * om * p.h ** 2 * hz * acc
    return W


def test_data_operator_matches_direct_sum():
    # non-square window and torus so that an x/y swap cannot pass
    p = synth.tiny_problem(nx=3, ny=2, nz=2, nd=3, px=8, py=6)
    vX = synth.random_field((p.nz, p.ny, p.nx), (5, 1))
    W = model.data_operator(p, 0, vX)
    Wb = _brute_data(p, 0, vX)
    assert np.linalg.norm(W - Wb) <= 1e-13 * np.linalg.norm(Wb)


def test_system_matrix_is_the_data_operator_per_wavenumber():
    p = synth.tiny_problem(nx=3, ny=2, nz=2, nd=3, px=8, py=6)
    vX = synth.random_field((p.nz, p.ny, p.nx), (5, 2))
    W = model.data_operator(p, 0, vX)
    What = np.fft.fft2(W).reshape(p.nd, -1)
    V = np.fft.fft2(model.embed(p, vX)).reshape(p.nz, -1)
    tab, idx = model.system_table(p, 0)
    ms = np.arange(p.px * p.py)
    A = model.system_matrices(p, 0, tab, idx, ms)
    lhs = np.einsum("mjl,lm->jm", A, V)
    assert np.linalg.norm(lhs - What) <= 1e-13 * np.linalg.norm(What)
    # on-lattice planes: nd + nz - 1 distinct heights, Toeplitz systems
    assert tab.shape[0] == p.nd + p.nz - 1
    assert np.allclose(A[:, 1:, 1:], A[:, :-1, :-1], rtol=0, atol=0)


def _brute_volume(p, f, vX):
    om = p.omegas[f]
    k0 = om / p.c0
    hz = p.h if p.hz is None else p.hz
    # the self cell: the ball of the cell's volume h^2 hz (quadrature-pinned
    # below)
    S = model.self_cell(k0, p.h, hz)
    out = np.zeros_like(vX)
    idx = [(l, iy, ix) for l in range(p.nz) for iy in range(p.ny) for ix in range(p.nx)]
    for a in idx:
        acc = 0j
        for b in idx:
            d = np.array(a) - np.array(b)
            if not d.any():
                acc += S * vX[b]
            else:
                r = np.sqrt((hz * d[0]) ** 2 + (p.h * d[1]) ** 2 + (p.h * d[2]) ** 2)
                acc += p.h ** 2 * hz * (-np.exp(1j * k0 * r) / (4 * np.pi * r)) * vX[b]
        out[a] = om * om * acc
    return out


@pytest.mark.parametrize("hz", [None, 0.05])
def test_volume_potential_matches_direct_sum(hz):
    # cubic cells, and flat ones (hz < h, as on the paper's grids)
    p = synth.tiny_problem(nx=3, ny=4, nz=2)
    p.hz = hz
    vX = synth.random_field((p.nz, p.ny, p.nx), (5, 3))
    u = model.volume_potential(p, 0, vX)
    ub = _brute_volume(p, 0, vX)
    assert np.linalg.norm(u - ub) <= 1e-13 * np.linalg.norm(ub)


def test_data_operator_with_flat_cells_matches_direct_sum():
    # hz != h: planes hz apart on X's vertical lattice, and off it
    p = synth.make_problem("flat", 3, 2, 3, [2 * np.pi], 2, (99, 1), (0.0,), nd=3, px=8, py=6,
                           hz=0.06)
    vX = synth.random_field((p.nz, p.ny, p.nx), (5, 7))
    for planes in (p.planes.copy(), p.nz * 0.06 + 0.3 + np.array([0.0, 0.011, 0.05])):
        p.planes = planes
        W = model.data_operator(p, 0, vX)
        Wb = _brute_data(p, 0, vX)
        assert np.linalg.norm(W - Wb) <= 1e-13 * np.linalg.norm(Wb)


@pytest.mark.parametrize("k0", [0.7, 2 * np.pi, 5 * np.pi])
def test_self_cell_is_the_ball_integral(k0):
    h = 0.125
    a = h * (3 / (4 * np.pi)) ** (1 / 3)
    # int_ball G dV = int_0^a 4 pi r^2 G(r) dr, evaluated numerically
    re = integrate.quad(lambda r: (-r * np.exp(1j * k0 * r)).real, 0, a, epsabs=1e-22, epsrel=1e-13)[0]
    im = integrate.quad(lambda r: (-r * np.exp(1j * k0 * r)).imag, 0, a, epsabs=1e-22, epsrel=1e-13)[0]
    S = model.self_cell(k0, h)
    assert abs(S - (re + 1j * im)) <= 1e-12 * abs(S)
    # the ball has the cell's volume
    assert abs(4 / 3 * np.pi * a ** 3 - h ** 3) < 1e-15
    # a flat cell h x h x hz: the ball of volume h^2 hz
    hz = 0.03
    a2 = (3 * h * h * hz / (4 * np.pi)) ** (1 / 3)
    re = integrate.quad(lambda r: (-r * np.exp(1j * k0 * r)).real, 0, a2, epsabs=1e-22, epsrel=1e-13)[0]
    im = integrate.quad(lambda r: (-r * np.exp(1j * k0 * r)).imag, 0, a2, epsabs=1e-22, epsrel=1e-13)[0]
    S2 = model.self_cell(k0, h, hz)
    assert abs(S2 - (re + 1j * im)) <= 1e-12 * abs(S2)


def test_self_cell_low_frequency_series():
    # -int_0^a r e^{ikr} dr = -a^2/2 - i k a^3/3 + k^2 a^4/8 + O(k^3 a^5)
    h = 0.125
    a = h * (3 / (4 * np.pi)) ** (1 / 3)
    k = 1e-2
    series = -a * a / 2 - 1j * k * a ** 3 / 3 + k * k * a ** 4 / 8
    assert abs(model.self_cell(k, h) - series) < 1e-8 * a * a


def test_green_solves_helmholtz_away_from_source():
    k0 = 2 * np.pi
    x0 = np.array([0.31, -0.22, 0.47])
    e = 1e-3
    g = lambda x: model.green(np.linalg.norm(x), k0)
    lap = sum(g(x0 + e * ei) + g(x0 - e * ei) - 2 * g(x0) for ei in np.eye(3)) / e ** 2
    assert abs(lap + k0 * k0 * g(x0)) < 1e-4 * abs(k0 * k0 * g(x0))


def test_green_unit_flux():
    # Delta G = delta: the flux of grad G through a small sphere tends to 1
    k0 = 2 * np.pi
    r, e = 1e-4, 1e-8
    dGdr = (model.green(r + e, k0) - model.green(r - e, k0)) / (2 * e)
    assert abs(4 * np.pi * r * r * dGdr - 1) < 1e-3


@pytest.mark.parametrize("kx,ky", [(1.0, 0.5), (3.0, -2.0), (8.0, 1.0)])
def test_closed_form_ghat_against_hankel_quadrature(kx, ky):
    # 2D transform of the (slightly damped) point-source field as the Hankel
    # integral 2 pi int_0^inf G(sqrt(rho^2 + zeta^2)) J0(|k| rho) rho drho
    k0 = 2 * np.pi * (1 + 0.05j)
    zeta = 0.3
    kk = np.hypot(kx, ky)
    def integrand(r, part):
        R = np.sqrt(r * r + zeta * zeta)
        val = 2 * np.pi * (-np.exp(1j * k0 * R) / (4 * np.pi * R)) * special.j0(kk * r) * r
        return val.real if part == 0 else val.imag
    edges = np.linspace(0, 120, 1201)
    tot = 0j
    for a, b in zip(edges[:-1], edges[1:]):
        tot += integrate.quad(integrand, a, b, args=(0,), epsabs=1e-15, epsrel=1e-13)[0]
        tot += 1j * integrate.quad(integrand, a, b, args=(1,), epsabs=1e-15, epsrel=1e-13)[0]
    ref = model.closed_form_ghat(kx, ky, zeta, k0)
    assert abs(tot - ref) <= 1e-8 * abs(ref)


def test_sampled_table_converges_to_the_continuous_transform():
    # With damping (k0 -> k0 (1 + 0.3 i)) the sampled field decays within the
    # torus, and h^2 * DFT(sampled G) converges to the continuous 2D transform
    # -i e^{i gamma |zeta|} / (2 gamma) as h -> 0 at fixed torus length: this
    # pins the h^2 weight, the DFT sign and the minimum-image layout.
    k0 = 2 * np.pi * (1 + 0.3j)
    zeta = 0.5
    L = 32.0
    errs = []
    for n in (64, 128, 256):
        h = L / n
        p = synth.make_problem("t", n // 2, n // 2, 2, [1.0], 1, (0, 0), h=h)
        g = model.plane_kernel_hat(p, k0, zeta)
        for (my, mx) in ((0, 8), (3, 5)):
            kx = 2 * np.pi * mx / (p.px * h)
            ky = 2 * np.pi * my / (p.py * h)
            ref = model.closed_form_ghat(kx, ky, zeta, k0)
            errs.append(abs(g[my, mx] - ref) / abs(ref))
    assert errs[0] > errs[2] > errs[4] and errs[1] > errs[3] > errs[5]
    assert max(errs[4], errs[5]) < 1e-9


def test_noise_has_exact_relative_level_and_parseval():
    p = synth.tiny_problem(nx=4, ny=4, nz=3, px=8, py=8)
    W = synth.random_field((1, p.nd, p.py, p.px), (6, 0))
    for d in (1e-3, 0.05):
        Wd = synth.add_noise(p, W, d)
        assert abs(np.linalg.norm(Wd - W) / np.linalg.norm(W) - d) < 1e-14
    # sum_m ||e^_m||^2 = N ||e||^2 for the unnormalized transform
    e = synth.noise_direction(p, 0)
    eh = np.fft.fft2(e)
    N = p.px * p.py
    assert abs(np.sum(abs(eh) ** 2) - N * np.sum(abs(e) ** 2)) < 1e-12 * N


def test_closed_form_table_matches_sampled_table_and_is_rank_one():
    # kernel_mode 1 puts the continuous transform at the torus wavenumbers
    # (pinned above by quadrature); with damping the sampled table converges
    # to it, so the two modes agree at low wavenumbers on a fine grid, and
    # every closed-form A_m = omega^2 h (-i/(2 gamma)) e^{i gamma z_j}
    # e^{-i gamma z'_l} has rank one (data planes above X)
    p = synth.make_problem("cf", 128, 128, 4, [2 * np.pi], 1, (0, 0), h=0.125)
    damping = 0.3
    f = 0
    tc, idx = model.system_table(p, f, kernel_mode=1, damping=damping)
    k0 = model.k0_of(p, f) * (1 + 1j * damping)
    ts = np.stack([model.plane_kernel_hat(p, k0, z) for z in model.zeta_index(p)[0]])
    for (my, mx) in ((0, 0), (0, 3), (2, 5), (p.py - 1, 1)):
        e = np.max(np.abs(tc[:, my, mx] - ts[:, my, mx]) / np.abs(tc[:, my, mx]))
        assert e < 1e-6, (my, mx, e)
    ms = np.array([0, 7, 129, 4000])
    A = model.system_matrices(p, f, tc, idx, ms)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.all(s[:, 1] <= 1e-12 * s[:, 0])
    assert np.all(s[:, 0] > 0)


@pytest.mark.parametrize("px,py", [(64, 64), (40, 30), (45, 45)])
def test_table_is_invariant_under_the_torus_symmetries(px, py):
    # G is radial, and the min-image samples of the torus are symmetric under
    # x -> -x, y -> -y (and x <-> y when px = py): so is G^, and every A_m
    # depends on the orbit of m only (the GPU path factorizes one A per orbit)
    p = synth.make_problem("sym", px // 2, py // 2, 4, [2 * np.pi], 3, (0, 0), (0.0,),
                           px=px, py=py)
    tab, _ = model.system_table(p, 0)
    scale = np.abs(tab).max()
    ix = (-np.arange(px)) % px
    iy = (-np.arange(py)) % py
    assert np.abs(tab[:, :, ix] - tab).max() <= 1e-13 * scale
    assert np.abs(tab[:, iy, :] - tab).max() <= 1e-13 * scale
    if px == py:
        assert np.abs(tab.transpose(0, 2, 1) - tab).max() <= 1e-13 * scale
    # and the symmetry is not vacuous: G^ does vary across the wavenumbers
    assert np.abs(tab - tab[:, :1, :1]).max() > 0.1 * scale


def test_thin_layer_data_operator_matches_direct_sum():
    # two data planes 0.01 apart, off X's z-lattice: nd * nz distinct heights
    p = synth.thin_problem("thin", 3, 2, 2, [2 * np.pi], 1, (0, 0), gap=0.3, spacing=0.01,
                           px=8, py=6)
    vX = synth.random_field((p.nz, p.ny, p.nx), (5, 3))
    W = model.data_operator(p, 0, vX)
    Wb = _brute_data(p, 0, vX)
    assert np.linalg.norm(W - Wb) <= 1e-13 * np.linalg.norm(Wb)
    tab, idx = model.system_table(p, 0)
    assert tab.shape[0] == p.nd * p.nz


def test_sampled_dft_is_the_fft_at_those_wavenumbers():
    # non-square torus (an x/y mix-up fails) and a leading batch axis
    rng = np.random.default_rng(7)
    a = rng.standard_normal((3, 6, 10)) + 1j * rng.standard_normal((3, 6, 10))
    ms = np.array([0, 1, 9, 10, 23, 59, 31])
    got = model.dft2_at(a, ms, 10, 6)
    ref = np.fft.fft2(a).reshape(3, -1)[:, ms]
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_sampled_table_matches_the_full_table():
    p = synth.tiny_problem(nx=3, ny=2, nz=3, nd=3, px=8, py=6)
    tab, idx = model.system_table(p, 0)
    ms = np.array([0, 5, 7, 13, 47])
    tab_s, idx_s = model.system_table_at(p, 0, ms)
    assert np.array_equal(idx, idx_s)
    ref = tab.reshape(tab.shape[0], -1)[:, ms]
    assert np.linalg.norm(tab_s - ref) <= 1e-13 * np.linalg.norm(ref)
    A = model.system_matrices(p, 0, tab, idx, ms)
    A_s = model.system_matrices(p, 0, tab_s, idx_s, None)
    assert np.linalg.norm(A_s - A) <= 1e-13 * np.linalg.norm(A)


def test_zconv_data_operator_matches_the_direct_one():
    # the z-convolution route against the (j, l) double loop, and against the
    # brute-force direct sum on a grid small enough for it
    p = synth.tiny_problem(nx=3, ny=2, nz=3, nd=3, px=8, py=6)
    vX = synth.random_field((p.nz, p.ny, p.nx), (5, 3))
    W = model.data_operator_zconv(p, 0, vX)
    Wb = _brute_data(p, 0, vX)
    assert np.linalg.norm(W - Wb) <= 1e-13 * np.linalg.norm(Wb)
    p = synth.make_problem("zc", 10, 8, 12, [2 * np.pi], 2, (5, 4), (0.0,), px=20, py=16)
    vX = synth.random_field((p.nz, p.ny, p.nx), (5, 4))
    W1 = model.data_operator(p, 0, vX)
    W2 = model.data_operator_zconv(p, 0, vX)
    assert np.linalg.norm(W2 - W1) <= 1e-13 * np.linalg.norm(W1)
    # off the lattice (a thin layer) it refuses
    p = synth.thin_problem("zt", 4, 4, 4, [2 * np.pi], 1, (5, 5))
    with pytest.raises(ValueError):
        model.data_operator_zconv(p, 0, synth.random_field((p.nz, p.ny, p.nx), (5, 6)))
