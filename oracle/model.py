"""Discrete model of the flat-layer problem (oracle; test infrastructure only).

Follows the paper's Section 1 (eq. 1-4), Section 2 (eq. 5) and Section 5
(discretization on uniform grids; G~ and U~0 from the FFT of sampled
functions). Conventions taken here, each a reading of a passage the paper
leaves open:

* X cells are centred: x_i = (i + 1/2) h, z'_l = (l + 1/2) hz, quadrature
  weight h per horizontal direction and hz vertically (midpoint rule for the
  mu_kl of Section 5.2; hz = p.dz, equal to h unless the cells are
  anisotropic, as on the paper's grids).
* The horizontal plane is a Px x Py torus; X's nx x ny window sits at offset
  o = ((Px - nx) // 2, (Py - ny) // 2). Horizontal distances use the minimum
  image, so for points inside the window the torus sum equals the infinite
  layer sum as long as Px >= 2 nx - 1.
* The 2D transform is the unnormalized DFT with exp(-i ...) (Section 2 prints
  exp(+i(Omega1 x + Omega1 y)); the sign flip leaves xi unchanged, a pinned
  invariant); the inverse carries 1/(Px Py).
* Ĝ_zeta[m] = h^2 * DFT(G sampled on the torus at height zeta) (Section 5:
  the discrete G~ comes from the FFT of sampled G).
* A_m[j, l] = omega^2 * hz * Ĝ_{z_j - z'_l}[m] (eq. 8 with mu = hz).
* The in-X volume potential of eq. (4)/(9) is the linear convolution of v
  with kappa[d] = h^2 hz G(|(h d_x, h d_y, hz d_z)|), d != 0, and at d = 0
  the integral of G over the ball of the cell's volume h^2 hz (the paper is
  silent on the self cell).

Parity: every function here is pinned (brute-force direct sums, numerical
quadrature, closed forms) by tests/test_oracle_model.py.
"""
from __future__ import annotations

import numpy as np


def green(rho, k0):
    """G(rho) = -exp(i k0 rho) / (4 pi rho) (Section 1, Green function of
    the Helmholtz operator with k0 = omega / c0)."""
    rho = np.asarray(rho, dtype=np.float64)
    return -np.exp(1j * k0 * rho) / (4.0 * np.pi * rho)


def min_image(n: int) -> np.ndarray:
    """Signed torus offsets 0, 1, ..., n/2, -(n/2 - 1), ..., -1 (n/2 kept
    positive; G is radial so its sign is immaterial)."""
    i = np.arange(n)
    return np.where(i <= n // 2, i, i - n)


def window_offset(p):
    return ((p.px - p.nx) // 2, (p.py - p.ny) // 2)


def z_cells(p) -> np.ndarray:
    return (np.arange(p.nz) + 0.5) * p.dz


def k0_of(p, f: int) -> float:
    return float(p.omegas[f]) / float(p.c0)


def horizontal_rho2(p) -> np.ndarray:
    """Squared horizontal minimum-image distances on the torus, (py, px)."""
    dx = p.h * min_image(p.px)
    dy = p.h * min_image(p.py)
    return dy[:, None] ** 2 + dx[None, :] ** 2


def plane_kernel_hat(p, k0: float, zeta: float) -> np.ndarray:
    """Ĝ_zeta[my, mx] = h^2 * sum_p G(sqrt(rho_p^2 + zeta^2)) e^{-2 pi i p.m/P}
    for one height difference zeta != 0 (Section 5, FFT of sampled G)."""
    g = green(np.sqrt(horizontal_rho2(p) + zeta * zeta), k0)
    return p.h * p.h * np.fft.fft2(g)


def dft2_at(arr: np.ndarray, ms, px: int, py: int) -> np.ndarray:
    """The unnormalized 2D DFT of arr (..., py, px) at the flat wavenumber
    indices ms (m = my*px + mx) only, by the definition
    sum_p arr[p] exp(-2 pi i (px mx / Px + py my / Py)) (the sum over x as a
    matrix product with the Fourier vectors, then over y): the transform of
    Section 2 for a sample of wavenumbers, without a full FFT."""
    ms = np.asarray(ms)
    mx, my = ms % px, ms // px
    ex = np.exp(-2j * np.pi * np.outer(np.arange(px), mx) / px)       # (px, S)
    ey = np.exp(-2j * np.pi * np.outer(np.arange(py), my) / py)       # (py, S)
    t = np.asarray(arr, np.complex128) @ ex                            # (..., py, S)
    return np.einsum("...ys,ys->...s", t, ey)


def system_table_at(p, f: int, ms):
    """Ĝ for every distinct zeta at frequency f and the sampled wavenumbers
    ms only: (n_zeta, len(ms)), plus the (nd, nz) index map (the FFT of
    sampled G of Section 5, evaluated by dft2_at)."""
    k0 = k0_of(p, f)
    zetas, idx = zeta_index(p)
    rho2 = horizontal_rho2(p)
    tab = np.stack([p.h * p.h * dft2_at(green(np.sqrt(rho2 + z * z), k0), ms, p.px, p.py)
                    for z in zetas])
    return tab, idx


def zeta_index(p):
    """Distinct height differences z_j - z'_l and the map (j, l) -> index.

    Returns (zetas, idx) with idx shaped (nd, nz). When the data planes lie
    on X's z-lattice there are nd + nz - 1 distinct values."""
    zeta = np.asarray(p.planes, np.float64)[:, None] - z_cells(p)[None, :]
    key = np.round(zeta / (p.h * 1e-9)).astype(np.int64)
    uniq, inv = np.unique(key, return_inverse=True)
    zetas = np.empty(len(uniq))
    zetas[inv.ravel()] = zeta.ravel()
    return zetas, inv.reshape(zeta.shape)


def torus_wavenumbers(p):
    """(kx, ky) of every DFT index on the torus, (py, px) each: 2 pi m / (P h)
    with m the signed index."""
    kx = 2.0 * np.pi * min_image(p.px) / (p.px * p.h)
    ky = 2.0 * np.pi * min_image(p.py) / (p.py * p.h)
    return np.broadcast_to(kx[None, :], (p.py, p.px)), np.broadcast_to(ky[:, None], (p.py, p.px))


def system_table(p, f: int, kernel_mode: int = 0, damping: float = 0.0):
    """Ĝ for every distinct zeta at frequency f: (n_zeta, py, px), plus the
    (nd, nz) index map of zeta_index. kernel_mode 0: the FFT of G sampled on
    the torus (Section 5); 1: the continuous transform (closed form) at the
    torus wavenumbers, with k0 -> k0 (1 + i damping)."""
    k0 = k0_of(p, f)
    zetas, idx = zeta_index(p)
    if kernel_mode == 0:
        tab = np.stack([plane_kernel_hat(p, k0, z) for z in zetas])
    else:
        kx, ky = torus_wavenumbers(p)
        k0c = k0 * (1.0 + 1j * damping)
        tab = np.stack([closed_form_ghat(kx, ky, z, k0c) for z in zetas])
    return tab, idx


def system_matrices(p, f: int, tab, idx, ms) -> np.ndarray:
    """A_m for the flat system indices ms (m = my*px + mx): (len(ms), nd, nz).

    A_m[j, l] = omega^2 * hz * Ĝ_{z_j - z'_l}[m] (eq. 8 with mu_kl = hz).
    With ms = None, tab holds the sampled columns already (system_table_at)."""
    om = float(p.omegas[f])
    if ms is None:
        flat = tab
    else:
        flat = tab.reshape(tab.shape[0], -1)[:, np.asarray(ms)]   # (n_zeta, len(ms))
    return (om * om * p.dz) * flat[idx].transpose(2, 0, 1)


def embed(p, vX: np.ndarray) -> np.ndarray:
    """Place a field on X's window, (nz, ny, nx), into the (nz, py, px) torus."""
    ox, oy = window_offset(p)
    out = np.zeros((vX.shape[0], p.py, p.px), np.complex128)
    out[:, oy:oy + p.ny, ox:ox + p.nx] = vX
    return out


def crop(p, v: np.ndarray) -> np.ndarray:
    """Restrict a torus field (..., py, px) to X's window (..., ny, nx)."""
    ox, oy = window_offset(p)
    return v[..., oy:oy + p.ny, ox:ox + p.nx]


def data_operator(p, f: int, vX: np.ndarray, tab=None, idx=None) -> np.ndarray:
    """W[j] = omega^2 * int_X G(|x - x'|) v(x') dx' on the data planes
    (eq. 3; eq. 7 second line after the 2D transform), discretized on the
    torus. vX: (nz, ny, nx) -> W: (nd, py, px)."""
    if tab is None:
        tab, idx = system_table(p, f)
    om = float(p.omegas[f])
    V = np.fft.fft2(embed(p, vX))                  # (nz, py, px)
    What = np.zeros((p.nd, p.py, p.px), np.complex128)
    for j in range(p.nd):
        for l in range(p.nz):
            What[j] += tab[idx[j, l]] * V[l]
    return (om * om * p.dz) * np.fft.ifft2(What)


def data_operator_zconv(p, f: int, vX: np.ndarray, tab=None, idx=None) -> np.ndarray:
    """data_operator for data planes on X's z-lattice (the Toeplitz case,
    idx[j, l] = j - l + nz - 1): the sum over l of Ĝ_{j-l} V_l is a linear
    convolution along z, evaluated here by a zero-padded FFT along z instead
    of the double loop over (j, l). Same operator, for grids where the loop
    is too slow (pinned against data_operator)."""
    if tab is None:
        tab, idx = system_table(p, f)
    jj, ll = np.meshgrid(np.arange(p.nd), np.arange(p.nz), indexing="ij")
    if not np.array_equal(idx, jj - ll + p.nz - 1):
        raise ValueError("data_operator_zconv needs data planes on X's z-lattice")
    om = float(p.omegas[f])
    V = np.fft.fft2(embed(p, vX))                  # (nz, py, px)
    L = p.nd + 2 * p.nz - 2                        # linear convolution length
    T = np.fft.fft(tab, n=L, axis=0)
    T *= np.fft.fft(V, n=L, axis=0)
    What = np.fft.ifft(T, axis=0)[p.nz - 1:p.nz - 1 + p.nd]
    return (om * om * p.dz) * np.fft.ifft2(What)


def self_cell(k0: float, h: float, hz: float | None = None) -> complex:
    """Integral of G over the ball of the cell's volume h^2 hz (h^3 when hz
    is None) centred at the singularity: a = (3 h^2 hz / (4 pi))^(1/3),
    S = (1 - (1 - i k0 a) e^{i k0 a}) / k0^2."""
    vol = h * h * (h if hz is None else hz)
    a = (3.0 * vol / (4.0 * np.pi)) ** (1.0 / 3.0)
    ika = 1j * k0 * a
    return complex((1.0 - (1.0 - ika) * np.exp(ika)) / (k0 * k0))


def conv_kernel(p, k0: float) -> np.ndarray:
    """kappa on the zero-padded (2nz, 2ny, 2nx) torus with minimum-image
    offsets: h^2 hz G(|(h d_x, h d_y, hz d_z)|) for d != 0 and the
    self-cell integral at d = 0."""
    dz = p.dz * min_image(2 * p.nz)
    dy = p.h * min_image(2 * p.ny)
    dx = p.h * min_image(2 * p.nx)
    r = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
    r[0, 0, 0] = 1.0
    kap = p.h * p.h * p.dz * green(r, k0)
    kap[0, 0, 0] = self_cell(k0, p.h, p.dz)
    return kap


def volume_potential(p, f: int, vX: np.ndarray) -> np.ndarray:
    """omega^2 * int_X G(|x - x'|) v(x') dx' for x in X (eq. 4 / eq. 9), as a
    zero-padded 3D FFT linear convolution. vX: (nz, ny, nx)."""
    k0 = k0_of(p, f)
    om = float(p.omegas[f])
    shape = (2 * p.nz, 2 * p.ny, 2 * p.nx)
    K = np.fft.fftn(conv_kernel(p, k0))
    Vp = np.zeros(shape, np.complex128)
    Vp[:p.nz, :p.ny, :p.nx] = vX
    out = np.fft.ifftn(K * np.fft.fftn(Vp))
    return (om * om) * out[:p.nz, :p.ny, :p.nx]


def closed_form_ghat(kx, ky, zeta, k0):
    """Continuous 2D transform of G at height difference zeta:
    -i exp(i gamma |zeta|) / (2 gamma), gamma = sqrt(k0^2 - |k|^2), Im gamma >= 0
    (Weyl expansion of the point-source field); k0 may be complex (damping)."""
    g = np.sqrt(np.asarray(k0 * k0 - kx * kx - ky * ky, np.complex128))
    g = np.where(g.imag < 0, -g, g)
    return -1j * np.exp(1j * g * abs(zeta)) / (2.0 * g)
