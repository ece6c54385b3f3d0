"""Seeded synthetic inputs for the flat-layer inversion workloads.

This module only draws random numbers and lays out grids; it holds none of
the inversion's arithmetic. Both the CPU oracle (through the tests) and the
GPU path take their inputs from here, so that the two sides see identical
data.

Geometry follows the paper's data-recording scheme (Section 2, flat layers
X = R^2 x [z1, z2] and Y = R^2 x [z3, z4]): the inhomogeneity layer X is the
box [0, nx*h] x [0, ny*h] x [0, nz*h] sampled at cell centres, the data
planes sit above it at heights ``planes[j]``, and the horizontal plane is
periodised on a Px x Py torus that holds X's window in its middle.

Workloads (all with c0 = 1, h = 0.125 and nd = nz data planes spaced h apart,
two cells above the top of X):

* ``small``   32x32x16 X, 64x64 torus, one frequency omega = 2*pi, 3 blobs.
* ``single``  128x128x64 X, 256x256 torus, omega = 2*pi, 3 blobs.
* ``multi5``  the ``single`` grid with omega = 2*pi*{0.5,1,1.5,2,2.5}, 5 blobs.
* ``uneven``  four grids 64^2x32, 96^2x48, 160^2x80, 192^2x96, three
  frequencies 2*pi*{0.75,1.25,1.75}, 3-8 blobs each.
* ``large``   256x256x128 X, 512x512 torus, omega = 2*pi*{0.5..2.0 step 0.25}.

The contrast xi is a sum of Gaussian blobs (centres uniform in X shrunk by
2 sigma per side, sigma ~ U[0.15, 0.4], amplitude ~ U[-0.3, 0.3]); the
incident field u0 is that of a unit point source placed one unit below the
centre of X's bottom face, as in the paper's point-source experiments
(Section 5, sources of the form sum A_m delta(x - x_m)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

H = 0.125
C0 = 1.0
TWO_PI = 2.0 * np.pi


@dataclass
class Problem:
    """One inversion instance: grid, frequencies and its random fields."""

    name: str
    nx: int
    ny: int
    nz: int
    nd: int
    h: float
    planes: np.ndarray  # (nd,) heights z_j of the data planes
    omegas: np.ndarray  # (n_omega,) angular frequencies
    c0: float
    px: int
    py: int
    n_blobs: int
    seed: tuple = ()
    deltas: tuple = (0.01,)
    source: tuple = field(default=(0.0, 0.0, 0.0))
    hz: float | None = None  # vertical cell size of X; None: h (cubic cells)

    @property
    def dz(self) -> float:
        """Vertical cell size of X (h unless the cells are anisotropic)."""
        return self.h if self.hz is None else self.hz

    @property
    def n_omega(self) -> int:
        return len(self.omegas)

    @property
    def voxel_frequencies(self) -> int:
        return self.nx * self.ny * self.nz * self.n_omega

    def cell_centres(self):
        """Cell-centre coordinates of X, each shaped (nz, ny, nx)."""
        xs = (np.arange(self.nx) + 0.5) * self.h
        ys = (np.arange(self.ny) + 0.5) * self.h
        zs = (np.arange(self.nz) + 0.5) * self.dz
        z3, y3, x3 = np.meshgrid(zs, ys, xs, indexing="ij")
        return x3, y3, z3


def _planes(nz: int, nd: int, h: float) -> np.ndarray:
    # Data planes two cells above the top of X, spaced h apart, so that
    # z_j - z'_l depends on j - l only.
    return nz * h + 2.0 * h + h * np.arange(nd)


def make_problem(name: str, nx: int, ny: int, nz: int, omegas, n_blobs: int,
                 seed: tuple, deltas=(0.01,), h: float = H, nd: int | None = None,
                 px: int | None = None, py: int | None = None,
                 hz: float | None = None) -> Problem:
    """hz: vertical cell size (None: h); the data planes then sit two
    vertical cells above X, hz apart."""
    nd = nz if nd is None else nd
    dz = h if hz is None else hz
    return Problem(
        name=name, nx=nx, ny=ny, nz=nz, nd=nd, h=h,
        planes=_planes(nz, nd, dz),
        omegas=np.asarray(omegas, dtype=np.float64),
        c0=C0, px=px or 2 * nx, py=py or 2 * ny, n_blobs=n_blobs,
        seed=tuple(seed), deltas=tuple(deltas),
        source=(nx * h / 2.0, ny * h / 2.0, -1.0), hz=hz,
    )


def thin_problem(name: str, nx: int, ny: int, nz: int, omegas, n_blobs: int, seed: tuple,
                 deltas=(0.01,), gap: float = 0.5, spacing: float = 0.01, nd: int = 2,
                 h: float = H, px: int | None = None, py: int | None = None) -> Problem:
    """Data in a thin layer (the paper's second experiment): nd planes
    `spacing` apart, the first `gap` above the top of X; the spacing need
    not be a multiple of h."""
    p = make_problem(name, nx, ny, nz, omegas, n_blobs, seed, deltas, h=h, nd=nd, px=px, py=py)
    p.planes = nz * h + gap + spacing * np.arange(nd)
    return p


def workload(name: str) -> list[Problem]:
    """The named workload as a list of instances (one except ``uneven``)."""
    if name == "small":
        return [make_problem("small", 32, 32, 16, [TWO_PI], 3, (0, 0), (0.0, 0.01))]
    if name == "single":
        return [make_problem("single", 128, 128, 64, [TWO_PI], 3, (1, 0), (0.01,))]
    if name == "multi5":
        om = TWO_PI * np.array([0.5, 1.0, 1.5, 2.0, 2.5])
        return [make_problem("multi5", 128, 128, 64, om, 5, (2, 0), (0.005, 0.02))]
    if name == "uneven":
        om = TWO_PI * np.array([0.75, 1.25, 1.75])
        out = []
        for i, (n, nz) in enumerate([(64, 32), (96, 48), (160, 80), (192, 96)]):
            rng = np.random.default_rng([3, i, 2])
            nb = int(rng.integers(3, 9))
            d = float(rng.uniform(0.005, 0.02))
            out.append(make_problem(f"uneven{i}", n, n, nz, om, nb, (3, i), (d,)))
        return out
    if name == "large":
        om = TWO_PI * np.arange(0.5, 2.0 + 1e-9, 0.25)
        return [make_problem("large", 256, 256, 128, om, 5, (4, 0), (0.01,))]
    raise KeyError(name)


def tiny_problem(nx=4, ny=4, nz=3, nd=None, px=None, py=None, omegas=(TWO_PI,),
                 h=0.125, seed=(99, 0), n_blobs=2) -> Problem:
    """A grid small enough for brute-force direct sums."""
    return make_problem("tiny", nx, ny, nz, omegas, n_blobs, seed, (0.0, 0.01),
                        h=h, nd=nd, px=px, py=py)


def blob_params(p: Problem):
    """Gaussian blob parameters (centres, sigmas, amplitudes), seeded."""
    rng = np.random.default_rng(list(p.seed) + [0])
    sig = rng.uniform(0.15, 0.4, p.n_blobs)
    amp = rng.uniform(-0.3, 0.3, p.n_blobs)
    ext = np.array([p.nx * p.h, p.ny * p.h, p.nz * p.dz])
    cen = np.empty((p.n_blobs, 3))
    for b in range(p.n_blobs):
        lo = np.minimum(2.0 * sig[b], ext / 2.0)
        cen[b] = rng.uniform(lo, ext - lo)
    return cen, sig, amp


def contrast(p: Problem) -> np.ndarray:
    """xi_true on X's cell centres, shaped (nz, ny, nx), float64."""
    x3, y3, z3 = p.cell_centres()
    cen, sig, amp = blob_params(p)
    xi = np.zeros_like(x3)
    for c, s, a in zip(cen, sig, amp):
        r2 = (x3 - c[0]) ** 2 + (y3 - c[1]) ** 2 + (z3 - c[2]) ** 2
        xi += a * np.exp(-r2 / (2.0 * s * s))
    return xi


def incident_field(p: Problem) -> np.ndarray:
    """u0 of a unit point source at ``p.source`` for every frequency,
    shaped (n_omega, nz, ny, nx), complex128: the free-space field
    -exp(i k0 r)/(4 pi r) of the source (Section 5, u0 of point sources)."""
    x3, y3, z3 = p.cell_centres()
    s = p.source
    r = np.sqrt((x3 - s[0]) ** 2 + (y3 - s[1]) ** 2 + (z3 - s[2]) ** 2)
    out = np.empty((p.n_omega,) + x3.shape, np.complex128)
    for f, om in enumerate(p.omegas):
        k0 = om / p.c0
        out[f] = -np.exp(1j * k0 * r) / (4.0 * np.pi * r)
    return out


def noise_direction(p: Problem, f: int) -> np.ndarray:
    """Unit-norm complex Gaussian direction e/||e|| on frequency f's data
    array (nd, py, px); the paper's noise is zero-mean normal (Section 5.1)."""
    rng = np.random.default_rng(list(p.seed) + [1, f])
    shape = (p.nd, p.py, p.px)
    e = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return e / np.linalg.norm(e)


def add_noise(p: Problem, W: np.ndarray, delta: float) -> np.ndarray:
    """W^delta = W + delta*||W|| e/||e|| per frequency, so that
    ||W^delta - W|| = delta*||W|| holds with equality."""
    out = np.array(W, dtype=np.complex128, copy=True)
    if delta == 0.0:
        return out
    for f in range(W.shape[0]):
        out[f] += delta * np.linalg.norm(W[f]) * noise_direction(p, f)
    return out


def random_field(shape, seed, dtype=np.complex128) -> np.ndarray:
    """Seeded i.i.d. complex normal array (for adjoint and tangent tests)."""
    rng = np.random.default_rng(list(seed))
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return a.astype(dtype)


def paper_contrast(x, y, z, a0=0.3):
    """The model solution of the paper's Section 5: three truncated quadratic
    bumps (radii 0.4, 0.25, 0.3; weights 1, 2, 2.5; two of them sheared in the
    (y, z) plane), scaled by A0 = 0.3. Coordinates in the paper's frame."""
    r1 = (x - 1) ** 2 + (y - 2) ** 2 + (z - 0.5) ** 2
    r2 = (x - 4) ** 2 + (y + 3) ** 2 + (z - 0.5) ** 2 + 1.5 * (y + 3) * (z - 0.5)
    r3 = (x + 3) ** 2 + y ** 2 + (z - 0.45) ** 2 - 1.5 * y * (z - 0.45)
    pos = lambda t: np.maximum(t, 0.0)
    return a0 * (pos(1 - r1 / 0.4 ** 2) + 2 * pos(1 - r2 / 0.25 ** 2)
                 + 2.5 * pos(1 - r3 / 0.3 ** 2))
