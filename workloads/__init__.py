"""Seeded synthetic inputs for the MatExPre hot path.

This module holds the problem *descriptions* only: grid sizes, spacing,
angular frequency, absorbing-layer widths, wave-speed fields and source
terms.  It holds none of the method's arithmetic (no operator coefficients,
no absorbing-layer profiles, no matrix functions, no Krylov code), so that
both the CPU oracle and the GPU path can draw identical inputs from it.

Conventions (the paper's scaling, Section 4 introduction): the grid spacing
is h = 1/(N_max - 1), the wave speed is scaled so that its minimum is 1, and
omega = 2*pi*c_min/(ppw*h) where ppw is points per wavelength.  Arrays are
NumPy, C order with shape (n2, n1, n0) in 3D and (n1, n0) in 2D, so the
flattened index is i + n0*(j + n1*k) with x fastest.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "Problem", "config1", "config2", "config3", "config4_main", "config4_extras",
    "small_problem", "delta_source", "gaussian_source", "grf_speed",
    "layered_speed", "random_vector", "config4_sources", "lens_problem", "lens_source",
    "homog_problem", "dipole_source",
]


@dataclasses.dataclass
class Problem:
    """A Helmholtz problem: omega^2/c^2 u + Lap_PML u = -f on a node grid."""
    name: str
    n: Tuple[int, ...]            # nodes per axis, x first; len 2 or 3
    h: float                      # grid spacing
    omega: float                  # angular frequency
    layer: int                    # absorbing-layer cells on every face
    c: Optional[np.ndarray]       # wave speed per node (shape n[::-1]) or None
    c_const: float = 1.0          # used when c is None
    pml_C: float = 20.0           # absorbing strength constant
    pml_power: int = 2            # quadratic profile
    absorber: str = "pml"         # "pml" (coordinate stretch), "cap" (absorbing potential) or
                                  # "abc" (boundary conditions on the grid's faces, no layer)
    hard_faces: Tuple[Tuple[int, int], ...] = ()  # "abc": sound-hard faces (axis, side); the rest absorb

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def npts(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(reversed(self.n))

    @property
    def freq(self) -> float:
        return self.omega / (2.0 * math.pi)

    def default_t(self) -> float:
        """Time length t = 40 h^2 (0.4/freq^2 at ppw 10; constant t*||A||)."""
        return 40.0 * self.h * self.h

    def default_shift(self) -> float:
        """Complex shift s = 1/freq."""
        return 1.0 / self.freq

    def c_array(self) -> np.ndarray:
        if self.c is not None:
            return self.c
        return np.full(self.shape, self.c_const)


def omega_for(ppw: float, h: float, c_min: float = 1.0) -> float:
    return 2.0 * math.pi * c_min / (ppw * h)


def delta_source(prob: Problem, node: Tuple[int, ...]) -> np.ndarray:
    """Discrete delta: 1/h^d at one node (node given x first)."""
    f = np.zeros(prob.shape, dtype=np.complex128)
    f[tuple(reversed(node))] = 1.0 / prob.h ** prob.dim
    return f


def gaussian_source(prob: Problem, centre: Tuple[float, ...], sigma: float) -> np.ndarray:
    """Normalised Gaussian (unit integral) with standard deviation sigma,
    centre in physical coordinates x_i = i*h (x first)."""
    axes = [np.arange(n) * prob.h for n in prob.n]
    grids = np.meshgrid(*reversed(axes), indexing="ij")  # z, y, x order
    r2 = np.zeros(prob.shape)
    for g, c in zip(grids, reversed(centre)):
        r2 = r2 + (g - c) ** 2
    d = prob.dim
    f = np.exp(-r2 / (2 * sigma * sigma)) / (2 * math.pi * sigma * sigma) ** (d / 2)
    return f.astype(np.complex128)


def grf_speed(shape: Tuple[int, ...], corr_cells: float, lo: float, hi: float,
              seed: int) -> np.ndarray:
    """Smooth Gaussian random field: white N(0,1) filtered in Fourier space by
    exp(-|k|^2 l^2/4) (covariance exp(-r^2/(2 l^2))), mapped affinely to [lo, hi]."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    W = np.fft.fftn(w)
    k2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = 2 * math.pi * np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = n
        k2 = k2 + (k.reshape(sh)) ** 2
    g = np.real(np.fft.ifftn(W * np.exp(-k2 * corr_cells ** 2 / 4)))
    g = (g - g.min()) / (g.max() - g.min())
    return lo + (hi - lo) * g


def layered_speed(n: Tuple[int, int, int], layer: int, nlayers: int, vlo: float,
                  vhi: float, nlens: int, seed: int) -> np.ndarray:
    """Horizontally layered model (z = depth = third axis) with speeds sorted
    increasing with depth, plus ellipsoidal low-speed lenses at vlo; returned
    divided by vlo so the minimum speed is 1."""
    rng = np.random.default_rng(seed)
    n0, n1, n2 = n
    zin = np.arange(layer, n2 - layer)
    depths = np.sort(rng.choice(zin, size=nlayers - 1, replace=False))
    speeds = np.sort(rng.uniform(vlo, vhi, size=nlayers))
    c = np.empty((n2, n1, n0))
    z = np.arange(n2)
    idx = np.searchsorted(depths, z, side="right")
    c[:] = speeds[idx][:, None, None]
    X = np.arange(n0)[None, None, :] / (n0 - 1)
    Y = np.arange(n1)[None, :, None] / (n1 - 1)
    Z = np.arange(n2)[:, None, None] / (n2 - 1)
    for _ in range(nlens):
        cen = rng.uniform(0.3, 0.7, size=3)
        ax = rng.uniform(0.05, 0.15, size=3)
        m = (((X - cen[0]) / ax[0]) ** 2 + ((Y - cen[1]) / ax[1]) ** 2
             + ((Z - cen[2]) / ax[2]) ** 2) <= 1.0
        c[m] = vlo
    return c / vlo


def random_vector(npts: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(npts) + 1j * rng.standard_normal(npts)


def config1() -> Problem:
    """2D homogeneous, 128^2, h = 1/127, c = 1, ppw 10, 16-cell layer."""
    n = 128
    h = 1.0 / (n - 1)
    return Problem("2d-homog-128", (n, n), h, omega_for(10, h), 16, None, 1.0)


def config2(seed: int = 2) -> Problem:
    """2D inhomogeneous, 2048^2, c = GRF (corr. 64 cells) in [1, 3], ppw 8 at
    c_min, 32-cell layer."""
    n = 2048
    h = 1.0 / (n - 1)
    c = grf_speed((n, n), 64.0, 1.0, 3.0, seed)
    return Problem("2d-grf-2048", (n, n), h, omega_for(8, h), 32, c)


def config3() -> Problem:
    """3D homogeneous, 256^3, c = 1, ppw 8, 20-cell layer."""
    n = 256
    h = 1.0 / (n - 1)
    return Problem("3d-homog-256", (n, n, n), h, omega_for(8, h), 20, None, 1.0)


def config4_main(seed: int = 4) -> Problem:
    """3D layered: 512 x 512 x 256, 12 layers in [1500, 4500] m/s + 2 lenses,
    ppw 8 at 1500 m/s, 32-cell layer (speeds scaled by 1/1500)."""
    n = (512, 512, 256)
    h = 1.0 / (max(n) - 1)
    c = layered_speed(n, 32, 12, 1500.0, 4500.0, 2, seed)
    return Problem("3d-layered-512x512x256", n, h, omega_for(8, h), 32, c)


def config4_extras(count: int = 16, seed: int = 44):
    """Uneven-size 3D layered problems, per-axis sizes in [96, 192], 16-cell layer."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = tuple(int(v) for v in rng.integers(96, 193, size=3))
        h = 1.0 / (max(n) - 1)
        c = layered_speed(n, 16, 12, 1500.0, 4500.0, 2, seed * 1000 + i)
        out.append(Problem(f"3d-layered-{n[0]}x{n[1]}x{n[2]}", n, h, omega_for(8, h), 16, c))
    return out


def config4_sources(prob: Problem, which, count: int = 32) -> np.ndarray:
    """Right-hand sides `which` (indices into the line of `count`) of the
    layered batch: discrete deltas at depth z = L + 2, y at the centre, x
    equally spaced over the inner region.  Returns (len(which), npts)."""
    n0, n1, n2 = prob.n
    L = prob.layer
    xs = np.linspace(L, n0 - 1 - L, count).round().astype(int)
    out = np.zeros((len(which), prob.npts), dtype=np.complex128)
    for k, w in enumerate(which):
        out[k] = delta_source(prob, (int(xs[w]), n1 // 2, L + 2)).ravel()
    return out


def small_problem(n: Tuple[int, ...], layer: int, ppw: float = 10.0,
                  inhomogeneous: bool = False, seed: int = 0, name: str = "small") -> Problem:
    """Small grids for oracle-sized parity runs.  h = 1/(N_max-1)."""
    h = 1.0 / (max(n) - 1)
    c = None
    if inhomogeneous:
        shape = tuple(reversed(n))
        c = grf_speed(shape, max(2.0, min(n) / 6.0), 1.0, 3.0, seed)
    return Problem(name, tuple(n), h, omega_for(ppw, h), layer, c, 1.0)


def lens_problem(dim: int, freq: float, layer: int = 20) -> Problem:
    """Converging-lens model (paper, Section 4.3.1, converging lens models):
    c = 1 - exp(-|x - x0|^2 / (2 sigma^2)) / 2 on the unit square or cube,
    sigma = 1/32, x0 = (0.5, 0.1) in 2D and (0.5, 0.25, 0.5) in 3D, so
    c_min = 1/2; h = 1/(20 freq) gives 10 points per wavelength at c_min.
    The absorbing layer (20 points in the paper) lies outside the unit domain:
    node i sits at x = (i - layer) h, so each axis has 20 freq + 1 + 2 layer
    nodes.  omega = 2 pi freq; the paper's t = 0.1/freq^2 and s = 1/freq equal
    this module's defaults 40 h^2 and 1/freq."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    m = int(round(20 * freq))
    h = 1.0 / m
    n = m + 1 + 2 * layer
    x0 = (0.5, 0.1) if dim == 2 else (0.5, 0.25, 0.5)
    sigma = 1.0 / 32.0
    coords = (np.arange(n) - layer) * h
    shape = (n,) * dim
    grids = np.meshgrid(*([coords] * dim), indexing="ij")  # (z,) y, x order
    r2 = np.zeros(shape)
    for g, c0 in zip(grids, reversed(x0)):
        r2 = r2 + (g - c0) ** 2
    c = 1.0 - 0.5 * np.exp(-r2 / (2.0 * sigma * sigma))
    name = f"lens-{dim}d-{n}"
    return Problem(name, (n,) * dim, h, 2.0 * math.pi * freq, layer, c)


def lens_source(prob: Problem) -> np.ndarray:
    """Discrete delta at the centre of the unit domain (the lens models' source)."""
    m = prob.n[0] - 1 - 2 * prob.layer
    centre = tuple(prob.layer + m // 2 for _ in prob.n)
    return delta_source(prob, centre)


def homog_problem(dim: int, freq: float) -> Problem:
    """Homogeneous model of the paper's 2D and 3D homogeneous experiments
    (Sections 5.1 and 5.2): c = 1 on the unit square or cube, 10 points per
    wavelength (h = 1/(10 freq)), and one wavelength (10 points) of absorbing
    layer outside the unit domain, so each axis has 10 freq + 21 nodes."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    m = int(round(10 * freq))
    layer = 10
    n = m + 1 + 2 * layer
    return Problem(f"homog-{dim}d-{n}", (n,) * dim, 1.0 / m, 2.0 * math.pi * freq, layer, None, 1.0)


def dipole_source(prob: Problem) -> np.ndarray:
    """The homogeneous experiments' source: pairs of normalised Gaussians
    (standard deviation 3h) at the unit domain's centre -+ 6h, the lower one
    negative; along x in 2D (Section 4.1), along each axis in 3D (Section
    4.2).  Coordinates of the unit domain start at the inner edge of the
    absorbing layer."""
    h, L = prob.h, prob.layer
    centre = 0.5 + L * h  # the unit domain's centre in grid coordinates
    f = np.zeros(prob.shape, dtype=np.complex128)
    for axis in range(1 if prob.dim == 2 else 3):
        for sign in (-1.0, 1.0):
            c = [centre] * prob.dim
            c[axis] = centre + sign * 6.0 * h
            f += sign * gaussian_source(prob, tuple(c), 3.0 * h)
    return f
