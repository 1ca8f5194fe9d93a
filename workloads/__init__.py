"""Seeded synthetic workloads: grids, media, sources, frequency and angle lists.

This module only draws and lays out inputs.  It holds none of the method's
arithmetic (no operator, no Krylov step, no exponential) and is the one piece
shared by the oracle and by the GPU path's tests and benchmark.

The workloads are 3D stand-ins for the random-cylinder waveguide of the
paper's experiments section (random dielectric inclusions, a quadratic
absorbing layer, a plane source near one face, sinusoidal sources over a
narrow frequency band).  Units are dimensionless: one grid step is one length
unit and c = 1 where eps = mu = 1, so omega = 2*pi*0.1 means ten cells per
vacuum wavelength and a period of ten time units.

Layout shared by every consumer: a state vector is six planes
[Hx, Hy, Hz, Ex, Ey, Ez], each an N^3 array in C order [k][j][i] (i fastest),
so n = 6 N^3.  Per-cell material arrays (eps, mu, sigma) are N^3 in the same
order; the cell (i, j, k) owns the three E edges and three H faces with its
own index.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

COMPONENTS = ("Hx", "Hy", "Hz", "Ex", "Ey", "Ez")
EX = 3  # index of the Ex plane inside a state vector


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload.  Ranges are (lo, hi) tuples drawn uniformly."""

    name: str
    N: int
    layer: int                      # absorbing-layer thickness L in cells
    sigma_max: float
    n_spheres: int
    radius: object                  # float, or (lo, hi)
    eps_sphere: object              # float, or (lo, hi)
    src_k: int                      # z-plane of the Ex source
    omegas: tuple                   # angular frequencies
    n_theta: int                    # number of incidence angles (1 -> normal)
    T: Optional[float]              # final time (None: stationary loss only)
    krylov_dim: int
    tol: float
    storage: str                    # "f64" or "f32"
    seed: int
    flux_plane: Optional[int] = None
    n_fd_cells: int = 0

    @property
    def n(self) -> int:
        return 6 * self.N ** 3

    @property
    def n_cols(self) -> int:
        return len(self.omegas) * self.n_theta


def _lin(lo, hi, k):
    return tuple(float(2 * math.pi * x) for x in np.linspace(lo, hi, k))


# The five workloads.  T is counted in periods of the centre frequency 0.1
# (period 10), so 20 periods -> T = 200.
C1 = Workload("c1_16cube_plain", 16, 4, 1.0, 20, 2.0, 2.5, 2,
              (2 * math.pi * 0.1,), 1, 200.0, 30, 1e-10, "f64", 1)
C2 = Workload("c2_128cube_plain", 128, 8, 1.0, 2000, (1.5, 3.0), (2.0, 3.0), 10,
              (2 * math.pi * 0.1,), 1, 500.0, 64, 1e-8, "f64", 2)
C3 = Workload("c3_96cube_batched", 96, 8, 1.0, 844, (1.5, 3.0), (2.0, 3.0), 10,
              _lin(0.08, 0.12, 32), 8, 400.0, 64, 1e-8, "f64", 3)
C4 = Workload("c4_64cube_grad", 64, 4, 1.0, 250, (1.5, 3.0), (2.0, 3.0), 6,
              _lin(0.09, 0.11, 8), 1, None, 64, 1e-13, "f64", 4,
              flux_plane=58, n_fd_cells=20)
C5 = Workload("c5_256cube_fp32", 256, 8, 1.0, 6000, (1.5, 3.0), (2.0, 3.0), 10,
              _lin(0.08, 0.12, 16), 1, 600.0, 48, 2e-6, "f32", 5)

CONFIGS = {"c1": C1, "c2": C2, "c3": C3, "c4": C4, "c5": C5}


def small(N: int, seed: int = 11, n_spheres: int = 3, layer: int = 2,
          omegas: Sequence[float] = (2 * math.pi * 0.1,), n_theta: int = 1,
          T: float = 20.0, sigma_max: float = 1.0, radius=(1.0, 2.0),
          eps_sphere=(2.0, 3.0), src_k: Optional[int] = None,
          krylov_dim: int = 30, tol: float = 1e-10, flux_plane=None,
          n_fd_cells: int = 0) -> Workload:
    """A reduced workload with the same recipe, for tests at small N."""
    if src_k is None:
        src_k = min(layer + 1, N - 1)
    return Workload(f"small_{N}_{seed}", N, layer, sigma_max, n_spheres, radius,
                    eps_sphere, src_k, tuple(float(w) for w in omegas), n_theta,
                    T, krylov_dim, tol, "f64", seed, flux_plane, n_fd_cells)


@dataclasses.dataclass
class Inputs:
    """Materialised inputs of a workload (host arrays, float64)."""

    wl: Workload
    eps: np.ndarray          # (N, N, N)
    mu: np.ndarray           # (N, N, N)
    sigma: np.ndarray        # (N, N, N)
    thetas: np.ndarray       # (n_theta,) radians
    centres: np.ndarray
    radii: np.ndarray
    eps_values: np.ndarray
    fd_cells: np.ndarray     # (n_fd_cells, 3) as (i, j, k)


def _draw(rng, spec, count):
    if isinstance(spec, tuple):
        return rng.uniform(spec[0], spec[1], size=count)
    return np.full(count, float(spec))


def sigma_profile(N: int, L: int, sigma_max: float) -> np.ndarray:
    """Quadratic absorbing layer on all six faces.

    For the cell centre c_d = idx + 1/2 along each axis d, the depth into the
    layer is delta = max_d max(0, L - c_d, c_d - (N - L)), and
    sigma = sigma_max * min(1, (delta / L)^2).
    """
    c = np.arange(N, dtype=np.float64) + 0.5
    d1 = np.maximum(0.0, np.maximum(L - c, c - (N - L)))
    delta = np.maximum(np.maximum(d1[:, None, None], d1[None, :, None]),
                       d1[None, None, :])
    if L == 0:
        return np.zeros((N, N, N))
    return sigma_max * np.minimum(1.0, (delta / L) ** 2)


def generate(wl: Workload) -> Inputs:
    """Draw the medium.  Draw order: centres, radii, eps, angles, FD cells."""
    N, L = wl.N, wl.layer
    rng = np.random.default_rng(wl.seed)
    lo, hi = float(L), float(N - L)
    if hi <= lo:
        lo, hi = 0.0, float(N)
    centres = rng.uniform(lo, hi, size=(wl.n_spheres, 3))
    radii = _draw(rng, wl.radius, wl.n_spheres)
    epsv = _draw(rng, wl.eps_sphere, wl.n_spheres)
    if wl.n_theta > 1:
        thetas = rng.uniform(0.0, math.radians(30.0), size=wl.n_theta)
    else:
        thetas = np.zeros(1)
    fd = np.zeros((0, 3), dtype=np.int64)
    if wl.n_fd_cells:
        kf = wl.flux_plane if wl.flux_plane is not None else N - L
        fi = rng.integers(L, N - L, size=wl.n_fd_cells)
        fj = rng.integers(L, N - L, size=wl.n_fd_cells)
        fk = rng.integers(wl.src_k + 1, kf, size=wl.n_fd_cells)
        fd = np.stack([fi, fj, fk], axis=1)

    eps = np.ones((N, N, N))
    cc = np.arange(N, dtype=np.float64) + 0.5
    for (cx, cy, cz), r, e in zip(centres, radii, epsv):
        i0, i1 = max(0, int(math.floor(cx - r - 1))), min(N, int(math.ceil(cx + r + 1)))
        j0, j1 = max(0, int(math.floor(cy - r - 1))), min(N, int(math.ceil(cy + r + 1)))
        k0, k1 = max(0, int(math.floor(cz - r - 1))), min(N, int(math.ceil(cz + r + 1)))
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        dz = (cc[k0:k1] - cz)[:, None, None] ** 2
        dy = (cc[j0:j1] - cy)[None, :, None] ** 2
        dx = (cc[i0:i1] - cx)[None, None, :] ** 2
        inside = (dx + dy + dz) <= r * r
        blk = eps[k0:k1, j0:j1, i0:i1]
        blk[inside] = np.maximum(blk[inside], e)
    mu = np.ones((N, N, N))
    sigma = sigma_profile(N, L, wl.sigma_max)
    return Inputs(wl, eps, mu, sigma, thetas, centres, radii, epsv, fd)


def source_plane(wl: Workload, omega: float, theta: float) -> np.ndarray:
    """Complex values of the Ex source on plane k = src_k, shape (N, N) as [j][i].

    Normal incidence gives 1 everywhere on the plane; an incidence angle theta
    adds the phase ramp exp(-i * omega * sin(theta) * (i + 1/2)) along x.
    """
    N = wl.N
    x = np.arange(N, dtype=np.float64) + 0.5
    row = np.exp(-1j * omega * math.sin(theta) * x)
    return np.broadcast_to(row[None, :], (N, N)).astype(np.complex128)


def source_vector(wl: Workload, omega: float, theta: float) -> np.ndarray:
    """The full complex source b (length n) for one (omega, theta) column."""
    N = wl.N
    b = np.zeros((6, N, N, N), dtype=np.complex128)
    b[EX, wl.src_k] = source_plane(wl, omega, theta)
    return b.reshape(-1)


def columns(wl: Workload, thetas: np.ndarray):
    """Column order of a batched solve: (omega index, theta index), theta fastest."""
    return [(w, t) for w in range(len(wl.omegas)) for t in range(len(thetas))]


def random_state(n: int, seed: int) -> np.ndarray:
    """A seeded random state vector (standard normal), for operator tests."""
    return np.random.default_rng(seed).standard_normal(n)
