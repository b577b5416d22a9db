"""Seeded synthetic inputs: Gaussian-well potentials on a periodic grid and random
initial orbital blocks.

This module holds no arithmetic of the orbital minimization method.  It only
draws the data that both the GPU library and the CPU oracle consume, so that the
two sides see bit-identical inputs.

Conventions (shared by every consumer):
  * domain [0, 2*pi)^dim, m points per axis, x_j = 2*pi*j/m;
  * flat grid index j = j1 + m*j2 (+ m*m*j3), i.e. j1 is the fastest axis;
  * orbital blocks are column-major n x N complex128 arrays (leading dim n).

The paper's tests use lattices of Gaussian wells with vacancies (Section 4,
Tests 1-3) but never gives the well's formula.  Here a well of depth d, width w
centred at c is  -d * sum_{s in {-1,0,1}^dim} exp(-|x - c - 2*pi*s|^2 / (2 w^2)),
i.e. a negative Gaussian with standard deviation w, summed over the nearest
periodic images.
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclasses.dataclass(frozen=True)
class Wells:
    """Gaussian wells: centers (k, dim), depths (k,), widths (k,)."""

    centers: np.ndarray
    depths: np.ndarray
    widths: np.ndarray


@dataclasses.dataclass
class Instance:
    """One eigenspace problem: grid, potential, orbital count and initial block."""

    name: str
    dim: int
    m: int
    N: int
    V: np.ndarray        # (n,) float64, flat grid order
    X0: np.ndarray       # (n, N) complex128, Fortran (column-major) order
    seed: int
    wells: Wells

    @property
    def n(self) -> int:
        return self.m ** self.dim


def grid_points(dim: int, m: int) -> np.ndarray:
    """Grid coordinates, shape (n, dim), flat order j = j1 + m*j2 (+ m^2*j3)."""
    axis = TWO_PI * np.arange(m) / m
    mesh = np.meshgrid(*([axis] * dim), indexing="ij")
    # meshgrid(indexing='ij') gives arrays indexed [j1, j2, (j3)]; flatten with
    # j1 fastest by transposing to [.., j2, j1] before a C-order ravel.
    cols = [g.transpose(tuple(range(dim))[::-1]).ravel() for g in mesh]
    return np.stack(cols, axis=1)


def well_potential(dim: int, m: int, wells: Wells) -> np.ndarray:
    """Evaluate the periodic Gaussian-well potential on the grid (float64)."""
    x = grid_points(dim, m)
    V = np.zeros(x.shape[0])
    shifts = np.array(list(itertools.product((-1, 0, 1), repeat=dim)), dtype=float)
    for c, d, w in zip(wells.centers, wells.depths, wells.widths):
        for s in shifts:
            r2 = np.sum((x - c - TWO_PI * s) ** 2, axis=1)
            V -= d * np.exp(-r2 / (2.0 * w * w))
    return V


def complex_gaussian_block(rng: np.random.Generator, n: int, N: int) -> np.ndarray:
    """Entries (a + i b)/sqrt(2n), a, b ~ N(0,1); so E[X^* X] = I."""
    a = rng.standard_normal((n, N))
    b = rng.standard_normal((n, N))
    return np.asfortranarray((a + 1j * b) / np.sqrt(2.0 * n))


def gaussian_test_block(n: int, cols: int, seed: int) -> np.ndarray:
    """Real standard-normal n x cols block from its own seeded generator (the random block of
    the randomized low-rank factorization, an input to both sides)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, cols)))


def random_wells(rng: np.random.Generator, dim: int, count: int,
                 depth=(5.0, 10.0), width=(0.3, 0.6)) -> Wells:
    """Uniformly placed wells; draw order: centers, depths, widths."""
    centers = rng.uniform(0.0, TWO_PI, size=(count, dim))
    depths = rng.uniform(*depth, size=count)
    widths = rng.uniform(*width, size=count)
    return Wells(centers, depths, widths)


def lattice_wells(rng: np.random.Generator, dim: int, cells: int, depth: float,
                  width: float, jitter: float = 0.1, depth_jitter: float = 0.1) -> Wells:
    """cells^dim jittered lattice.  Draw order: centre jitters, then depth jitters.

    Centre of cell i along an axis: (i + 1/2)*h + U(-jitter, jitter)*h, h = 2*pi/cells.
    Depth: depth * (1 + U(-depth_jitter, depth_jitter)).
    """
    h = TWO_PI / cells
    idx = np.array(list(itertools.product(range(cells), repeat=dim)), dtype=float)
    idx = idx[:, ::-1]  # axis 0 fastest, matching the grid ordering
    centers = (idx + 0.5) * h + rng.uniform(-jitter, jitter, size=idx.shape) * h
    depths = depth * (1.0 + rng.uniform(-depth_jitter, depth_jitter, size=idx.shape[0]))
    widths = np.full(idx.shape[0], width)
    return Wells(centers, depths, widths)


def make_instance(name: str, dim: int, m: int, N: int, wells: Wells,
                  rng: np.random.Generator, seed: int) -> Instance:
    V = well_potential(dim, m, wells)
    X0 = complex_gaussian_block(rng, m ** dim, N)
    return Instance(name, dim, m, N, V, X0, seed, wells)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

SEED_SMALL = 1603
SEED_LATTICE2D = 1604
SEED_LATTICE3D = 1605
SEED_BATCH = 1606


def small_2d(seed: int = SEED_SMALL, m: int = 32, N: int = 8) -> Instance:
    """2D 32x32 grid (n = 1024), N = 8, four random wells depth U(5,10), width U(0.3,0.6)."""
    rng = np.random.default_rng(seed)
    wells = random_wells(rng, 2, 4)
    return make_instance("well4_2d_m%d_N%d" % (m, N), 2, m, N, wells, rng, seed)


def lattice_2d(seed: int = SEED_LATTICE2D, m: int = 128, N: int = 64) -> Instance:
    """2D 128x128 grid (n = 16384), N = 64, 8x8 jittered lattice, depth 8, width 0.4."""
    rng = np.random.default_rng(seed)
    wells = lattice_wells(rng, 2, 8, depth=8.0, width=0.4)
    return make_instance("lattice8_2d_m%d_N%d" % (m, N), 2, m, N, wells, rng, seed)


def lattice_3d(seed: int = SEED_LATTICE3D, m: int = 64, N: int = 256) -> Instance:
    """3D 64^3 grid (n = 262144), N = 256, 4x4x4 jittered lattice, depth 6, width 0.5."""
    rng = np.random.default_rng(seed)
    wells = lattice_wells(rng, 3, 4, depth=6.0, width=0.5)
    return make_instance("lattice4_3d_m%d_N%d" % (m, N), 3, m, N, wells, rng, seed)


def random_2d(seed: int, sides=(32, 48, 64, 96, 128), N_range=(8, 64),
              wells_range=(2, 16)) -> Instance:
    """One instance of the many-instance batch: side, N and well count drawn from seed."""
    rng = np.random.default_rng(seed)
    m = int(rng.choice(sides))
    N = int(rng.integers(N_range[0], N_range[1] + 1))
    count = int(rng.integers(wells_range[0], wells_range[1] + 1))
    wells = random_wells(rng, 2, count)
    return make_instance("rand2d_m%d_N%d_s%d" % (m, N, seed), 2, m, N, wells, rng, seed)
