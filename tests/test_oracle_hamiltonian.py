"""Pins for the oracle's Hamiltonian (Section 4.1 discretization)."""

import numpy as np
import pytest

from oracle import hamiltonian as ham
from paper_1603_09724_amd import inputs


@pytest.mark.parametrize("dim,m", [(1, 8), (2, 6), (2, 8), (3, 4)])
def test_kinetic_kron_equals_bruteforce_sum(dim, m):
    """The factorized dense kinetic matrix equals the defining sum over K entry by entry."""
    T = ham.kinetic_dense(dim, m)
    Tb = ham.kinetic_dense_bruteforce(dim, m)
    assert np.max(np.abs(T - Tb)) < 1e-12 * np.max(np.abs(Tb))


@pytest.mark.parametrize("dim,m", [(2, 8), (2, 16), (3, 6)])
def test_free_spectrum_closed_form(dim, m):
    """V = 0: eigenvalues are |k|^2/2 over K (k_i from -m/2 to m/2 - 1)."""
    T = ham.kinetic_dense(dim, m)
    k = np.arange(-m // 2, m // 2)
    grids = np.meshgrid(*([k] * dim), indexing="ij")
    expect = np.sort(0.5 * sum(g.ravel() ** 2 for g in grids))
    got = np.linalg.eigvalsh(T)
    assert np.allclose(got, expect, atol=1e-10 * expect.max())


def test_fft_apply_matches_dense(small_instance):
    """FFT apply of H_sigma equals the dense H_sigma on random complex vectors (16x16 and 32x32)."""
    rng = np.random.default_rng(3)
    for m in (16, 32):
        inst = inputs.small_2d(m=m)
        sigma = 7.25
        H = ham.dense_h(2, m, inst.V, sigma)
        X = rng.standard_normal((m * m, 3)) + 1j * rng.standard_normal((m * m, 3))
        HX = ham.apply_h(2, m, inst.V, X, sigma)
        assert np.max(np.abs(HX - H @ X)) < 1e-12 * np.max(np.abs(H @ X))


def test_fft_apply_3d_matches_dense():
    rng = np.random.default_rng(4)
    wells = inputs.Wells(np.array([[1.0, 2.0, 3.0]]), np.array([5.0]), np.array([0.6]))
    V = inputs.well_potential(3, 6, wells)
    H = ham.dense_h(3, 6, V)
    x = rng.standard_normal(216) + 1j * rng.standard_normal(216)
    assert np.max(np.abs(ham.apply_h(3, 6, V, x) - H @ x)) < 1e-12 * np.max(np.abs(H @ x))


def test_hamiltonian_real_symmetric_and_bounds(small_instance):
    inst = small_instance
    H = ham.dense_h(2, inst.m, inst.V)
    assert np.allclose(H, H.T, atol=0)
    lo, hi = ham.spectral_bounds(2, inst.m, inst.V)
    w = np.linalg.eigvalsh(H)
    assert lo <= w[0] and w[-1] <= hi
    sigma = ham.canonical_shift(2, inst.m, inst.V)
    assert np.max(np.linalg.eigvalsh(H - sigma * np.eye(H.shape[0]))) < 0


def test_potential_is_periodic_and_negative():
    """The generated wells are negative Gaussians with periodic images."""
    wells = inputs.Wells(np.array([[0.0, 0.0]]), np.array([3.0]), np.array([0.4]))
    V = inputs.well_potential(2, 32, wells).reshape(32, 32)      # indexed [j2, j1]
    assert V.max() <= 0.0
    assert abs(V[0, 0] + 3.0) < 1e-6          # centre on a grid point: depth (+ tiny image tails)
    # the well sits on the corner: wrapped neighbours equal the direct ones
    assert abs(V[0, 1] - V[0, 31]) < 1e-14 and abs(V[1, 0] - V[31, 0]) < 1e-14
