"""Pins for the oracle's randomized low-rank preconditioner (Section 3.3, Algorithm 2)."""

import numpy as np
import pytest

from oracle import hamiltonian as ham, lowrank as olr, metrics, poles, precond, solve as osolve
from paper_1603_09724_amd import inputs


def test_basis_is_a_column_pivoted_qr():
    """U has orthonormal columns, the first N pivoted columns of Y lie in its span with an
    upper-triangular factor, and the pivot order makes |R_jj| the largest remaining column
    norm at every step (the rank-revealing property)."""
    rng = np.random.default_rng(5)
    n, c, N = 200, 12, 7
    Y = (rng.standard_normal((n, 9)) + 1j * rng.standard_normal((n, 9))) @ \
        (rng.standard_normal((9, c)) + 1j * rng.standard_normal((9, c)))
    Y *= np.geomspace(1.0, 1e-3, c)[None, :]
    U, R, piv = olr.lowrank_basis(Y, N)
    assert np.linalg.norm(U.conj().T @ U - np.eye(N)) < 1e-13
    assert np.linalg.norm(np.tril(R[:N, :N], -1)) == 0.0
    assert np.linalg.norm(Y[:, piv[:N]] - U @ R[:N, :N]) < 1e-12 * np.linalg.norm(Y)
    d = np.abs(np.diag(R))
    for j in range(c):
        rest = np.linalg.norm(R[j:, j:], axis=0)
        assert d[j] >= rest.max() * (1 - 1e-12)
    assert np.all(np.diff(d) <= 1e-12 * d[0])


def test_basis_spans_the_occupied_space_for_the_exact_pole_sum():
    """With Y the exact pole sum applied to a Gaussian block (dense direct solves), U U* is the
    spectral projector onto the N lowest eigenvectors, up to the filter error."""
    inst = inputs.small_2d(m=16, N=4)
    H = ham.dense_h(2, 16, inst.V)
    lam, Ue = np.linalg.eigh(H)
    N, k = 4, 4
    z, w = poles.elliptic_poles(lam[0] - 0.5, lam[N - 1], lam[N], 30)
    B = inputs.gaussian_test_block(256, N + k, 11)
    Y = precond.exact_pole_sum(H, B.astype(complex), z, w)
    U, _, _ = olr.lowrank_basis(Y, N)
    assert metrics.sin_theta_max(U, Ue[:, :N]) < 1e-8
    G = inst.X0[:, :3]
    assert np.linalg.norm(olr.apply(U, G) - Ue[:, :N] @ (Ue[:, :N].T @ G)) < 1e-8 * np.linalg.norm(G)


def _leak_bound(lam, Ue, N, B, z, w):
    """First-order bound on the angle between span(U) and the occupied space: the filter's
    leak into the unoccupied eigenvectors over the smallest occupied singular value of the
    filtered block (both from eigh)."""
    r = poles.filter_function(lam, z, w)
    C = Ue.T @ B
    occ, unocc = r[:N, None] * C[:N], r[N:, None] * C[N:]
    return np.linalg.norm(unocc, 2) / np.linalg.svd(occ, compute_uv=False)[N - 1]


@pytest.mark.parametrize("npoles", [30, 40])
def test_basis_angle_is_the_filter_leak(npoles):
    """With GMRES converged, U's angle to the occupied space is set by the pole filter's leak
    (within a factor 4 either way of the first-order bound), and falls with more poles."""
    inst = inputs.small_2d()
    n, N = inst.n, inst.N
    H = ham.dense_h(2, inst.m, inst.V)
    lam, Ue = np.linalg.eigh(H)
    lo = float(inst.V.min()) - 0.5
    B = inputs.gaussian_test_block(n, N + 8, 21)
    opts = osolve.SolveOptions(npoles=npoles, gmres_rtol=1e-12, filter_rtol=1e-12)
    P = osolve.FermiPreconditioner(2, inst.m, inst.V, lo, lam[N - 1], lam[N], opts)
    U = olr.precompute(P, B, N, 1e-12)
    bound = _leak_bound(lam, Ue, N, B, P.z, P.w)
    angle = metrics.sin_theta_max(U, Ue[:, :N])
    assert bound / 4 <= angle <= 4 * bound
    assert angle < (1e-6 if npoles == 30 else 1e-9)


def test_lowrank_solve_reaches_the_minimum():
    """Algorithm 1 with the precomputed preconditioner converges to the lowest-N eigenspace's
    energy (eigh's N lowest eigenvalues) to 1e-10.  The preconditioner has rank N, so the
    iterates stay in span(U): the subspace is as accurate as U, whose angle is the pole
    filter's leak (above), not the GMRES tolerance."""
    inst = inputs.small_2d()
    n, N = inst.n, inst.N
    H = ham.dense_h(2, inst.m, inst.V)
    lam, Ue = np.linalg.eigh(H)
    lo = float(inst.V.min()) - 0.5
    B = inputs.gaussian_test_block(n, N + 8, 21)
    opts = osolve.SolveOptions(gmres_rtol=1e-8, filter_rtol=1e-8)
    res = olr.solve(2, inst.m, inst.V, inst.X0, B, lo, lam[N - 1], lam[N], opts=opts)
    Estar = 0.5 * np.sum(lam[:N] - res.sigma)
    assert abs(res.energy - Estar) <= 1e-10 * abs(Estar)
    assert metrics.sin_theta_max(res.X, Ue[:, :N]) <= 4 * _leak_bound(lam, Ue, N, B, res.poles, res.weights)
