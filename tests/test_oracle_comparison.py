"""Pins for the comparison preconditioners (Section 3.1, eqs. Lap and TPA) and Algorithm 1
with them."""

import numpy as np
import pytest

from oracle import comparison as cmp, hamiltonian as ham, omm, solve as osolve
from paper_1603_09724_amd import inputs


def test_laplace_apply_is_the_dense_shifted_inverse():
    """F^{-1} diag(1/(1 + |k|^2/tau)) F G = (I - Delta/tau)^{-1} G with the dense Laplacian."""
    m, tau = 16, 3.7
    T = ham.kinetic_dense(2, m)                 # -Delta/2, dense
    G = inputs.small_2d(m=m, N=3).X0
    expect = np.linalg.solve(np.eye(m * m) + 2.0 * T / tau, G)
    got = cmp.apply(2, m, cmp.laplace_symbol(2, m, tau), G)
    assert np.linalg.norm(got - expect) < 1e-12 * np.linalg.norm(expect)


def test_tpa_apply_is_the_dense_rational_function():
    """With S = -Delta/tau dense: (27 + 18S + 12S^2 + 8S^3)(27 + 18S + 12S^2 + 8S^3 + 16S^4)^{-1} G."""
    m, tau = 16, 5.1
    S = 2.0 * ham.kinetic_dense(2, m) / tau
    I = np.eye(m * m)
    S2 = S @ S
    S3 = S2 @ S
    num = 27 * I + 18 * S + 12 * S2 + 8 * S3
    den = num + 16 * S3 @ S
    G = inputs.small_2d(m=m, N=3).X0
    expect = num @ np.linalg.solve(den, G)
    got = cmp.apply(2, m, cmp.tpa_symbol(2, m, tau), G)
    assert np.linalg.norm(got - expect) < 1e-10 * np.linalg.norm(expect)


def test_tpa_limits():
    """TPA = 1 - (16/27) s^4 + (32/81) s^5 + O(s^6) near k = 0 and 1/(2s) + O(1/s^2) for large s."""
    tau = 1.0
    k2 = 2.0 * ham.kinetic_symbol(2, 64)
    sym = cmp.tpa_symbol(2, 64, tau)
    s = k2 / tau
    small = (s > 0) & (s <= 4)
    assert sym[0] == 1.0
    big = s >= 1000
    assert np.max(np.abs(2 * s[big] * sym[big] - 1)) < 2e-3
    t = 2.0 * ham.kinetic_symbol(2, 16) / 1e4     # s <= 0.0128
    assert np.max(np.abs(cmp.tpa_symbol(2, 16, 1e4) - (1 - 16 / 27 * t ** 4 + 32 / 81 * t ** 5))) < 5e-12
    assert np.all((sym[small] < 1) & (sym[small] > 0))


def test_tau_rule_is_the_largest_kinetic_energy():
    """For plane waves e^{ik.x} the kinetic energy is |k|^2/2 exactly."""
    m = 16
    x = inputs.grid_points(2, m)
    ks = [(1, 0), (2, 3), (0, 5)]
    U = np.stack([np.exp(1j * (x @ np.array(k, dtype=float))) for k in ks], axis=1)
    assert abs(cmp.tau_rule(2, m, U) - 0.5 * (25)) < 1e-12


def test_tpa_outer_iteration_reaches_the_minimum_slowly():
    """Algorithm 1 with TPA converges to the energy of the N lowest eigenvalues, in many more
    iterations than with the Fermi projection (the paper's contrast)."""
    inst = inputs.small_2d(m=16, N=4)
    H = ham.dense_h(2, 16, inst.V)
    lam, U = np.linalg.eigh(H)
    N = 4
    sigma = ham.canonical_shift(2, 16, inst.V)
    tau = cmp.tau_rule(2, 16, U[:, :N])
    sym = cmp.tpa_symbol(2, 16, tau)
    res = omm.minimize(lambda X: ham.apply_h(2, 16, inst.V, X, sigma), inst.X0,
                       lambda G: cmp.apply(2, 16, sym, G), tol=1e-10, maxit=4000)
    Estar = 0.5 * np.sum(lam[:N] - sigma)
    assert abs(res.energy - Estar) <= 1e-10 * abs(Estar)
    fermi = osolve.solve(2, 16, inst.V, inst.X0, float(inst.V.min()), lam[N - 1], lam[N],
                         opts=osolve.SolveOptions(inner="pp", gmres_rtol=1e-8, filter_rtol=1e-10))
    assert res.iters > 3 * fermi.iters
