"""Pins for the oracle's OMM functional, gradient, Hessian, quartic and Algorithm 1."""

import numpy as np
import pytest

from oracle import hamiltonian as ham, metrics, omm
from paper_1603_09724_amd import inputs


@pytest.fixture(scope="module")
def tiny():
    """16x16 grid, N = 4, shifted negative definite; dense spectrum for reference."""
    inst = inputs.small_2d(m=16, N=4)
    sigma = ham.canonical_shift(2, 16, inst.V)
    H = ham.dense_h(2, 16, inst.V, sigma)
    w, U = np.linalg.eigh(H)
    return inst, sigma, H, w, U


def _rand(rng, n, N, scale=1.0):
    return scale * (rng.standard_normal((n, N)) + 1j * rng.standard_normal((n, N)))


def test_energy_at_eigenvectors_is_half_trace(tiny):
    inst, sigma, H, w, U = tiny
    X = U[:, :4].astype(complex)
    assert abs(omm.energy(X, H @ X) - 0.5 * w[:4].sum()) < 1e-12 * abs(w[:4].sum())
    # minimizer property: gradient vanishes there
    assert np.linalg.norm(omm.gradient(X, H @ X)) < 1e-10 * np.linalg.norm(H @ X)


def test_energy_gauge_invariance(tiny):
    inst, sigma, H, w, U = tiny
    rng = np.random.default_rng(1)
    X = _rand(rng, 256, 4, 0.1)
    W, _ = np.linalg.qr(_rand(rng, 4, 4))
    e1 = omm.energy(X, H @ X)
    e2 = omm.energy(X @ W, H @ X @ W)
    assert abs(e1 - e2) < 1e-12 * abs(e1)


def test_energy_closed_form_on_eigen_coordinates(tiny):
    """X = U_N W for any W: E = 1/2 tr((2I - W*W) W* Lam W), evaluated independently."""
    inst, sigma, H, w, U = tiny
    rng = np.random.default_rng(2)
    Wm = _rand(rng, 4, 4, 0.4)
    X = U[:, :4] @ Wm
    L = np.diag(w[:4])
    expect = 0.5 * np.real(np.trace((2 * np.eye(4) - Wm.conj().T @ Wm) @ (Wm.conj().T @ L @ Wm)))
    assert abs(omm.energy(X, H @ X) - expect) < 1e-12 * abs(expect)


def test_gradient_matches_finite_differences(tiny):
    """dE(X + tZ)/dt = Re tr(Z* G(X)) (central differences)."""
    inst, sigma, H, w, U = tiny
    rng = np.random.default_rng(3)
    X = _rand(rng, 256, 4, 0.05)
    for _ in range(3):
        Z = _rand(rng, 256, 4, 0.05)
        h = 1e-5
        fd = (omm.energy(X + h * Z, H @ (X + h * Z)) - omm.energy(X - h * Z, H @ (X - h * Z))) / (2 * h)
        an = omm.inner(Z, omm.gradient(X, H @ X))
        assert abs(fd - an) < 1e-6 * abs(an)


def test_hessian_matches_finite_differences(tiny):
    inst, sigma, H, w, U = tiny
    rng = np.random.default_rng(4)
    X = _rand(rng, 256, 4, 0.05)
    Z = _rand(rng, 256, 4, 0.05)
    h = 1e-5
    gp = omm.gradient(X + h * Z, H @ (X + h * Z))
    gm = omm.gradient(X - h * Z, H @ (X - h * Z))
    fd = (gp - gm) / (2 * h)
    an = omm.hessian_apply(X, H @ X, Z, H @ Z)
    assert np.linalg.norm(fd - an) < 1e-6 * np.linalg.norm(an)


def test_hessian_at_minimizer_reduces_for_perpendicular_directions(tiny):
    """At X0 = U_N with Z*X0 = 0 the Hessian is HZ - Z Lam0 (Section 2.3)."""
    inst, sigma, H, w, U = tiny
    X0 = U[:, :4].astype(complex)
    rng = np.random.default_rng(5)
    Z = _rand(rng, 256, 4)
    Z = Z - X0 @ (X0.conj().T @ Z)
    an = omm.hessian_apply(X0, H @ X0, Z, H @ Z)
    assert np.linalg.norm(an - (H @ Z - Z @ np.diag(w[:4]))) < 1e-10 * np.linalg.norm(an)


def test_quartic_interpolates_energy(tiny):
    inst, sigma, H, w, U = tiny
    rng = np.random.default_rng(6)
    X = _rand(rng, 256, 4, 0.05)
    D = _rand(rng, 256, 4, 0.05)
    c = omm.quartic_coefficients(X, H @ X, D, H @ D)
    for a in (-2.0, -0.3, 0.0, 0.7, 3.1):
        Xa = X + a * D
        e = omm.energy(Xa, H @ Xa)
        assert abs(omm.quartic_value(c, a) - e) < 1e-11 * max(1.0, abs(e))
    # c1 = Re tr(D* G), c2 = 1/2 Re tr(D* Hess D), c4 >= 0 for H_sigma < 0
    assert abs(c[1] - omm.inner(D, omm.gradient(X, H @ X))) < 1e-11 * abs(c[1])
    c2 = 0.5 * omm.inner(D, omm.hessian_apply(X, H @ X, D, H @ D))
    assert abs(c[2] - c2) < 1e-11 * abs(c2)
    assert c[4] > 0


def test_exact_line_search_is_global_minimum(tiny):
    inst, sigma, H, w, U = tiny
    rng = np.random.default_rng(7)
    for _ in range(5):
        X = _rand(rng, 256, 4, 0.05)
        D = _rand(rng, 256, 4, 0.05)
        c = omm.quartic_coefficients(X, H @ X, D, H @ D)
        a = omm.exact_line_search(c)
        grid = np.linspace(a - 5 * (abs(a) + 1), a + 5 * (abs(a) + 1), 20001)
        assert omm.quartic_value(c, a) <= np.min(omm.quartic_value(c, grid)) + 1e-12 * abs(c[0])


def test_unpreconditioned_omm_cg_converges_to_eigenspace(tiny):
    """Algorithm 1 with P = I reaches E* = 1/2 sum lambda_i and X*X -> I (Section 1)."""
    inst, sigma, H, w, U = tiny
    res = omm.minimize(lambda X: H @ X, inst.X0, None, tol=1e-11, maxit=3000, stall=0)
    assert res.converged
    Estar = 0.5 * w[:4].sum()
    assert abs(res.energy - Estar) < 1e-12 * abs(Estar)
    S = res.X.conj().T @ res.X
    assert np.linalg.norm(S - np.eye(4)) < 1e-8
    assert metrics.sin_theta_max(res.X, U[:, :4]) < 1e-7
    # energy is monotone under the exact line search
    energies = [h[0] for h in res.history]
    assert all(e2 <= e1 + 1e-10 * abs(e1) for e1, e2 in zip(energies, energies[1:]))


def test_metrics_known_angle():
    """sin theta of a plane rotated by a known angle; d of identical spaces is 0."""
    n = 50
    U = np.zeros((n, 1))
    U[0, 0] = 1.0
    th = 1e-9
    X = np.zeros((n, 1), dtype=complex)
    X[0, 0] = 3 * np.cos(th)
    X[1, 0] = 3 * np.sin(th)
    assert abs(metrics.sin_theta_max(X, U) - np.sin(th)) < 1e-20
    assert metrics.projector_distance(U.astype(complex), U.astype(complex)) == 0.0
