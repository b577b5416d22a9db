"""Pins for the oracle's pole expansion, GMRES, sparsifying preconditioner and preconditioned OMM."""

import numpy as np
import pytest
import scipy.linalg

from oracle import gmres as gm, hamiltonian as ham, metrics, omm, poles, precond, spp
from paper_1603_09724_amd import inputs


# ------------------------------------------------------------------ poles

def test_circle_rule_matches_closed_form():
    z, w = poles.circle_poles(-3.0, 2.5, 30)
    lam = np.linspace(-9, 4, 301)
    r = poles.filter_function(lam, z, w)
    assert np.max(np.abs(r - poles.circle_filter_closed_form(lam, -3.0, 2.5, 30))) < 1e-13


@pytest.mark.parametrize("lo,a,b", [(-10.0, -3.0, -2.5), (-8.1, 0.22, 0.34), (-2.0, 5.0, 5.01)])
def test_elliptic_filter_is_step_within_rate(lo, a, b):
    """r(lambda) ~ 1 on [lo, a], ~ 0 on [b, inf), error within a small multiple of exp(-pi K' p/4K)."""
    for p in (16, 30):
        z, w = poles.elliptic_poles(lo, a, b, p)
        rate = poles.elliptic_error_rate(lo, a, b, p)
        occ = poles.filter_function(np.linspace(lo, a, 3001), z, w)
        unocc = poles.filter_function(np.concatenate([np.linspace(b, b + 50, 3001),
                                                      np.geomspace(b + 50, 1e7, 400)]), z, w)
        assert np.max(np.abs(occ - 1)) < 8 * rate + 1e-13
        assert np.max(np.abs(unocc)) < 8 * rate + 1e-13
        assert np.max(np.abs(occ.imag)) < 1e-12            # conjugate-pair symmetry


def test_auto_pole_count_meets_rate():
    """The automatic count is the smallest even p >= 30 whose rate meets the target."""
    for lo, a, b in [(-16.2, -3.029, -2.984), (-8.08, 0.22, 0.34)]:
        p = poles.auto_npoles(lo, a, b, 1e-9)
        assert p % 2 == 0 and p >= 30
        assert poles.elliptic_error_rate(lo, a, b, p) <= 1e-9 or p == 64
        if p > 30:
            assert poles.elliptic_error_rate(lo, a, b, p - 2) > 1e-9


def test_elliptic_poles_conjugate_pairs_and_contour():
    z, w = poles.elliptic_poles(-10.0, -3.0, -2.5, 30)
    # every pole has its conjugate in the set (and the weights pair up the same way)
    dist = np.abs(np.conj(z)[:, None] - z[None, :])
    partner = np.argmin(dist, axis=1)
    assert np.max(dist[np.arange(z.size), partner]) < 1e-12 * np.max(np.abs(z))
    assert np.max(np.abs(np.conj(w) - w[partner])) < 1e-12 * np.max(np.abs(w))
    # the contour crosses the real axis left of lo and inside the gap
    assert np.all(np.abs(z.imag) > 0)
    assert z.real.min() < -10.0 and -3.0 < z.real[np.argmin(np.abs(z.imag))] < -2.5


def test_pole_sum_equals_filter_in_eigenbasis():
    """sum_j w_j (H - z_j)^{-1} b = U r(Lam) U* b with dense direct solves (n = 256)."""
    inst = inputs.small_2d(m=16, N=4)
    H = ham.dense_h(2, 16, inst.V)
    lam, U = np.linalg.eigh(H)
    z, w = poles.elliptic_poles(lam[0] - 0.5, lam[3], lam[4], 30)
    b = inst.X0[:, :2]
    got = precond.exact_pole_sum(H, b, z, w)
    r = poles.filter_function(lam, z, w)
    expect = U @ (r[:, None] * (U.T @ b))
    assert np.linalg.norm(got - expect) < 1e-11 * np.linalg.norm(expect)
    # and it is (nearly) the spectral projector
    proj = U[:, :4] @ (U[:, :4].T @ b)
    assert np.linalg.norm(got - proj) < 1e-9 * np.linalg.norm(b)


# ------------------------------------------------------------------ GMRES

@pytest.mark.parametrize("side", ["right", "left"])
def test_gmres_tight_solve_matches_dense(side):
    inst = inputs.small_2d(m=16, N=4)
    H = ham.dense_h(2, 16, inst.V)
    z = -1.0 + 0.3j
    b = inst.X0[:, 0]
    inv_sym = 1.0 / precond.pp_symbol(2, 16, inst.V, z)
    x, info = gm.gmres(lambda v: H @ v - z * v,
                       lambda v: ham.apply_kinetic_diag(2, 16, v, inv_sym),
                       b, b, rtol=1e-13, restart=30, max_cycles=40, side=side)
    assert info.converged
    xd = np.linalg.solve(H - z * np.eye(256), b)
    assert np.linalg.norm(x - xd) < 1e-10 * np.linalg.norm(xd)


def test_gmres_one_cycle_is_minimal_residual():
    """k steps of GMRES minimize ||b - A(x0 + M^-1 u)|| over u in the Krylov space of A M^-1 and r0."""
    rng = np.random.default_rng(9)
    n = 60
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 8 * np.eye(n)
    Mi = np.diag(1.0 / (np.diag(A) + 0.5))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x0 = rng.standard_normal(n) + 0j
    for k in (1, 3, 7):
        x, info = gm.gmres(lambda v: A @ v, lambda v: Mi @ v, b, x0, rtol=0.0, restart=k, max_cycles=1)
        r0 = b - A @ x0
        K = [r0]
        for _ in range(k - 1):
            K.append(A @ (Mi @ K[-1]))
        K = np.stack(K, axis=1)
        # least squares over u = K c: min ||r0 - A M^-1 K c||
        c, *_ = np.linalg.lstsq(A @ Mi @ K, r0, rcond=None)
        xe = x0 + Mi @ (K @ c)
        assert np.linalg.norm(x - xe) < 1e-9 * np.linalg.norm(xe)


def test_gmres_left_one_cycle_minimizes_preconditioned_residual():
    """Left preconditioning: k steps minimize ||M^-1 (b - A(x0 + u))|| over u in the Krylov
    space of M^-1 A and M^-1 r0; the reported residual is relative to ||M^-1 r0||."""
    rng = np.random.default_rng(10)
    n = 60
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 8 * np.eye(n)
    Mi = np.diag(1.0 / (np.diag(A) + 0.5))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x0 = rng.standard_normal(n) + 0j
    for k in (1, 3, 7):
        x, info = gm.gmres(lambda v: A @ v, lambda v: Mi @ v, b, x0, rtol=0.0, restart=k, max_cycles=1,
                           side="left")
        s0 = Mi @ (b - A @ x0)
        K = [s0]
        for _ in range(k - 1):
            K.append(Mi @ (A @ K[-1]))
        K = np.stack(K, axis=1)
        c, *_ = np.linalg.lstsq(Mi @ A @ K, s0, rcond=None)
        xe = x0 + K @ c
        assert np.linalg.norm(x - xe) < 1e-9 * np.linalg.norm(xe)
        expect = np.linalg.norm(Mi @ (b - A @ xe)) / np.linalg.norm(s0)
        assert abs(info.rel_residual - expect) < 1e-9


# ------------------------------------------------------------------ SPP

@pytest.fixture(scope="module")
def spp16():
    inst = inputs.small_2d(m=16, N=4)
    z = -0.8 + 0.4j
    return inst, z, spp.SparsifyingPreconditioner(2, 16, inst.V, z)


def test_spp_matrix_matches_definition(spp16):
    """P equals Q + QG(V - l) restricted to S, with Q and G built densely from their definitions."""
    inst, z, sp = spp16
    n, m = 256, 16
    offs = spp.stencil_offsets(2)
    coords = spp.all_coords(2, m)
    Q = np.zeros((n, n), dtype=complex)
    for r, s in enumerate(offs):
        Q[np.arange(n), spp._flat(2, m, coords + s)] = sp.q[r]
    l = np.mean(inst.V)
    Gd = np.linalg.inv(ham.kinetic_dense(2, m) + (l - z) * np.eye(n))
    full = Q + Q @ Gd @ np.diag(inst.V - l)
    mask = np.abs(Q) > 0
    Pd = sp.P.toarray()
    assert np.max(np.abs((Pd - full)[mask])) < 1e-12 * np.max(np.abs(full))
    assert np.all(Pd[~mask] == 0)
    # q minimizes the off-support norm of q^T G: compare with the SVD of Z = G(a, a^c)
    inside = np.zeros(n, bool)
    inside[spp._flat(2, m, offs)] = True
    Z = Gd[spp._flat(2, m, offs)][:, ~inside]
    smin = np.linalg.svd(Z.T, compute_uv=False)[-1]
    assert abs(np.linalg.norm(Z.T @ sp.q) - smin) < 1e-10 * smin + 1e-15
    # the rhs Q(G b) equals the dense product
    b = inst.X0[:, 0]
    assert np.linalg.norm(sp.rhs(b) - Q @ Gd @ b) < 1e-12 * np.linalg.norm(Q @ Gd @ b)


def test_spp_stencil_sparsifies_green_function():
    """The 3x3 stencil leaves a small off-support remainder ||q^T G(a, a^c)|| relative to
    the minimal one over unit vectors supported at one point (the centre row of G)."""
    inst = inputs.small_2d()
    z = -1.0 + 0.5j
    q, t, far = spp.build_stencil(2, 32, inst.V, z)
    g = spp.green_kernel(2, 32, inst.V, z)
    offs = spp.stencil_offsets(2)
    inside = np.zeros(1024, bool)
    inside[spp._flat(2, 32, offs)] = True
    single = np.linalg.norm(g[~inside])          # e_0^T G restricted to a^c
    assert far < 0.05 * single


def test_spp_solve_matches_dense_and_preconditions(spp16):
    inst, z, sp = spp16
    b = inst.X0[:, 1]
    u = sp(b)
    Pd = sp.P.toarray()
    assert np.linalg.norm(Pd @ u - sp.rhs(b)) < 1e-12 * np.linalg.norm(sp.rhs(b))
    # as a right preconditioner it makes GMRES converge in a handful of steps
    H = ham.dense_h(2, 16, inst.V)
    x, info = gm.gmres(lambda v: H @ v - z * v, sp, b, b, rtol=1e-8, restart=15, max_cycles=5)
    assert info.converged and info.steps <= 12


# ------------------------------------------------------------------ whole method

@pytest.mark.slow
def test_preconditioned_omm_reaches_eigenspace():
    """Filter + Algorithm 1 with the SPP-Fermi preconditioner on 16x16, N = 4."""
    inst = inputs.small_2d(m=16, N=4)
    V, m, N = inst.V, 16, 4
    lo, hi = ham.spectral_bounds(2, m, V)
    sigma = hi + 1.0
    lam, U = np.linalg.eigh(ham.dense_h(2, m, V))
    z, w = poles.elliptic_poles(lo, lam[N - 1], lam[N], 30)
    S = [spp.SparsifyingPreconditioner(2, m, V, zz) for zz in z]

    def P(G, rtol):
        out = np.zeros(G.shape, complex)
        for zz, ww, sp in zip(z, w, S):
            for c in range(G.shape[1]):
                y, _ = gm.gmres(lambda x: ham.apply_h(2, m, V, x) - zz * x, sp, G[:, c], G[:, c], rtol)
                out[:, c] += ww * y
        return out

    X1 = P(inst.X0, 1e-10)
    res = omm.minimize(lambda X: ham.apply_h(2, m, V, X, sigma), X1, lambda G: P(G, 1e-8),
                       tol=1e-10, maxit=25)
    Estar = 0.5 * np.sum(lam[:N] - sigma)
    assert abs(res.energy - Estar) < 1e-10 * abs(Estar)
    assert metrics.sin_theta_max(res.X, U[:, :N]) < 1e-8
