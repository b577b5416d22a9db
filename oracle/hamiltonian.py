"""Planewave (Fourier pseudospectral) Hamiltonian H = -Laplacian/2 + V.

Follows Section 4.1 (discretization of eq. ex1): grid index set J, frequency set
K = {k : -m/2 <= k_i < m/2}, kinetic operator F^{-1} diag(|k|^2 symbol) F and a
potential diagonal in real space.  Here the domain is [0, 2*pi)^dim, so the
kinetic symbol is |k|^2/2 with integer k (the paper's unit box gives 2*pi^2|k|^2,
the same operator after rescaling).  The Nyquist frequency k = -m/2 appears once,
exactly as K is written, which keeps H real symmetric.

Section 1 (after eq. omm): shifting the diagonal by a constant leaves the
eigenspace unchanged, so H_sigma = H - sigma*I with sigma above the spectrum is
negative definite.
"""

from __future__ import annotations

import numpy as np


def frequencies(m: int) -> np.ndarray:
    """Integer frequencies in FFT order: index j -> k = j for j < m/2, else j - m.

    Covers exactly K = {-m/2, ..., m/2 - 1} (Section 4.1)."""
    j = np.arange(m)
    return np.where(j < m // 2, j, j - m)


def kinetic_symbol(dim: int, m: int) -> np.ndarray:
    """|k|^2/2 on the FFT-ordered frequency grid, flat with k1 fastest."""
    k = frequencies(m).astype(float)
    grids = np.meshgrid(*([k] * dim), indexing="ij")       # [k1, k2, (k3)]
    ksq = sum(g * g for g in grids)
    return 0.5 * ksq.transpose(tuple(range(dim))[::-1]).ravel()


def kinetic_1d_dense(m: int) -> np.ndarray:
    """Dense 1D kinetic matrix from its definition:
    T1[j, j'] = (1/m) sum_{k in K} exp(i k (x_j - x_j')) k^2/2,  x_j = 2 pi j/m."""
    k = frequencies(m).astype(float)
    j = np.arange(m)
    dx = 2.0 * np.pi * (j[:, None] - j[None, :]) / m
    T = np.zeros((m, m), dtype=complex)
    for kk in k:
        T += np.exp(1j * kk * dx) * (0.5 * kk * kk)
    T /= m
    assert np.max(np.abs(T.imag)) < 1e-10 * max(1.0, np.max(np.abs(T.real)))
    return T.real


def kinetic_dense(dim: int, m: int) -> np.ndarray:
    """Dense kinetic matrix on the dim-dimensional grid (flat order, j1 fastest).

    The defining sum over K factorizes over axes because |k|^2 = sum_a k_a^2 and
    K is a product set, so T = sum_a I x ... x T1 (axis a) x ... x I."""
    T1 = kinetic_1d_dense(m)
    I = np.eye(m)
    n = m ** dim
    T = np.zeros((n, n))
    for a in range(dim):
        # flat index j = j1 + m j2 + ...: axis 0 is the fastest -> last Kronecker factor
        factors = [I] * dim
        factors[dim - 1 - a] = T1
        term = factors[0]
        for f in factors[1:]:
            term = np.kron(term, f)
        T += term
    return T


def kinetic_dense_bruteforce(dim: int, m: int) -> np.ndarray:
    """The defining d-dimensional sum, evaluated entry by entry (tiny grids only):
    T[j, j'] = (1/n) sum_{k in K} exp(i k.(x_j - x_j')) |k|^2/2."""
    axis = 2.0 * np.pi * np.arange(m) / m
    mesh = np.meshgrid(*([axis] * dim), indexing="ij")
    x = np.stack([g.transpose(tuple(range(dim))[::-1]).ravel() for g in mesh], axis=1)
    k1 = frequencies(m).astype(float)
    ks = np.stack([g.ravel() for g in np.meshgrid(*([k1] * dim), indexing="ij")], axis=1)
    n = m ** dim
    T = np.zeros((n, n), dtype=complex)
    for kv in ks:
        phase = np.exp(1j * (x @ kv))
        T += np.outer(phase, phase.conj()) * (0.5 * kv @ kv)
    T /= n
    return T.real


def dense_h(dim: int, m: int, V: np.ndarray, sigma: float = 0.0) -> np.ndarray:
    """Dense H_sigma = T + diag(V) - sigma I (real symmetric)."""
    H = kinetic_dense(dim, m)
    H[np.diag_indices_from(H)] += V - sigma
    return H


def _grid_shape(dim: int, m: int):
    return (m,) * dim


def apply_h(dim: int, m: int, V: np.ndarray, X: np.ndarray, sigma: float = 0.0) -> np.ndarray:
    """H_sigma X via FFTs: F^{-1}(|k|^2/2 . F X) + (V - sigma) . X, column by column."""
    X = np.asarray(X)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    n, N = X.shape
    sym = kinetic_symbol(dim, m).reshape(_grid_shape(dim, m))
    out = np.empty((n, N), dtype=complex)
    for c in range(N):
        x = X[:, c].reshape(_grid_shape(dim, m))          # indexed [.., j2, j1]
        t = np.fft.ifftn(sym * np.fft.fftn(x))
        out[:, c] = t.ravel() + (V - sigma) * X[:, c]
    return out[:, 0] if vec else out


def apply_kinetic_diag(dim: int, m: int, X: np.ndarray, diag_k: np.ndarray) -> np.ndarray:
    """F^{-1} diag(diag_k) F X column by column (diag_k in FFT order, flat)."""
    X = np.asarray(X)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    shape = _grid_shape(dim, m)
    d = diag_k.reshape(shape)
    out = np.empty(X.shape, dtype=complex)
    for c in range(X.shape[1]):
        out[:, c] = np.fft.ifftn(d * np.fft.fftn(X[:, c].reshape(shape))).ravel()
    return out[:, 0] if vec else out


def kinetic_max(dim: int, m: int) -> float:
    """Largest kinetic eigenvalue: dim * (m/2)^2 / 2 (from k = -m/2 on every axis)."""
    return 0.5 * dim * (m // 2) ** 2


def spectral_bounds(dim: int, m: int, V: np.ndarray):
    """Rigorous bounds lo <= lambda_1 and lambda_n <= hi of the unshifted H.

    T is positive semidefinite, so lambda_1 >= min V; and lambda_max(T + V)
    <= lambda_max(T) + max V."""
    return float(np.min(V)), kinetic_max(dim, m) + float(np.max(V))


def canonical_shift(dim: int, m: int, V: np.ndarray) -> float:
    """sigma = hi + 1, which makes H - sigma I negative definite."""
    return spectral_bounds(dim, m, V)[1] + 1.0


def eigh_dense(dim: int, m: int, V: np.ndarray, sigma: float = 0.0, count: int | None = None):
    """Eigenvalues (ascending) and eigenvectors of the dense H_sigma.

    If count is given only the lowest `count` pairs are returned."""
    import scipy.linalg
    H = dense_h(dim, m, V, sigma)
    if count is None:
        return np.linalg.eigh(H)
    w, U = scipy.linalg.eigh(H, subset_by_index=[0, count - 1], driver="evr")
    return w, U
