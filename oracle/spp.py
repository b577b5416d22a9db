"""Sparsifying preconditioner (Section 3.2, eqs. Disc, GLu, QG, P).

For (-Laplacian/2 + V - z) u = b, with l = <V> and the constant-coefficient
Green's function G = (-Laplacian/2 + l - z)^{-1} (applied by FFT), the system is
(I + G(V - l)) u = G b (eq. GLu).  A sparse Q with rows supported on a local
neighbourhood a(j) is chosen so that (QG)(j, a(j)^c) ~= 0; then
Q + QG(V - l) is essentially supported on S = {(j, a(j))}, and P, its
restriction to S (eq. P), is sparse.  The preconditioner returns the solution
of P u = Q(G b), here by a sparse direct LU (the paper uses nested dissection;
any exact sparse factorization gives the same u).

Readings (the paper defers the construction of Q to Ying's work):
  * a(j) is the 3^dim box {j + s : s in {-1,0,1}^dim}, periodic;
  * G is circulant, so every row of Q is the same stencil q; q is the unit
    vector minimizing || q^T G(a, a^c) ||_2, i.e. the eigenvector of the
    smallest eigenvalue of the 3^dim x 3^dim matrix conj(Z Z^*), Z = G(a, a^c),
    with its phase fixed so that q at the centre is real and positive;
  * P(i, i + s) = q_s + t_s (V_{i+s} - l), with t_s = (QG)(0, s).
"""

from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from . import hamiltonian as ham


def stencil_offsets(dim: int) -> np.ndarray:
    """Offsets s in {-1,0,1}^dim, axis 0 fastest, shape (3^dim, dim)."""
    return np.array(list(itertools.product((-1, 0, 1), repeat=dim)))[:, ::-1]


def _flat(dim, m, coords):
    coords = np.mod(coords, m)
    idx = np.zeros(coords.shape[0], dtype=np.int64)
    for a in range(dim - 1, -1, -1):
        idx = idx * m + coords[:, a]
    return idx


def green_kernel(dim: int, m: int, V: np.ndarray, z: complex) -> np.ndarray:
    """g(d) = G(0, d) = G(j, j + d) for the circulant G, flat over displacements d."""
    sym = ham.kinetic_symbol(dim, m) + np.mean(V) - z
    shape = (m,) * dim
    return np.fft.ifftn((1.0 / sym).reshape(shape)).ravel()


def all_coords(dim: int, m: int) -> np.ndarray:
    """Integer coordinates (j1, j2, ...) of every flat grid index, shape (n, dim)."""
    n = m ** dim
    j = np.arange(n)
    return np.stack([(j // m ** a) % m for a in range(dim)], axis=1)


def build_stencil(dim: int, m: int, V: np.ndarray, z: complex):
    """Stencil q and t_s = (QG)(0, s) for s in the 3^dim neighbourhood."""
    g = green_kernel(dim, m, V, z)
    offs = stencil_offsets(dim)
    coords = all_coords(dim, m)
    # displacement d (as a grid point) lies outside a(0) unless it is one of the offsets
    inside = np.zeros(m ** dim, dtype=bool)
    inside[_flat(dim, m, offs)] = True
    outside = np.nonzero(~inside)[0]
    # Z[s, d] = G(s, d) = g(d - s)
    Z = np.empty((offs.shape[0], outside.size), dtype=complex)
    for r, s in enumerate(offs):
        Z[r] = g[_flat(dim, m, coords[outside] - s)]
    Mq = np.conj(Z @ Z.conj().T)
    Mq = 0.5 * (Mq + Mq.conj().T)
    evals, evecs = np.linalg.eigh(Mq)
    q = evecs[:, 0]
    centre = int(np.nonzero(np.all(offs == 0, axis=1))[0][0])
    q = q * (abs(q[centre]) / q[centre])
    # t_s = sum_{s'} q_{s'} G(s', s) = sum_{s'} q_{s'} g(s - s')
    t = np.array([sum(q[r2] * g[_flat(dim, m, (s - offs[r2])[None, :])[0]]
                      for r2 in range(offs.shape[0])) for s in offs])
    return q, t, float(np.sqrt(max(evals[0], 0.0)))


def assemble_p(dim: int, m: int, V: np.ndarray, z: complex):
    """Sparse P (eq. P) as a scipy CSC matrix, plus (q, t)."""
    q, t, _ = build_stencil(dim, m, V, z)
    offs = stencil_offsets(dim)
    n = m ** dim
    coords = all_coords(dim, m)
    l = np.mean(V)
    rows, cols, vals = [], [], []
    for r, s in enumerate(offs):
        jj = _flat(dim, m, coords + s)
        rows.append(np.arange(n))
        cols.append(jj)
        vals.append(q[r] + t[r] * (V[jj] - l))
    P = scipy.sparse.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(n, n))
    return P, q, t


def q_symbol(dim: int, m: int, q: np.ndarray) -> np.ndarray:
    """Fourier multiplier of (Q u)(j) = sum_s q_s u(j + s), flat FFT order."""
    k = ham.frequencies(m)
    grids = np.meshgrid(*([k] * dim), indexing="ij")
    kv = np.stack([g.transpose(tuple(range(dim))[::-1]).ravel() for g in grids], axis=1)
    offs = stencil_offsets(dim)
    phase = np.exp(2j * np.pi * (kv @ offs.T) / m)       # (n, 3^dim)
    return phase @ q


class SparsifyingPreconditioner:
    """u = P^{-1} Q G b for one pole z (setup once, apply many times)."""

    def __init__(self, dim: int, m: int, V: np.ndarray, z: complex):
        self.dim, self.m, self.z = dim, m, z
        self.P, self.q, self.t = assemble_p(dim, m, V, z)
        self.lu = scipy.sparse.linalg.splu(self.P.tocsc())
        sym = ham.kinetic_symbol(dim, m) + np.mean(V) - z
        self.rhs_symbol = q_symbol(dim, m, self.q) / sym      # (Q G) in k-space

    def rhs(self, b: np.ndarray) -> np.ndarray:
        return ham.apply_kinetic_diag(self.dim, self.m, b, self.rhs_symbol)

    def __call__(self, b: np.ndarray) -> np.ndarray:
        return self.lu.solve(self.rhs(b))
