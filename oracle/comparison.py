"""The comparison preconditioners of Section 3.1: the inverse shifted Laplacian (eq. Lap) and
the TPA preconditioner (eq. TPA), both diagonal in Fourier space, used as the outer
preconditioner of Algorithm 1 in place of the Fermi projection.

Test infrastructure: only tests/, the smoke check and the benchmark's CPU baseline use it.

With integer frequencies k on [0, 2 pi)^d, -Delta has the symbol |k|^2:
  Lap:  P(k) = 1 / (1 + |k|^2 / tau)
  TPA:  P(k) = q(s) / (q(s) + 16 s^4),  q(s) = 27 + 18 s + 12 s^2 + 8 s^3,  s = |k|^2 / tau.
The scale tau follows Section 4's rule: the largest kinetic energy sum_k |k|^2/2 |x_j(k)|^2
among the occupied eigenvectors x_j (unit norm).
"""

from __future__ import annotations

import numpy as np

from . import hamiltonian as ham


def laplace_symbol(dim: int, m: int, tau: float) -> np.ndarray:
    k2 = 2.0 * ham.kinetic_symbol(dim, m)
    return 1.0 / (1.0 + k2 / tau)


def tpa_symbol(dim: int, m: int, tau: float) -> np.ndarray:
    s = 2.0 * ham.kinetic_symbol(dim, m) / tau
    q = 27.0 + 18.0 * s + 12.0 * s ** 2 + 8.0 * s ** 3
    return q / (q + 16.0 * s ** 4)


def apply(dim: int, m: int, symbol: np.ndarray, G: np.ndarray) -> np.ndarray:
    """F^{-1} diag(symbol) F G, column by column."""
    return ham.apply_kinetic_diag(dim, m, G, symbol)


def tau_rule(dim: int, m: int, U: np.ndarray) -> float:
    """max_j x_j^* T x_j over the columns of U (normalized), T the kinetic operator."""
    U = np.asarray(U, dtype=complex)
    U = U / np.linalg.norm(U, axis=0)[None, :]
    TU = ham.apply_kinetic_diag(dim, m, U, ham.kinetic_symbol(dim, m))
    return float(np.max(np.real(np.sum(U.conj() * TU, axis=0))))
