"""Accuracy metrics against the exact eigenspace.

* energy error against E* = 1/2 sum_{i<=N} lambda_i(H_sigma), the minimum of
  eq. (tracemin) (Section 1);
* sin of the largest principal angle between span(X) and span(U_N), computed
  from the perpendicular part (no sqrt(1 - cos^2) cancellation);
* the paper's distance d(X, X0) of Section 4: entrywise max-norm of the
  difference of orthogonal projectors divided by that of X0's projector.
"""

from __future__ import annotations

import numpy as np


def orthonormalize(X: np.ndarray) -> np.ndarray:
    """Q = X (X*X)^{-1/2}."""
    S = X.conj().T @ X
    w, U = np.linalg.eigh(S)
    return X @ (U @ np.diag(w ** -0.5) @ U.conj().T)


def sin_theta_max(X: np.ndarray, U: np.ndarray) -> float:
    """|| Q - U (U* Q) ||_2 with Q an orthonormal basis of span(X), U orthonormal."""
    Q = orthonormalize(X)
    R = Q - U @ (U.conj().T @ Q)
    return float(np.linalg.norm(R, 2))


def projector_distance(X: np.ndarray, X0: np.ndarray) -> float:
    """d(X, X0) of Section 4 (entrywise l-infinity norms)."""
    def proj(Y):
        S = Y.conj().T @ Y
        return Y @ np.linalg.solve(S, Y.conj().T)
    P0 = proj(X0)
    return float(np.max(np.abs(proj(X) - P0)) / np.max(np.abs(P0)))


def ritz_values(X: np.ndarray, HX: np.ndarray) -> np.ndarray:
    """Eigenvalues of the pencil (X*HX, X*X), ascending."""
    import scipy.linalg
    A = X.conj().T @ HX
    S = X.conj().T @ X
    A = 0.5 * (A + A.conj().T)
    S = 0.5 * (S + S.conj().T)
    return scipy.linalg.eigh(A, S, eigvals_only=True)


def residual_angle_bound(X: np.ndarray, HX: np.ndarray, gap: float) -> float:
    """Davis-Kahan sin-theta bound  ||H Q - Q Theta||_F / gap  for the Ritz basis Q.

    `gap` must be the distance between the Ritz values and the unwanted part of
    the spectrum (for example lambda_{N+1} - max Ritz value)."""
    import scipy.linalg
    A = X.conj().T @ HX
    S = X.conj().T @ X
    A = 0.5 * (A + A.conj().T)
    S = 0.5 * (S + S.conj().T)
    theta, W = scipy.linalg.eigh(A, S)
    Q = X @ W              # W^* S W = I, so Q has orthonormal columns
    HQ = HX @ W
    R = HQ - Q * theta[None, :]
    return float(np.linalg.norm(R) / gap)
