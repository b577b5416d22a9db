"""Algorithm 2 (Section 3.3, precomputing the preconditioner): a randomized low-rank
representation U U* of the approximate Fermi operator projection.

Test infrastructure: only tests/, the smoke check and the benchmark's CPU baseline use it.

Steps in the paper's order:
  1. the pole set of the contour integral (the same as Algorithm 1's);
  2. a Gaussian random block B (n x (N+k), real) -- drawn by the caller from the seeded
     generator and passed in;
  3. (H - z_j) Y_j = B by GMRES started from B, for every pole j;
  4. Y = sum_j w_j Y_j;
  5. a rank-revealing QR factorization of Y (column-pivoted Householder QR here);
  6. U = the first N columns of the orthogonal factor;
  7. the preconditioner is G -> U (U* G).
"""

from __future__ import annotations

import time

import numpy as np
import scipy.linalg

from . import hamiltonian as ham
from . import omm
from .solve import FermiPreconditioner, SolveOptions, SolveResult


def lowrank_basis(Y: np.ndarray, N: int):
    """Steps 5-6: column-pivoted QR of Y, and its first N orthonormal columns.

    Returns (U, R, piv) with Y[:, piv] = Q R, U = Q[:, :N]."""
    Q, R, piv = scipy.linalg.qr(Y, mode="economic", pivoting=True)
    return Q[:, :N], R, piv


def precompute(P: FermiPreconditioner, B: np.ndarray, N: int, rtol: float) -> np.ndarray:
    """Steps 3-6 for the preconditioner P (steps 1 and its inner solves) and the block B."""
    Y = P(np.asarray(B, dtype=complex), rtol)
    U, _, _ = lowrank_basis(Y, N)
    return U


def apply(U: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Step 7: U (U* G)."""
    return U @ (U.conj().T @ G)


def solve(dim, m, V, X0, B, lo, a, b, sigma=None, opts: SolveOptions | None = None) -> SolveResult:
    """Algorithm 1 with the precomputed preconditioner: U from B, then the filter X1 = U U* X0
    and the preconditioned conjugate gradient iteration with G -> U U* G."""
    opts = opts or SolveOptions()
    if sigma is None:
        sigma = ham.canonical_shift(dim, m, V)
    N = X0.shape[1]
    t0 = time.perf_counter()
    P = FermiPreconditioner(dim, m, V, lo, a, b, opts)
    U = precompute(P, B, N, opts.gmres_rtol)
    t1 = time.perf_counter()
    X1 = apply(U, np.asarray(X0, dtype=complex))
    res = omm.minimize(lambda X: ham.apply_h(dim, m, V, X, sigma), X1, lambda G: apply(U, G),
                       tol=opts.tol, maxit=opts.maxit)
    t2 = time.perf_counter()
    return SolveResult(res.X, res.energy, res.rel_grad, res.iters, res.stop_rule, P.steps,
                       t1 - t0, t2 - t1, sigma, P.z, P.w)
