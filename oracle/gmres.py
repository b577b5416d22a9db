"""Restarted GMRES for the rough shifted solves (Section 3.1, eq. lst; Section 4 settings).

The paper solves (H - z_j I) Y = G(X_m) roughly with GMRES (Saad & Schultz 1986)
at relative tolerance 1e-5, restart 15, at most 5 restart cycles, starting from
the right-hand side itself.  It does not state the preconditioning side or the
orthogonalization; the readings taken here:
  * right preconditioning (side="right", the default): solve (A M^{-1}) u = r,
    x = x0 + M^{-1} u, so the residual that is monitored is the true residual
    of A x = b;
  * left preconditioning (side="left"): GMRES on M^{-1} A x = M^{-1} b, the
    monitored quantity is the preconditioned residual M^{-1}(b - A x) relative
    to its value at x0.  For a stiff operator (|k|^2/2 up to the grid's cutoff)
    evaluated in single precision, the true residual carries round-off of size
    eps * ||A|| * ||x|| at high frequencies, which the preconditioner damps;
    the mixed-precision path therefore uses this side;
  * modified Gram-Schmidt Arnoldi, Givens rotations for the least-squares
    problem;
  * the true residual b - A x is recomputed at the start of every cycle; the
    solve stops when ||r|| <= rtol ||b|| (true residual at a restart, or the
    Givens estimate inside a cycle) or after max_cycles cycles.
"""

from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np


@dataclasses.dataclass
class GmresInfo:
    steps: int          # Arnoldi steps taken (operator applications inside cycles)
    cycles: int
    rel_residual: float  # at exit: ||b - A x|| / ||b|| (right), ||M^-1(b - A x)|| / ||M^-1(b - A x0)|| (left)
    converged: bool


def gmres(apply_a: Callable[[np.ndarray], np.ndarray],
          apply_minv: Callable[[np.ndarray], np.ndarray],
          b: np.ndarray, x0: np.ndarray, rtol: float = 1e-5,
          restart: int = 15, max_cycles: int = 5, side: str = "right"):
    if side not in ("right", "left"):
        raise ValueError(side)
    left = side == "left"
    b = np.asarray(b, dtype=complex)
    x = np.array(x0, dtype=complex)
    if np.linalg.norm(b) == 0.0:
        return np.zeros_like(b), GmresInfo(0, 0, 0.0, True)
    steps = 0
    cycles = 0
    bnorm = None     # reference norm: ||b|| (right) or ||M^{-1}(b - A x0)|| (left)
    while True:
        r = b - apply_a(x)
        if left:
            r = apply_minv(r)
        beta = np.linalg.norm(r)
        if bnorm is None:
            bnorm = beta if left else np.linalg.norm(b)
            if bnorm == 0.0:
                return x, GmresInfo(0, 0, 0.0, True)
        if beta <= rtol * bnorm or cycles == max_cycles:
            return x, GmresInfo(steps, cycles, float(beta / bnorm), bool(beta <= rtol * bnorm))
        cycles += 1
        n = b.shape[0]
        Vb = np.zeros((restart + 1, n), dtype=complex)
        Hh = np.zeros((restart + 1, restart), dtype=complex)
        cs = np.zeros(restart, dtype=complex)
        sn = np.zeros(restart, dtype=complex)
        g = np.zeros(restart + 1, dtype=complex)
        g[0] = beta
        Vb[0] = r / beta
        k = 0
        for j in range(restart):
            w = apply_minv(apply_a(Vb[j])) if left else apply_a(apply_minv(Vb[j]))
            steps += 1
            for i in range(j + 1):                      # modified Gram-Schmidt
                Hh[i, j] = np.vdot(Vb[i], w)
                w = w - Hh[i, j] * Vb[i]
            hn = np.linalg.norm(w)
            Hh[j + 1, j] = hn
            if hn > 0.0:
                Vb[j + 1] = w / hn
            for i in range(j):                          # previous rotations
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -np.conj(sn[i]) * Hh[i, j] + np.conj(cs[i]) * Hh[i + 1, j]
                Hh[i, j] = t
            # new rotation zeroing Hh[j+1, j]
            aa, bb = Hh[j, j], Hh[j + 1, j]
            den = np.sqrt(abs(aa) ** 2 + abs(bb) ** 2)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = np.conj(aa) / den, np.conj(bb) / den
            Hh[j, j] = den
            Hh[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            if abs(g[j + 1]) <= rtol * bnorm or hn == 0.0:
                break
        y = np.zeros(k, dtype=complex)                  # back substitution R y = g
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - Hh[i, i + 1:k] @ y[i + 1:k]) / Hh[i, i]
        x = x + (y @ Vb[:k] if left else apply_minv(y @ Vb[:k]))
