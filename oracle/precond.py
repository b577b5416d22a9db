"""Fermi-pole preconditioner (Section 3.1, eqs. direct and lst; Section 3.2 inner preconditioner).

P G ~= sum_j w_j Y_j, where Y_j is a rough GMRES solution of (H - z_j I) Y_j = G
started from Y_j = G (Section 3.1), column by column.

Inner preconditioner "PP" (Section 3.2, and Test 1 of Section 4): the inverse
shifted Laplacian.  The paper's shift is "a proper shift s"; the reading taken
here is the Green's function G_j = (-Laplacian/2 + l - z_j)^{-1} of the
sparsifying preconditioner's constant part, with l = <V> the spatial average of
V, i.e. the k-space diagonal 1/(|k|^2/2 + l - z_j).

The preconditioner is stated for the unshifted H and unshifted poles z_j; the
same operator in the frame H_sigma = H - sigma I has poles z_j - sigma.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import hamiltonian as ham
from .gmres import gmres


@dataclasses.dataclass
class PrecondStats:
    systems: int = 0
    steps: int = 0
    unconverged: int = 0
    max_rel_residual: float = 0.0


def pp_symbol(dim: int, m: int, V: np.ndarray, z: complex) -> np.ndarray:
    """|k|^2/2 + <V> - z on the FFT-ordered frequency grid."""
    return ham.kinetic_symbol(dim, m) + np.mean(V) - z


def solve_shifted(dim, m, V, z, b, rtol=1e-5, restart=15, cycles=5, inner="pp"):
    """Rough solve of (H - z I) y = b from y0 = b."""
    apply_a = lambda x: ham.apply_h(dim, m, V, x) - z * x
    if inner == "pp":
        inv_sym = 1.0 / pp_symbol(dim, m, V, z)
        apply_minv = lambda v: ham.apply_kinetic_diag(dim, m, v, inv_sym)
    elif inner == "none":
        apply_minv = lambda v: v
    else:
        raise ValueError(inner)
    return gmres(apply_a, apply_minv, b, b, rtol, restart, cycles)


def fermi_precondition(dim, m, V, G, poles, weights, rtol=1e-5, restart=15,
                       cycles=5, inner="pp", stats: PrecondStats | None = None):
    """sum_j w_j (H - z_j)^{-1} G, each resolvent applied by rough GMRES (per column)."""
    G = np.asarray(G, dtype=complex)
    vec = G.ndim == 1
    if vec:
        G = G[:, None]
    out = np.zeros(G.shape, dtype=complex)
    for z, w in zip(poles, weights):
        for c in range(G.shape[1]):
            y, info = solve_shifted(dim, m, V, z, G[:, c], rtol, restart, cycles, inner)
            out[:, c] += w * y
            if stats is not None:
                stats.systems += 1
                stats.steps += info.steps
                stats.unconverged += int(not info.converged)
                stats.max_rel_residual = max(stats.max_rel_residual, info.rel_residual)
    return out[:, 0] if vec else out


def exact_pole_sum(H_dense: np.ndarray, G: np.ndarray, poles, weights) -> np.ndarray:
    """sum_j w_j (H - z_j)^{-1} G with dense direct solves (tiny grids only)."""
    n = H_dense.shape[0]
    out = np.zeros(G.shape, dtype=complex)
    for z, w in zip(poles, weights):
        out += w * np.linalg.solve(H_dense - z * np.eye(n), G)
    return out
