"""Reference preconditioned OMM solve: filter, then Algorithm 1 (Sections 3-4).

Section 4: the contour is built from exact spectral information, the initial
guess is filtered by the preconditioner before the conjugate gradient
iteration, 30 poles are used, and each resolvent is applied by rough GMRES.
Here the inner preconditioner is the sparsifying preconditioner of Section 3.2
("spp") or the inverse shifted Laplacian ("pp").
"""

from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import gmres as gm
from . import hamiltonian as ham
from . import omm, poles, precond, spp


@dataclasses.dataclass
class SolveOptions:
    npoles: int = 30
    inner: str = "spp"
    gmres_rtol: float = 1e-8
    filter_rtol: float = 1e-10
    restart: int = 15
    cycles: int = 5
    side: str = "right"      # GMRES preconditioning side
    tol: float = 1e-10
    maxit: int = 4000


@dataclasses.dataclass
class SolveResult:
    X: np.ndarray
    energy: float
    rel_grad: float
    iters: int
    stop_rule: str
    gmres_steps: int
    setup_seconds: float
    solve_seconds: float
    sigma: float
    poles: np.ndarray
    weights: np.ndarray


class FermiPreconditioner:
    """Pole set plus one inner preconditioner per pole; apply(G, rtol) = sum_j w_j Y_j."""

    def __init__(self, dim, m, V, lo, a, b, opts: SolveOptions):
        self.dim, self.m, self.V, self.opts = dim, m, V, opts
        p = opts.npoles if opts.npoles else poles.auto_npoles(lo, a, b)
        self.z, self.w = poles.elliptic_poles(lo, a, b, p)
        if opts.inner == "spp":
            self.inner = [spp.SparsifyingPreconditioner(dim, m, V, zz) for zz in self.z]
        elif opts.inner == "pp":
            self.inner = []
            for zz in self.z:
                inv = 1.0 / precond.pp_symbol(dim, m, V, zz)
                self.inner.append(lambda v, inv=inv: ham.apply_kinetic_diag(dim, m, v, inv))
        else:
            raise ValueError(opts.inner)
        self.steps = 0

    def __call__(self, G: np.ndarray, rtol: float) -> np.ndarray:
        out = np.zeros(G.shape, dtype=complex)
        for zz, ww, minv in zip(self.z, self.w, self.inner):
            apply_a = lambda x, zz=zz: ham.apply_h(self.dim, self.m, self.V, x) - zz * x
            for c in range(G.shape[1]):
                y, info = gm.gmres(apply_a, minv, G[:, c], G[:, c], rtol,
                                   self.opts.restart, self.opts.cycles, self.opts.side)
                self.steps += info.steps
                out[:, c] += ww * y
        return out


def solve(dim, m, V, X0, lo, a, b, sigma=None, opts: SolveOptions | None = None) -> SolveResult:
    """Filter X0, then minimize E_omm for H_sigma with the Fermi-pole preconditioner."""
    opts = opts or SolveOptions()
    if sigma is None:
        sigma = ham.canonical_shift(dim, m, V)
    t0 = time.perf_counter()
    P = FermiPreconditioner(dim, m, V, lo, a, b, opts)
    t1 = time.perf_counter()
    X1 = P(np.asarray(X0, dtype=complex), opts.filter_rtol)
    res = omm.minimize(lambda X: ham.apply_h(dim, m, V, X, sigma), X1,
                       lambda G: P(G, opts.gmres_rtol), tol=opts.tol, maxit=opts.maxit)
    t2 = time.perf_counter()
    return SolveResult(res.X, res.energy, res.rel_grad, res.iters, res.stop_rule, P.steps,
                       t1 - t0, t2 - t1, sigma, P.z, P.w)
