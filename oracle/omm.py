"""Orbital minimization: energy, gradient, Hessian and Algorithm 1 (oracle side).

Section 1, eq. (omm):       E_omm(X) = 1/2 tr((2I - X*X)(X*HX)).
Section 2.1, gradient:      G(X) = 2HX - X(X*HX) - HX(X*X).
Section 2.3, Hessian:       H(X)Z = 2HZ - Z(X*HX) - X(Z*HX) - X(X*HZ)
                                    - HZ(X*X) - HX(Z*X) - HX(X*Z).
Section 2.1, Algorithm 1:   preconditioned nonlinear CG with Polak-Ribiere beta.

The paper leaves the line search unspecified.  E_omm is a quartic polynomial in
alpha along a direction D, so the line search here is exact: the five
coefficients come from the Gram matrices of [X, D] and [HX, HD] and alpha is
the global minimizer among the real roots of the cubic E'(alpha) = 0.

Two readings of Algorithm 1 are taken:
  * its direction update prints D_m = G_m + beta_m G_{m-1}; the standard
    nonlinear CG update D_m = G_m + beta_m D_{m-1} is used;
  * the matrix inner product in beta is <A, B> = Re tr(A^* B), clipped at 0.

All operators act through a callable `apply_h(X) -> H_sigma X`.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

ApplyH = Callable[[np.ndarray], np.ndarray]


def inner(A: np.ndarray, B: np.ndarray) -> float:
    """Re tr(A^* B)."""
    return float(np.real(np.vdot(A, B)))


def energy(X: np.ndarray, HX: np.ndarray) -> float:
    """E_omm = 1/2 tr((2I - X*X)(X*HX)), eq. (omm)."""
    S = X.conj().T @ X
    A = X.conj().T @ HX
    N = X.shape[1]
    return 0.5 * float(np.real(np.trace((2.0 * np.eye(N) - S) @ A)))


def gradient(X: np.ndarray, HX: np.ndarray) -> np.ndarray:
    """G(X) = 2HX - X(X*HX) - HX(X*X) (Section 2.1)."""
    S = X.conj().T @ X
    A = X.conj().T @ HX
    return 2.0 * HX - X @ A - HX @ S


def hessian_apply(X: np.ndarray, HX: np.ndarray, Z: np.ndarray, HZ: np.ndarray) -> np.ndarray:
    """The seven-term Hessian of E_omm applied to Z (Section 2.3)."""
    XhHX = X.conj().T @ HX
    ZhHX = Z.conj().T @ HX
    XhHZ = X.conj().T @ HZ
    XhX = X.conj().T @ X
    ZhX = Z.conj().T @ X
    XhZ = X.conj().T @ Z
    return (2.0 * HZ - Z @ XhHX - X @ ZhHX - X @ XhHZ
            - HZ @ XhX - HX @ ZhX - HX @ XhZ)


def quartic_coefficients(X, HX, D, HD):
    """c0..c4 of E(alpha) = E_omm(X + alpha D).

    With S(a) = S0 + a S1 + a^2 S2 and A(a) = A0 + a A1 + a^2 A2, where
    S0 = X*X, S1 = X*D + D*X, S2 = D*D, A0 = X*HX, A1 = X*HD + D*HX, A2 = D*HD,
    E(a) = tr A(a) - 1/2 tr(S(a) A(a)); collect powers of a."""
    h = lambda P, Q: P.conj().T @ Q
    S0, S2 = h(X, X), h(D, D)
    S1 = h(X, D) + h(D, X)
    A0, A2 = h(X, HX), h(D, HD)
    A1 = h(X, HD) + h(D, HX)
    tr = lambda M: float(np.real(np.trace(M)))
    c0 = tr(A0) - 0.5 * tr(S0 @ A0)
    c1 = tr(A1) - 0.5 * (tr(S0 @ A1) + tr(S1 @ A0))
    c2 = tr(A2) - 0.5 * (tr(S0 @ A2) + tr(S1 @ A1) + tr(S2 @ A0))
    c3 = -0.5 * (tr(S1 @ A2) + tr(S2 @ A1))
    c4 = -0.5 * tr(S2 @ A2)
    return np.array([c0, c1, c2, c3, c4])


def quartic_value(c, a):
    return c[0] + a * (c[1] + a * (c[2] + a * (c[3] + a * c[4])))


def exact_line_search(c) -> float:
    """Global minimizer of the quartic over real alpha.

    Candidates are the real roots of E'(a) = c1 + 2 c2 a + 3 c3 a^2 + 4 c4 a^3;
    ties go to the smaller |a|.  Requires c4 > 0 (true when H_sigma < 0)."""
    if not (c[4] > 0.0):
        raise FloatingPointError("quartic leading coefficient is not positive: %r" % c[4])
    roots = np.roots([4.0 * c[4], 3.0 * c[3], 2.0 * c[2], c[1]])
    scale = np.max(np.abs(roots)) + 1.0
    real = [float(r.real) for r in roots if abs(r.imag) <= 1e-9 * scale]
    if not real:  # numerical safety: fall back to the root with smallest imaginary part
        real = [float(roots[np.argmin(np.abs(roots.imag))].real)]
    vals = [(quartic_value(c, a), abs(a), a) for a in real]
    vals.sort()
    return vals[0][2]


@dataclasses.dataclass
class OmmResult:
    X: np.ndarray
    HX: np.ndarray
    energy: float
    rel_grad: float
    iters: int
    converged: bool
    history: list
    stop_rule: str = ""


def rel_grad(X, HX) -> float:
    """||G(X)||_F / ||H_sigma X||_F, the convergence measure."""
    return float(np.linalg.norm(gradient(X, HX)) / np.linalg.norm(HX))


def minimize(apply_h: ApplyH, X0: np.ndarray,
             precondition: Optional[Callable[[np.ndarray], np.ndarray]] = None,
             tol: float = 1e-10, maxit: int = 4000, stall: int = 3) -> OmmResult:
    """Algorithm 1: preconditioned nonlinear CG on E_omm with exact line search.

    `precondition(G) -> P G` is the preconditioner P applied to a gradient
    block; None means P = I.  Stopping rules, checked before each
    preconditioner application: rel_grad <= tol ("grad"); the energy changed by
    at most 8 eps |E| in `stall` consecutive iterations ("energy", the paper
    names a tolerance but not the quantity, and a near-projector preconditioner
    leaves a gradient floor); or maxit line searches ("maxit")."""
    P = precondition if precondition is not None else (lambda G: G)
    X = np.array(X0, dtype=complex, order="F")
    HX = apply_h(X)
    history = []
    Gprev = None
    D = None
    flat = 0
    eps = np.finfo(float).eps
    for it in range(maxit + 1):
        grad = gradient(X, HX)
        rg = float(np.linalg.norm(grad) / np.linalg.norm(HX))
        E = energy(X, HX)
        if history and abs(E - history[-1][0]) <= 8.0 * eps * abs(E):
            flat += 1
        else:
            flat = 0
        history.append((E, rg))
        if rg <= tol:
            return OmmResult(X, HX, E, rg, it, True, history, "grad")
        if stall and flat >= stall:
            return OmmResult(X, HX, E, rg, it, True, history, "energy")
        if it == maxit:
            break
        G = -P(grad)                                   # G_m = -P G(X_m)
        if D is None:
            D = G                                      # D_1 = -P G(X_1)
        else:
            beta = inner(G, G - Gprev) / inner(Gprev, Gprev)
            D = G + max(beta, 0.0) * D
        Gprev = G
        HD = apply_h(D)
        c = quartic_coefficients(X, HX, D, HD)
        alpha = exact_line_search(c)
        X = X + alpha * D
        HX = HX + alpha * HD
    return OmmResult(X, HX, history[-1][0], history[-1][1], maxit, False, history, "maxit")
