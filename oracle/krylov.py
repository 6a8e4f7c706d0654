"""Stabilised saddle-point matrix and BiCGSTAB, written out densely (FP64).

Test infrastructure only (see the package header).  Sec. 5 ("Solving the saddle point problem")
describes the paper's robust fall-back for saddle-point systems that the direct solver returns
inaccurately: BiCGSTAB (van der Vorst 1992) preconditioned by the LDL^T of the stabilised matrix,
i.e. K_SGN with eps_x added on the x block and -eps_lambda on the multiplier block of the diagonal
(eps_x = eps_lambda = 1e-6 there).  The iteration converges to the solution of the unstabilised
system, whose plain definition is the dense solve; this module holds the stabilised matrix and the
iteration itself so that its convergence from the stabilised preconditioner can be pinned.

Pins (tests/test_oracle_krylov.py): BiCGSTAB solves random nonsymmetric systems to its tolerance
(against numpy's LU); with the exact inverse as preconditioner it converges in one iteration; on
the SGN system preconditioned by the stabilised matrix it reaches the dense Gauss-Newton step
(Theorem 1 of Appendix A), while the stabilised matrix alone gives a step that differs by the
stabilisation's O(eps) effect.
"""
from __future__ import annotations

import numpy as np

from sgn_inputs import Problem

from . import dense as D


def stabilised_sgn_matrix(prob: Problem, x: np.ndarray, p: np.ndarray, eps_x: float, eps_lambda: float) -> np.ndarray:
    """K_SGN + diag([eps_x 1_{n_x}, 0_{n_p}, -eps_lambda 1_{n_c}]) (Sec. 5), dense."""
    K = D.sgn_matrix_dense(prob, x, p)
    nx, npar = prob.n_x, prob.n_p
    e = np.concatenate([np.full(nx, eps_x), np.zeros(npar), np.full(nx, -eps_lambda)])
    return K + np.diag(e)


def bicgstab(A: np.ndarray, b: np.ndarray, prec, tol: float, maxit: int = 200):
    """Right-preconditioned BiCGSTAB for A x = b from x = 0 (van der Vorst 1992): prec(v) applies the
    inverse of the preconditioner.  Stops when |b - A x|_2 <= tol |b|_2 (recursive residual, checked
    after each half step).  Returns (x, iterations, recursive residual norms)."""
    x = np.zeros_like(b)
    r = b.copy()
    r_shadow = r.copy()
    rho_prev = alpha = omega = 1.0
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    bn = np.linalg.norm(b)
    hist = [np.linalg.norm(r)]
    for it in range(1, maxit + 1):
        rho = r_shadow @ r
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        y = prec(p)
        v = A @ y
        alpha = rho / (r_shadow @ v)
        s = r - alpha * v
        if np.linalg.norm(s) <= tol * bn:
            x = x + alpha * y
            hist.append(np.linalg.norm(s))
            return x, it, hist
        z = prec(s)
        t = A @ z
        omega = (t @ s) / (t @ t)
        x = x + alpha * y + omega * z
        r = s - omega * t
        hist.append(np.linalg.norm(r))
        if hist[-1] <= tol * bn:
            return x, it, hist
        rho_prev = rho
    return x, maxit, hist
