"""Sparse Newton with inertia control (test infrastructure; see ``oracle/__init__``).

The full second-order step for log-modulus parameters (Sec. 4, "Generalization to Arbitrary
Objectives", eq. totalHessian, and its Lagrangian form in Appendix A, Theorem 2): with the
adjoint multipliers lam = -Kx^-T df/dx^T the Hessian of the reduced objective f(x(p), p) is the
reduced Hessian of the Lagrangian L = f + lam^T c,

    H = S^T A S + B S + S^T B^T + C,     S = -Kx^-1 Kp,
    A = d2f/dx2 + d2(lam^T c)/dx2,  B = d2f/dp dx + d2(lam^T c)/dp dx,  C = d2f/dp2 + d2(lam^T c)/dp2,

and the saddle-point system of eq. sparseSystemGN with these blocks and the right-hand side
[0; -g; 0] yields the Newton step H dp = -g (Theorem 1).  Unlike Gauss-Newton, H need not be
positive definite.  Sec. 5 tests that with the inertia of the LDL^T factorisation of the
saddle-point matrix -- (n_x + n_p, n_x, 0) exactly when H is positive definite, since the
(x, lambda) part [[A, Kx^T], [Kx, 0]] alone has inertia (n_x, n_x, 0) whenever Kx is
nonsingular (Haynsworth) -- and adds diagonal regularisation until it holds.  The form of the
regularisation is a reading (the paper cites an inertia-correction method without details):
delta on the whole primal block (x and p), which turns H into H + delta (I + S^T S), with the
trial sequence of ``inertia_corrected_step``.

lam^T c is a sum of element terms phi_e(x_e, p_e) = lam_e . g_e(x_e, p_e) with g_e the element
gradient (dc/dx has the element Hessians as blocks, dc/dp_e = dg_e/dp_e).  Its second derivatives
are taken as complex-step derivatives (exact to rounding) of first derivatives that are computed
in forward mode: the directional derivative of g_e along (dx_e, dp_e) follows the closed-form
Piola stress through Jacobi's formula d det F = det F tr(F^-1 dF), d F^-1 = -F^-1 dF F^-1 and
d ln J = dJ / J (``element_gradient_dir``).  Pinned in tests against the complex-step element
Hessians, the symmetry of mixed partials, a difference quotient of those Hessians, and the
reduced Hessian against difference quotients of the adjoint gradient.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import dense as D
from . import fem
from sgn_inputs import P_LOGE, Problem

CS_H = fem.CS_H


# ----------------------------------------------------------------------------- element level

def element_gradient_dir(xe, dxe, Xe, mu, lam, dmu, dlam):
    """(g_e, dg_e): the element gradient (fem.element_gradient) and its directional derivative along
    node displacements dxe [ne, d+1, d] and modulus changes (dmu, dlam) [ne], in forward mode.
    Works for complex inputs (for a complex step on top)."""
    Dminv, V0 = fem.rest_data(Xe)
    F = fem.edge_matrix(xe) @ Dminv
    dF = fem.edge_matrix(dxe) @ Dminv
    Fi = np.linalg.inv(F)
    J = fem._det(F)
    dJ = J * np.einsum("...ij,...ji->...", Fi, dF)         # Jacobi's formula
    lnJ = np.log(J)
    dlnJ = dJ / J
    dFi = -Fi @ dF @ Fi                                     # derivative of the inverse
    FiT = np.swapaxes(Fi, -1, -2)
    dFiT = np.swapaxes(dFi, -1, -2)
    m = mu[:, None, None]
    l = lam[:, None, None]
    P = m * (F - FiT) + (l * lnJ[:, None, None]) * FiT
    dP = (dmu[:, None, None] * (F - FiT) + m * (dF - dFiT)
          + (dlam * lnJ + lam * dlnJ)[:, None, None] * FiT + (l * lnJ[:, None, None]) * dFiT)
    DmiT = np.swapaxes(Dminv, -1, -2)

    def nodes(Pm):
        G = V0[:, None, None] * (Pm @ DmiT)
        Gt = np.swapaxes(G, 1, 2)
        return np.concatenate([-np.sum(Gt, axis=1, keepdims=True), Gt], axis=1)

    return nodes(P), nodes(dP)


def element_lagrangian_hessian(xe, Xe, mu, lam, lam_e):
    """Hessian of phi_e = lam_e . g_e over (x_e, p_e) for log-modulus parameters, [ne, n+1, n+1]
    (n = (d+1) d; last row/column p_e), by complex steps on the forward-mode first derivatives:
      d phi/dx_e = (dg_e/dx_e)^T lam_e = directional derivative of g_e along lam_e (Hessian symmetric),
      d phi/dp_e = lam_e . dg_e/dp_e   (E_e = E0 exp(p_e): both Lame moduli scale with exp(p_e)).
    Both the x-p block from the x rows and the p-x block from the p row are kept (they must agree)."""
    ne, nv, d = xe.shape
    n = nv * d
    lam_e = lam_e.reshape(ne, nv, d)
    zero_x = np.zeros_like(lam_e)
    zero_m = np.zeros(ne)

    def first(xc, sc):
        m, l = mu * sc, lam * sc
        _, gx = element_gradient_dir(xc, lam_e.astype(complex), Xe, m, l, zero_m, zero_m)
        _, gp = element_gradient_dir(xc, zero_x.astype(complex), Xe, m, l, m, l)
        return np.concatenate([gx.reshape(ne, n), np.sum(gp.reshape(ne, n) * lam_e.reshape(ne, n), axis=1)[:, None]],
                              axis=1)

    Hm = np.empty((ne, n + 1, n + 1))
    x0 = xe.astype(complex)
    one = np.ones(ne, dtype=complex)
    for k in range(n):
        xc = x0.copy()
        xc[:, k // d, k % d] += 1j * CS_H
        Hm[:, :, k] = np.imag(first(xc, one)) / CS_H
    Hm[:, :, n] = np.imag(first(x0, np.exp(np.full(ne, 1j * CS_H)))) / CS_H
    return Hm


# ----------------------------------------------------------------------------- global blocks

def adjoint_multipliers(prob: Problem, x: np.ndarray, p: np.ndarray) -> np.ndarray:
    """lam = -Kx^-T df/dx^T (Appendix A, the adjoint variables as Lagrange multipliers)."""
    fx, *_ = D.objective_blocks(prob, x, p)
    Kx = D.stiffness(prob, x, p).toarray()
    return -sla.cho_solve(sla.cho_factor(Kx, lower=True), fx)


def lagrangian_second_derivatives(prob: Problem, x: np.ndarray, p: np.ndarray, lam: np.ndarray):
    """(Axx, Bpx, Cpp): d2(lam^T c)/dx2 [n_x, n_x], d2(lam^T c)/dp dx [n_p, n_x] and d2(lam^T c)/dp2
    [n_p, n_p] (diagonal: p_e enters element e only), sparse, from the element Hessians of phi_e."""
    if prob.param_kind != P_LOGE:
        raise ValueError("the Newton blocks are built for log-modulus parameters")
    xe, Xe, mu, lamL = D._gather(prob, x, p)
    dofs = D._elem_dofs(prob)
    ne, n = dofs.shape
    lam_e = np.where(dofs >= 0, lam[np.maximum(dofs, 0)], 0.0)
    Hm = element_lagrangian_hessian(xe, Xe, mu, lamL, lam_e)
    R = np.broadcast_to(dofs[:, :, None], (ne, n, n))
    Cc = np.broadcast_to(dofs[:, None, :], (ne, n, n))
    m = (R >= 0) & (Cc >= 0)
    Axx = sp.coo_matrix((Hm[:, :n, :n][m], (R[m], Cc[m])), shape=(prob.n_x, prob.n_x)).tocsr()
    E = np.broadcast_to(np.arange(ne)[:, None], (ne, n))
    mb = dofs >= 0
    Bpx = sp.coo_matrix((Hm[:, n, :n][mb], (E[mb], dofs[mb])), shape=(prob.n_p, prob.n_x)).tocsr()
    Cpp = sp.diags(Hm[:, n, n], format="csr")
    return Axx, Bpx, Cpp


def newton_blocks(prob: Problem, x: np.ndarray, p: np.ndarray, lam: np.ndarray = None):
    """(A, B, C, lam) of the Lagrangian Hessian at the adjoint multipliers (Appendix A)."""
    if lam is None:
        lam = adjoint_multipliers(prob, x, p)
    _, _, Af, Bf, Cf = D.objective_blocks(prob, x, p)
    Axx, Bpx, Cpp = lagrangian_second_derivatives(prob, x, p, lam)
    return (Af + Axx).tocsr(), (Bf + Bpx).tocsr(), (Cf + Cpp).tocsr(), lam


def newton_matrix_sparse(prob: Problem, x: np.ndarray, p: np.ndarray, delta: float = 0.0,
                         lam: np.ndarray = None) -> sp.csr_matrix:
    """[[A + delta I, B^T, Kx^T], [B, C + delta I, Kp^T], [Kx, Kp, 0]] with the Newton blocks."""
    A, B, C, _ = newton_blocks(prob, x, p, lam)
    Kx = D.stiffness(prob, x, p)
    Kp = D.param_jacobian(prob, x, p)
    Ix = sp.identity(prob.n_x, format="csr")
    Ip = sp.identity(prob.n_p, format="csr")
    return sp.bmat([[A + delta * Ix, B.T, Kx.T], [B, C + delta * Ip, Kp.T], [Kx, Kp, None]], format="csr")


@dataclasses.dataclass
class NewtonStep:
    dx: np.ndarray
    dp: np.ndarray
    dlam: np.ndarray
    grad: np.ndarray
    lam_adj: np.ndarray
    delta: float
    trials: int          # factorisations the inertia test needed (1 = accepted without regularisation)
    inertia: tuple       # of the accepted matrix


def reduced_newton_hessian(prob: Problem, x: np.ndarray, p: np.ndarray):
    """(H, g, S, lam): H = S^T A S + B S + S^T B^T + C with the Newton blocks (eq. totalHessian in
    its Lagrangian form, Appendix A), g the adjoint gradient, dense."""
    A, B, C, lam = newton_blocks(prob, x, p)
    Kx = D.stiffness(prob, x, p).toarray()
    Kp = D.param_jacobian(prob, x, p).toarray()
    fx, fp, *_ = D.objective_blocks(prob, x, p)
    S = -sla.cho_solve(sla.cho_factor(Kx, lower=True), Kp)
    g = fp + S.T @ fx
    Bd = B.toarray()
    H = S.T @ (A @ S) + Bd @ S + S.T @ Bd.T + C.toarray()
    return 0.5 * (H + H.T), g, S, lam


def saddle_inertia(H: np.ndarray, n_x: int, zero_tol: float = 1e-12):
    """Inertia (positive, negative, zero) of the saddle-point matrix whose reduced Hessian is H:
    (n_x, n_x, 0) from the (x, lambda) part plus the inertia of H (Haynsworth)."""
    ev = np.linalg.eigvalsh(H)
    tol = zero_tol * max(1.0, float(np.max(np.abs(ev))))
    return (n_x + int(np.sum(ev > tol)), n_x + int(np.sum(ev < -tol)), int(np.sum(np.abs(ev) <= tol)))


# inertia correction (a reading; Sec. 5 names the test and a diagonal regularisation only):
# trial 1 without regularisation; then delta = DELTA0 if no earlier step needed one, else
# max(DELTA_MIN, delta_last / 3); grow by 8 per failed trial; give up beyond DELTA_MAX.
DELTA0 = 1e-4
DELTA_MIN = 1e-20
DELTA_MAX = 1e20
DELTA_GROW = 8.0
DELTA_SHRINK = 3.0  # divisor


def delta_trials(delta_last: float):
    """The sequence of regularisations the inertia test tries, in order."""
    yield 0.0
    d = DELTA0 if delta_last <= 0.0 else max(DELTA_MIN, delta_last / DELTA_SHRINK)
    while d <= DELTA_MAX:
        yield d
        d *= DELTA_GROW


def inertia_corrected_step(prob: Problem, x: np.ndarray, p: np.ndarray, delta_last: float = 0.0) -> NewtonStep:
    """The Newton step of the smallest trial delta whose saddle-point matrix has the inertia
    (n_x + n_p, n_x, 0):  (H + delta (I + S^T S)) dp = -g, dx = S dp, and the multiplier block of the
    system with right-hand side [0; -g; 0]: Kx^T dlam = -((A + delta I) dx + B^T dp)."""
    H, g, S, lam = reduced_newton_hessian(prob, x, p)
    A, B, C, _ = newton_blocks(prob, x, p, lam)
    Kx = D.stiffness(prob, x, p).toarray()
    nx, npar = prob.n_x, prob.n_p
    want = (nx + npar, nx, 0)
    StS = S.T @ S
    for trials, delta in enumerate(delta_trials(delta_last), start=1):
        Hd = H + delta * (np.eye(npar) + StS)
        Hd = 0.5 * (Hd + Hd.T)
        ine = saddle_inertia(Hd, nx)
        if ine != want:
            continue
        dp = -sla.cho_solve(sla.cho_factor(Hd, lower=True), g)
        dx = S @ dp
        dlam = -np.linalg.solve(Kx.T, A @ dx + delta * dx + B.T @ dp)
        return NewtonStep(dx, dp, dlam, g, lam, delta, trials, ine)
    raise RuntimeError("no regularisation up to DELTA_MAX gives the inertia of a minimum")


def newton_iterations(prob: Problem, p: np.ndarray, x: np.ndarray, iters: int = 10, c1: float = 1e-4,
                      max_halvings: int = 30):
    """Outer loop with the inertia-corrected Newton step: Armijo backtracking with one equilibrium per
    trial, as the Gauss-Newton loop (``dense.sgn_iterations``), and the last nonzero delta carried to
    the next step's trial sequence.  Returns the trace [(f, |g|, alpha, delta, trials)] and (p, x)."""
    trace = []
    delta_last = 0.0
    for _ in range(iters):
        st = inertia_corrected_step(prob, x, p, delta_last)
        if st.delta > 0.0:
            delta_last = st.delta
        f0 = D.objective(prob, x, p)
        slope = float(st.grad @ st.dp)
        a = 1.0
        for _ in range(max_halvings):
            pt = p + a * st.dp
            xt, info = D.equilibrium(prob, pt, x)
            if info.converged and D.objective(prob, xt, pt) <= f0 + c1 * a * slope:
                break
            a *= 0.5
        else:
            if abs(slope) > 1e-12 * abs(f0):
                raise RuntimeError("line search failed")
            trace.append((f0, float(np.linalg.norm(st.grad)), 0.0, st.delta, st.trials))
            continue
        trace.append((f0, float(np.linalg.norm(st.grad)), a, st.delta, st.trials))
        p, x = pt, xt
    return trace, p, x
