"""Dense FP64 Gauss-Newton oracle (test infrastructure; see ``oracle/__init__``).

Problem statement (Sec. 3, eq. optProb): min_{x,p} f(x, p) s.t. c(x, p) = 0
with as many constraints as states.  Here c is static force balance,
c(x, p) = dPi/dx with Pi(x, p) = sum_e E_e(x, p) - f_ext^T x (for the test-only
nodal-force parameters, Pi also subtracts p^T x).  The objective is the
nonlinear least-squares form of eq. leastSquaresObjective plus a Tikhonov
regulariser (a reading: without it the reduced Hessian is singular whenever
parameters outnumber residuals):

    f = w/2 sum_{i in T} ((x_i - t_i) / ell)^2 + mu/2 |p - p_ref|^2,

so in the notation of eq. reducedGN, A = (w / ell^2) I_T, B = 0, C = mu I.
For rest-position parameters (lengths, like x) the regulariser is measured
in the same normalised units as the misfit, mu/2 |(p - p_ref)/ell|^2, i.e.
C = (mu / ell^2) I (a reading; with mu on raw metres the reduced Hessian of
the small cantilevers has condition numbers near 1e9).

Every vector over states uses the free-DOF layout (free nodes ascending, dim
components each).  Parameters: one log-modulus per element, the rest
positions of the free nodes, or (tests only) one nodal force per free DOF.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem
from sgn_inputs import P_LOGE, P_NODAL_FORCE, P_REST_POS, Problem


# ----------------------------------------------------------------------------- element gather

def _elem_dofs(prob: Problem) -> np.ndarray:
    """[ne, (d+1)d] free-DOF index of every element DOF, -1 for fixed components."""
    fd = prob.free_dof_of_node()
    d = prob.dim
    base = fd[prob.elems]  # [ne, d+1]
    dofs = base[:, :, None] + np.arange(d)[None, None, :]
    dofs[base < 0] = -1
    return dofs.reshape(prob.n_elems, -1)


def full_positions(prob: Problem, x: np.ndarray, base: np.ndarray = None) -> np.ndarray:
    """Node positions [n_nodes, d] from the free-DOF vector x (fixed nodes keep base)."""
    pos = (prob.rest_pos if base is None else base).astype(x.dtype).copy()
    pos[prob.free_nodes] = x.reshape(-1, prob.dim)
    return pos


def rest_positions(prob: Problem, p: np.ndarray) -> np.ndarray:
    if prob.param_kind == P_REST_POS:
        return full_positions(prob, p, prob.rest_pos)
    return prob.rest_pos


def element_moduli(prob: Problem, p: np.ndarray):
    mu0, lam0 = fem.lame(prob.E0, prob.nu)
    ne = prob.n_elems
    if prob.param_kind == P_LOGE:
        s = np.exp(p)
        return mu0 * s, lam0 * s
    return np.full(ne, mu0), np.full(ne, lam0)


def _gather(prob, x, p):
    X = rest_positions(prob, p)
    pos = full_positions(prob, x)
    mu, lam = element_moduli(prob, p)
    return pos[prob.elems], X[prob.elems], mu, lam


def fext_free(prob: Problem) -> np.ndarray:
    return prob.f_ext[prob.free_nodes].reshape(-1)


# ----------------------------------------------------------------------------- physics

def potential(prob: Problem, x: np.ndarray, p: np.ndarray) -> float:
    """Pi(x, p); +inf when any element is inverted (the Newton guard J > 0)."""
    xe, Xe, mu, lam = _gather(prob, x, p)
    Ee = fem.element_energy(xe, Xe, mu, lam)
    if not np.all(np.isfinite(Ee)):
        return np.inf
    f = fext_free(prob)
    if prob.param_kind == P_NODAL_FORCE:
        f = f + p
    return float(np.sum(Ee) - f @ x)


def residual(prob: Problem, x: np.ndarray, p: np.ndarray) -> np.ndarray:
    """c(x, p) = dPi/dx over free DOFs."""
    xe, Xe, mu, lam = _gather(prob, x, p)
    ge = fem.element_gradient(xe, Xe, mu, lam).reshape(prob.n_elems, -1)
    dofs = _elem_dofs(prob)
    c = np.zeros(prob.n_x)
    m = dofs >= 0
    np.add.at(c, dofs[m], ge[m])
    c -= fext_free(prob)
    if prob.param_kind == P_NODAL_FORCE:
        c -= p
    return c


def stiffness(prob: Problem, x: np.ndarray, p: np.ndarray) -> sp.csr_matrix:
    """Kx = dc/dx (sparse, symmetric)."""
    xe, Xe, mu, lam = _gather(prob, x, p)
    He = fem.element_hessian(xe, Xe, mu, lam)
    dofs = _elem_dofs(prob)
    ne, n = dofs.shape
    R = np.broadcast_to(dofs[:, :, None], (ne, n, n))
    Cc = np.broadcast_to(dofs[:, None, :], (ne, n, n))
    m = (R >= 0) & (Cc >= 0)
    return sp.coo_matrix((He[m], (R[m], Cc[m])), shape=(prob.n_x, prob.n_x)).tocsr()


def param_jacobian(prob: Problem, x: np.ndarray, p: np.ndarray) -> sp.csr_matrix:
    """Kp = dc/dp (sparse, n_x x n_p)."""
    dofs = _elem_dofs(prob)
    ne, n = dofs.shape
    if prob.param_kind == P_NODAL_FORCE:
        return -sp.identity(prob.n_x, format="csr")
    xe, Xe, mu, lam = _gather(prob, x, p)
    if prob.param_kind == P_LOGE:
        G = fem.element_dgrad_dlogE(xe, Xe, mu, lam)  # [ne, n]
        R = dofs
        Cc = np.broadcast_to(np.arange(ne)[:, None], (ne, n))
        m = R >= 0
        return sp.coo_matrix((G[m], (R[m], Cc[m])), shape=(prob.n_x, prob.n_p)).tocsr()
    M = fem.element_dgrad_drest(xe, Xe, mu, lam)  # [ne, n, n]; columns = rest DOFs
    R = np.broadcast_to(dofs[:, :, None], (ne, n, n))
    Cc = np.broadcast_to(dofs[:, None, :], (ne, n, n))  # rest DOF of a free node = same index
    m = (R >= 0) & (Cc >= 0)
    return sp.coo_matrix((M[m], (R[m], Cc[m])), shape=(prob.n_x, prob.n_p)).tocsr()


# ----------------------------------------------------------------------------- objective

def reg_weight(prob: Problem) -> float:
    """Diagonal C of the regulariser (mu, or mu / ell^2 for rest-position parameters)."""
    if prob.param_kind == P_REST_POS:
        return prob.reg_mu / prob.length_scale ** 2
    return prob.reg_mu


def objective(prob: Problem, x: np.ndarray, p: np.ndarray) -> float:
    r = (x[prob.target_dof] - prob.target_val) / prob.length_scale
    dp = p - prob.p_ref
    return float(0.5 * prob.target_w * r @ r + 0.5 * reg_weight(prob) * dp @ dp)


def objective_blocks(prob: Problem, x: np.ndarray, p: np.ndarray):
    """(df/dx, df/dp, A, B, C) of the least-squares objective (eq. reducedGN)."""
    ell2 = prob.length_scale ** 2
    fx = np.zeros(prob.n_x)
    fx[prob.target_dof] = prob.target_w * (x[prob.target_dof] - prob.target_val) / ell2
    mu = reg_weight(prob)
    fp = mu * (p - prob.p_ref)
    a = np.zeros(prob.n_x)
    a[prob.target_dof] = prob.target_w / ell2
    A = sp.diags(a, format="csr")
    B = sp.csr_matrix((prob.n_p, prob.n_x))
    C = sp.diags(np.full(prob.n_p, mu), format="csr")
    return fx, fp, A, B, C


# ----------------------------------------------------------------------------- equilibrium

@dataclasses.dataclass
class EqInfo:
    iters: int
    res_norm: float
    converged: bool
    shifts: int
    alphas: list


def _spd_factor(K: np.ndarray):
    """Cholesky of K, retrying with K + tau I (tau0 = 1e-8 max diag, x10) when K is not SPD."""
    tau = 0.0
    shifts = 0
    dmax = float(np.max(np.abs(np.diag(K))))
    while True:
        try:
            return sla.cho_factor(K + tau * np.eye(K.shape[0]), lower=True), shifts
        except np.linalg.LinAlgError:
            tau = 1e-8 * dmax if tau == 0.0 else tau * 10.0
            shifts += 1
            if shifts > 30:
                raise


def equilibrium(prob: Problem, p: np.ndarray, x0: np.ndarray = None, rtol: float = 1e-10,
                max_iter: int = 50, max_halvings: int = 40, dense_limit: int = 30000,
                atol: float = 0.0):
    """Forward Newton solve of c(x, p) = 0 with monotone backtracking on Pi (Sec. 5).

    Step acceptance: no inverted element and
    Pi(x + a dx) <= Pi(x) + 1e-4 a c^T dx + 1e-12 (sum_e |E_e| + |f^T x|), the
    last term absorbing rounding in Pi near convergence.  Stops at
    |c|_2 <= rtol |f_ext|_2 + atol, or when the residual has stalled at its
    rounding floor: below 1e-7 |f_ext|_2 and no longer halving per step.
    """
    x = prob.x_rest() if x0 is None else x0.copy()
    fn = np.linalg.norm(fext_free(prob))
    alphas = []
    shifts = 0
    prev = np.inf
    for it in range(max_iter + 1):
        c = residual(prob, x, p)
        rn = np.linalg.norm(c)
        stalled = it > 0 and rn <= 1e-7 * fn and rn > 0.5 * prev
        prev = rn
        if rn <= rtol * fn + atol or stalled:
            return x, EqInfo(it, rn, True, shifts, alphas)
        if it == max_iter:
            break
        K = stiffness(prob, x, p)
        if prob.n_x <= dense_limit:
            fac, s = _spd_factor(K.toarray())
            shifts += s
            dx = -sla.cho_solve(fac, c)
        else:
            dx = -banded_spd_solve(prob, K, c)
        Pi0 = potential(prob, x, p)
        xe, Xe, mu, lam = _gather(prob, x, p)
        scale = float(np.sum(np.abs(fem.element_energy(xe, Xe, mu, lam))) + abs(fext_free(prob) @ x))
        slope = float(c @ dx)
        a = 1.0
        for _ in range(max_halvings):
            Pi1 = potential(prob, x + a * dx, p)
            if Pi1 <= Pi0 + 1e-4 * a * slope + 1e-12 * scale:
                break
            a *= 0.5
        else:
            break
        alphas.append(a)
        x = x + a * dx
    c = residual(prob, x, p)
    return x, EqInfo(max_iter, np.linalg.norm(c), False, shifts, alphas)


def banded_spd_solve(prob: Problem, K: sp.csr_matrix, rhs: np.ndarray) -> np.ndarray:
    """Solve with LAPACK banded Cholesky in a node order with the longest grid axis slowest."""
    d = prob.dim
    fn = prob.free_nodes
    pos = prob.rest_pos[fn]
    ext = pos.max(0) - pos.min(0)
    axes = np.argsort(ext)  # fastest .. slowest
    key = np.lexsort(tuple(np.round(pos[:, a], 9) for a in axes))
    perm = (key[:, None] * d + np.arange(d)[None, :]).ravel()
    Kp = K[perm][:, perm].tocoo()
    bw = int(np.max(np.abs(Kp.row - Kp.col)))
    n = K.shape[0]
    ab = np.zeros((bw + 1, n))
    m = Kp.row >= Kp.col
    ab[Kp.row[m] - Kp.col[m], Kp.col[m]] = Kp.data[m]
    cb = sla.cholesky_banded(ab, lower=True)
    y = sla.cho_solve_banded((cb, True), rhs[perm])
    out = np.empty_like(y)
    out[perm] = y
    return out


# ----------------------------------------------------------------------------- sensitivities and steps

@dataclasses.dataclass
class Step:
    dx: np.ndarray
    dp: np.ndarray
    dlam: np.ndarray
    grad: np.ndarray
    lam_adj: np.ndarray


def adjoint_gradient(prob, x, p, Kx=None, Kp=None):
    """g = df/dp^T + Kp^T lam, Kx^T lam = -df/dx^T: one linear solve (eq. totalGradient)."""
    Kx = stiffness(prob, x, p) if Kx is None else Kx
    Kp = param_jacobian(prob, x, p) if Kp is None else Kp
    fx, fp, *_ = objective_blocks(prob, x, p)
    fac = sla.cho_factor(Kx.toarray(), lower=True)
    lam = -sla.cho_solve(fac, fx)  # Kx symmetric
    return fp + Kp.T @ lam, lam


def dense_gn_step(prob: Problem, x: np.ndarray, p: np.ndarray) -> Step:
    """The dense Gauss-Newton step (Sec. 3.2) with dx and the multiplier block.

    S = -Kx^-1 Kp (eq. dxdp); g = df/dp^T + S^T df/dx^T (eq. totalGradient);
    H = S^T A S + B S + S^T B^T + C (eq. reducedGN); H dp = -g (eq.
    newtonStep); dx = S dp; Kx^T dlam + B^T dp + A dx = 0 (eq. GNdlambda).
    Every factorisation is a dense Cholesky (Kx and H are SPD).
    """
    Kx = stiffness(prob, x, p).toarray()
    Kp = param_jacobian(prob, x, p).toarray()
    fx, fp, A, B, C = objective_blocks(prob, x, p)
    fac = sla.cho_factor(Kx, lower=True)
    S = -sla.cho_solve(fac, Kp)
    g = fp + S.T @ fx
    Ad = A.toarray()
    Bd = B.toarray()
    H = S.T @ Ad @ S + Bd @ S + S.T @ Bd.T + C.toarray()
    H = 0.5 * (H + H.T)
    dp = -sla.cho_solve(sla.cho_factor(H, lower=True), g)
    dx = S @ dp
    dlam = -sla.cho_solve(fac, Ad @ dx + Bd.T @ dp)
    lam_adj = -sla.cho_solve(fac, fx)
    return Step(dx, dp, dlam, g, lam_adj)


def sgn_matrix_dense(prob: Problem, x: np.ndarray, p: np.ndarray) -> np.ndarray:
    """K_SGN = [[A, B^T, Kx^T], [B, C, Kp^T], [Kx, Kp, 0]] (eq. sparseSystemGN), dense."""
    Kx = stiffness(prob, x, p).toarray()
    Kp = param_jacobian(prob, x, p).toarray()
    _, _, A, B, C = objective_blocks(prob, x, p)
    nx, npar = Kx.shape[0], Kp.shape[1]
    Z = np.zeros((nx, nx))
    return np.block([[A.toarray(), B.toarray().T, Kx.T],
                     [B.toarray(), C.toarray(), Kp.T],
                     [Kx, Kp, Z]])


def sgn_matrix_sparse(prob: Problem, x: np.ndarray, p: np.ndarray) -> sp.csr_matrix:
    """The same K_SGN (eq. sparseSystemGN) from the sparse blocks, for meshes where a dense matrix does
    not fit; every block comes from the oracle's own element derivatives."""
    Kx = stiffness(prob, x, p)
    Kp = param_jacobian(prob, x, p)
    _, _, A, B, C = objective_blocks(prob, x, p)
    return sp.bmat([[A, B.T, Kx.T], [B, C, Kp.T], [Kx, Kp, None]], format="csr")


def equilibrated_residual(K: sp.spmatrix, z: np.ndarray, b: np.ndarray) -> float:
    """|S (b - K z)|_2 / |S b|_2 with S = diag(1 / sqrt(max_j |K_ij|)): the relative residual in the
    one-pass symmetric equilibration the solves are judged in."""
    rowmax = abs(sp.csr_matrix(K)).max(axis=1).toarray().ravel()
    s = 1.0 / np.sqrt(rowmax)
    return float(np.linalg.norm(s * (b - K @ z)) / np.linalg.norm(s * b))


def sgn_dense_solve(prob: Problem, x: np.ndarray, p: np.ndarray, rhs_kind: str = "adjoint"):
    """Solve the saddle-point system directly with dense LU.

    rhs_kind 'adjoint': right-hand side [0; -g; 0] (eq. sparseSystemGN).
    rhs_kind 'kkt': right-hand side [-df/dx^T; -df/dp^T; 0], the KKT form of
    Appendix A with c = 0 and lambda = 0; it yields the same dp and a
    multiplier block shifted by the adjoint multiplier (Appendix A, Theorem 2).
    """
    K = sgn_matrix_dense(prob, x, p)
    nx, npar = prob.n_x, prob.n_p
    fx, fp, *_ = objective_blocks(prob, x, p)
    if rhs_kind == "adjoint":
        g, _ = adjoint_gradient(prob, x, p)
        b = np.concatenate([np.zeros(nx), -g, np.zeros(nx)])
    else:
        b = np.concatenate([-fx, -fp, np.zeros(nx)])
    z = np.linalg.solve(K, b)
    return z[:nx], z[nx:nx + npar], z[nx + npar:], K, b


def sgn_rhs(prob: Problem, x: np.ndarray, p: np.ndarray, rhs_kind: str = "adjoint") -> np.ndarray:
    nx = prob.n_x
    fx, fp, *_ = objective_blocks(prob, x, p)
    if rhs_kind == "adjoint":
        g, _ = adjoint_gradient(prob, x, p)
        return np.concatenate([np.zeros(nx), -g, np.zeros(nx)])
    return np.concatenate([-fx, -fp, np.zeros(nx)])


def reduced_objective(prob: Problem, p: np.ndarray, x0: np.ndarray) -> float:
    x, info = equilibrium(prob, p, x0)
    assert info.converged
    return objective(prob, x, p)


def setup_targets(prob: Problem, rtol: float = 1e-10) -> Problem:
    """Fill target values and the frozen length scale ell (problem set-up, not the method).

    ell = max |x(p0) - X| over free DOFs.  2D: targets are x(p*) on the target
    DOFs.  3D: targets are x(p0) + the seeded noise.
    """
    prob = prob.copy()
    p0 = prob.p_init()
    x0, info = equilibrium(prob, p0, rtol=rtol)
    assert info.converged, info
    prob.length_scale = float(np.max(np.abs(x0 - prob.x_rest())))
    if prob.target_noise is not None:
        prob.target_val = x0[prob.target_dof] + prob.target_noise
    else:
        ps = prob.p_star if prob.p_star is not None else p0
        xs, info = equilibrium(prob, ps, x0, rtol=rtol)
        assert info.converged, info
        prob.target_val = xs[prob.target_dof].copy()
    return prob


def sgn_iterations(prob: Problem, p: np.ndarray, x: np.ndarray, iters: int = 10,
                   c1: float = 1e-4, max_halvings: int = 30):
    """Outer loop (Sec. 3.2): dense GN step, then backtracking with one equilibrium per trial.

    Armijo acceptance f(a) <= f(0) + c1 a g^T dp, halving a (a reading: the
    paper only states that steps are accepted or rejected by the objective).
    When every trial fails while the predicted decrease |g^T dp| is below
    1e-12 |f(0)| the iterate is stationary to working precision (the Armijo
    test compares rounding noise) and the iteration stays put (alpha = 0).
    Returns the trace [(f, |g|, alpha)] and the final (p, x).
    """
    trace = []
    for _ in range(iters):
        st = dense_gn_step(prob, x, p)
        f0 = objective(prob, x, p)
        slope = float(st.grad @ st.dp)
        a = 1.0
        for _ in range(max_halvings):
            pt = p + a * st.dp
            xt, info = equilibrium(prob, pt, x)
            if info.converged:
                f1 = objective(prob, xt, pt)
                if f1 <= f0 + c1 * a * slope:
                    break
            a *= 0.5
        else:
            if abs(slope) > 1e-12 * abs(f0):
                raise RuntimeError("line search failed")
            trace.append((f0, float(np.linalg.norm(st.grad)), 0.0))
            continue
        trace.append((f0, float(np.linalg.norm(st.grad)), a))
        p, x = pt, xt
    return trace, p, x


# ----------------------------------------------------------------------------- variants (Sec. 4)

def block_gn_step(prob: Problem, x: np.ndarray, p: np.ndarray) -> Step:
    """Block Gauss-Newton step (Sec. 4 "Block Solve", Appendix B) for objectives without a direct
    parameter term (B = 0, C = 0) and a square, invertible Kp = dc/dp.

    Block substitution of eq. sparseSystemGN with the adjoint right-hand side [0; -g; 0]:
      Kp^T dlam = -g                   -> dlam = -Kp^-T g  (= -lam_adj, as g = Kp^T lam_adj)
      A dx + Kx^T dlam = 0             -> dx = -A^-1 df/dx^T
      Kx dx + Kp dp = 0                -> dp = -Kp^-1 Kx dx = Kp^-1 Kx A^-1 df/dx^T
    (the appendix's sign; the body of Sec. 4 prints the opposite one).  Dense LU solves with Kp.
    """
    Kx = stiffness(prob, x, p).toarray()
    Kp = param_jacobian(prob, x, p).toarray()
    fx, fp, A, B, C = objective_blocks(prob, x, p)
    if Kp.shape[0] != Kp.shape[1]:
        raise ValueError("block solve needs a square Kp")
    if B.nnz or np.any(C.diagonal() != 0):
        raise ValueError("block solve needs B = 0 and C = 0")
    a = A.diagonal()
    if np.any(a == 0):
        raise ValueError("block solve needs an invertible A (every free DOF a target)")
    dx = -fx / a
    dp = np.linalg.solve(Kp, -(Kx @ dx))
    lam_adj = -np.linalg.solve(Kx.T, fx)
    g = fp + Kp.T @ lam_adj
    dlam = -np.linalg.solve(Kp.T, g)
    return Step(dx, dp, dlam, g, lam_adj)


def dense_gn_hessian(prob: Problem, x: np.ndarray, p: np.ndarray):
    """(H, g): the reduced Gauss-Newton Hessian H = S^T A S + B S + S^T B^T + C (eq. reducedGN) and the
    gradient g = df/dp^T + S^T df/dx^T (eq. totalGradient), dense."""
    Kx = stiffness(prob, x, p).toarray()
    Kp = param_jacobian(prob, x, p).toarray()
    fx, fp, A, B, C = objective_blocks(prob, x, p)
    S = -sla.cho_solve(sla.cho_factor(Kx, lower=True), Kp)
    g = fp + S.T @ fx
    Bd = B.toarray()
    H = S.T @ (A.diagonal()[:, None] * S) + Bd @ S + S.T @ Bd.T + C.toarray()
    return 0.5 * (H + H.T), g


def lbfgs_direction(g: np.ndarray, pairs, h0_solve) -> np.ndarray:
    """-H_k g by the L-BFGS two-loop recursion (Nocedal & Wright, Algorithm 7.4) over the curvature
    pairs [(s_i, y_i)] (oldest first) with the initial inverse Hessian applied by h0_solve (for the
    SGN-initialised form: the inverse Gauss-Newton Hessian of the current iterate, Sec. 4
    "Combination with L-BFGS")."""
    q = g.copy()
    alphas = []
    for s, y in reversed(pairs):
        a = (s @ q) / (y @ s)
        alphas.append(a)
        q = q - a * y
    r = h0_solve(q)
    for (s, y), a in zip(pairs, reversed(alphas)):
        b = (y @ r) / (y @ s)
        r = r + s * (a - b)
    return -r


def lbfgs_sgn_iterations(prob: Problem, p: np.ndarray, x: np.ndarray, iters: int = 10, m: int = 5,
                         c1: float = 1e-4, max_halvings: int = 30, curvature_eps: float = 1e-12):
    """L-BFGS whose initial inverse Hessian is the Gauss-Newton one of the current iterate (Sec. 4,
    "Combination with L-BFGS": one saddle-point solve per search direction), with the outer loop's
    Armijo backtracking (one equilibrium per trial).  A pair (s, y) = (p+ - p, g+ - g) enters the
    memory of the newest m pairs only when s^T y > curvature_eps |s| |y| (a reading: the paper gives
    no memory size or curvature rule).  Returns the trace [(f, |g|, alpha)] and the final (p, x)."""
    pairs = []
    prev = None
    trace = []
    for _ in range(iters):
        H, g = dense_gn_hessian(prob, x, p)
        if prev is not None:
            s, y = p - prev[0], g - prev[1]
            if m > 0 and s @ y > curvature_eps * np.linalg.norm(s) * np.linalg.norm(y):
                pairs = (pairs + [(s, y)])[-m:]
        fac = sla.cho_factor(H, lower=True)
        d = lbfgs_direction(g, pairs, lambda q: sla.cho_solve(fac, q))
        f0 = objective(prob, x, p)
        slope = float(g @ d)
        a = 1.0
        for _ in range(max_halvings):
            pt = p + a * d
            xt, info = equilibrium(prob, pt, x)
            if info.converged and objective(prob, xt, pt) <= f0 + c1 * a * slope:
                break
            a *= 0.5
        else:
            if abs(slope) > 1e-12 * abs(f0):
                raise RuntimeError("line search failed")
            trace.append((f0, float(np.linalg.norm(g)), 0.0))
            prev = (p, g)
            continue
        trace.append((f0, float(np.linalg.norm(g)), a))
        prev = (p, g)
        p, x = pt, xt
    return trace, p, x


def equilibrated_residual_extended(K: sp.spmatrix, z: np.ndarray, b: np.ndarray) -> float:
    """equilibrated_residual with b - K z accumulated in extended precision (np.longdouble): the residual
    of z itself, free of the FP64 rounding of its evaluation."""
    K = sp.csr_matrix(K)
    r = b.astype(np.longdouble) - np.add.reduceat(K.data.astype(np.longdouble) * z.astype(np.longdouble)[K.indices],
                                                  K.indptr[:-1])
    rowmax = abs(K).max(axis=1).toarray().ravel()
    s = 1.0 / np.sqrt(rowmax)
    return float(np.linalg.norm(s * r.astype(np.float64)) / np.linalg.norm(s * b))


def refine_extended(K: sp.spmatrix, b: np.ndarray, z0: np.ndarray, sweeps: int = 3):
    """Iterative refinement with residuals in extended precision (Wilkinson; np.longdouble, 64-bit
    mantissa on x86): z <- z + M^-1 (b - K z) with M^-1 a sparse LU (SuperLU) of the symmetrically
    equilibrated K in FP64 and the residual b - K z accumulated in extended precision, so the
    iteration converges (when cond(K) u_64 < 1) to the exact solution within u_64 + cond(K) u_ext in
    the forward error, not merely to a small residual.  Returns (z, [equilibrated residual before and
    after every sweep])."""
    import scipy.sparse.linalg as spla
    K = sp.csr_matrix(K)
    rowmax = abs(K).max(axis=1).toarray().ravel()
    s = 1.0 / np.sqrt(rowmax)
    lu = spla.splu((sp.diags(s) @ K @ sp.diags(s)).tocsc())
    data = K.data.astype(np.longdouble)
    bl = b.astype(np.longdouble)

    def residual(z):
        prod = data * z.astype(np.longdouble)[K.indices]
        return bl - np.add.reduceat(prod, K.indptr[:-1])

    z = z0.copy()
    hist = [equilibrated_residual(K, z, b)]
    for _ in range(sweeps):
        r = residual(z).astype(np.float64)
        z = z + s * lu.solve(s * r)
        hist.append(equilibrated_residual(K, z, b))
    return z, hist


def polish_sgn_solution(prob: Problem, x: np.ndarray, p: np.ndarray, z0: np.ndarray, b: np.ndarray,
                        sweeps: int = 3):
    """The solution of eq. sparseSystemGN refined from z0 (e.g. the dense Gauss-Newton step, the same
    solution by Theorem 1) with extended-precision residuals (refine_extended).  The dense step forms
    H = S^T A S + C explicitly and rounds at the level of cond(Kx) u in S (at the 40 x 10 x 10 size
    its equilibrated residual in the saddle-point system is about 3e-11); the refined one is the
    saddle-point solution to FP64 accuracy."""
    return refine_extended(sgn_matrix_sparse(prob, x, p), b, z0, sweeps)
