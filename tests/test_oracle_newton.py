"""Pins of the oracle's Sparse Newton step with inertia control (CPU only; Sec. 4 "Generalization to
Arbitrary Objectives", eq. totalHessian; Appendix A, Theorem 2; Sec. 5, the inertia test).

Element level: the forward-mode directional derivative of the element gradient equals the
complex-step element Hessian applied to the direction (and, along the modulus, the complex-step
dc/dp); the complex-step Hessian of lam . g_e is symmetric across its two independent
constructions (x rows from the x-direction derivative, p row from the modulus derivative), its
x-x block matches a fourth-order difference quotient of complex-step Hessians along lam, its x-p
column is K_e lam_e and its p-p entry lam . g_e (log-modulus closed forms), and the third
derivative it contracts is fully symmetric.

Global level: the reduced Newton Hessian equals the central difference quotient of the adjoint
gradient over re-solved equilibria (the plain definition of d2f/dp2); the saddle-point system with
the Newton blocks gives the same dp, dx and multiplier block as the dense reduced step (Theorem 1);
the saddle-point inertia equals (n_x, n_x, 0) plus the inertia of H (Haynsworth) counted on the
dense matrix; the inertia correction accepts the first trial with a positive definite H + delta
(I + S^T S); the outer loop decreases f, and converges quadratically once no regularisation is
needed.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import sgn_inputs as si
from oracle import dense as D
from oracle import fem
from oracle import newton as N

_CASE = {}


def _grid5():
    if "g5" not in _CASE:
        prob = D.setup_targets(si.problem_2d(5, seed=0))
        p = prob.p_init()
        x, info = D.equilibrium(prob, p, rtol=1e-12)
        assert info.converged
        _CASE["g5"] = (prob, x, p)
    return _CASE["g5"]


def _elements(dim):
    if dim == 2:
        prob, x, p = _grid5()
    else:
        prob = D.setup_targets(si.problem_3d(4, 2, 2, 0.5, seed=0))
        p = prob.p_init() + 0.2 * np.sin(np.arange(prob.n_p))
        x, info = D.equilibrium(prob, p, rtol=1e-12)
        assert info.converged
    xe, Xe, mu, lam = D._gather(prob, x, p)
    return xe, Xe, mu, lam


@pytest.mark.parametrize("dim", [2, 3])
def test_forward_directional_derivative_matches_complex_step(dim):
    xe, Xe, mu, lam = _elements(dim)
    ne = xe.shape[0]
    rng = np.random.default_rng(dim)
    v = rng.standard_normal(xe.shape)
    g, dg = N.element_gradient_dir(xe, v, Xe, mu, lam, 0 * mu, 0 * mu)
    assert np.max(np.abs(g - fem.element_gradient(xe, Xe, mu, lam))) <= 1e-14 * np.max(np.abs(g))
    H = fem.element_hessian(xe, Xe, mu, lam)
    ref = np.einsum("eij,ej->ei", H, v.reshape(ne, -1))
    assert np.max(np.abs(dg.reshape(ne, -1) - ref)) <= 1e-13 * np.max(np.abs(ref))
    _, dgp = N.element_gradient_dir(xe, 0 * v, Xe, mu, lam, mu, lam)
    ref = fem.element_dgrad_dlogE(xe, Xe, mu, lam)
    assert np.max(np.abs(dgp.reshape(ne, -1) - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("dim", [2, 3])
def test_element_lagrangian_hessian(dim):
    xe, Xe, mu, lam = _elements(dim)
    ne = xe.shape[0]
    rng = np.random.default_rng(10 + dim)
    lam_e = rng.standard_normal(xe.shape)
    Hm = N.element_lagrangian_hessian(xe, Xe, mu, lam, lam_e)
    n = Hm.shape[1] - 1
    scale = np.max(np.abs(Hm))
    # mixed partials: the x-p column (from the modulus step on the x rows) against the p row (from the
    # x steps on the modulus derivative), and the x-x block against itself transposed
    assert np.max(np.abs(Hm - np.swapaxes(Hm, 1, 2))) <= 1e-13 * scale
    # x-x: the derivative of the element Hessian along lam, by a fourth-order central difference
    h = 3e-5

    def K(s):
        return fem.element_hessian(xe + s * lam_e, Xe, mu, lam)

    fd = (8.0 * (K(h) - K(-h)) - (K(2 * h) - K(-2 * h))) / (12.0 * h)
    assert np.max(np.abs(Hm[:, :n, :n] - fd)) <= 1e-10 * np.max(np.abs(fd))
    # log-modulus closed forms: d2(lam.g)/dx dp = K lam, d2(lam.g)/dp2 = lam.g
    H = fem.element_hessian(xe, Xe, mu, lam)
    klam = np.einsum("eij,ej->ei", H, lam_e.reshape(ne, -1))
    assert np.max(np.abs(Hm[:, :n, n] - klam)) <= 1e-13 * np.max(np.abs(klam))
    lg = np.sum(fem.element_gradient(xe, Xe, mu, lam).reshape(ne, -1) * lam_e.reshape(ne, -1), axis=1)
    assert np.max(np.abs(Hm[:, n, n] - lg)) <= 1e-13 * np.max(np.abs(lg))
    # full symmetry of the third derivative: u . T[lam] v = lam . T[u] v
    u = rng.standard_normal(xe.shape)
    w = rng.standard_normal((ne, n))
    Hu = N.element_lagrangian_hessian(xe, Xe, mu, lam, u)
    a = np.einsum("ei,eij,ej->e", u.reshape(ne, -1), Hm[:, :n, :n], w)
    b = np.einsum("ei,eij,ej->e", lam_e.reshape(ne, -1), Hu[:, :n, :n], w)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_reduced_newton_hessian_is_the_derivative_of_the_adjoint_gradient():
    prob, x, p = _grid5()
    H, g, S, lam = N.reduced_newton_hessian(prob, x, p)
    g_ref, lam_ref = D.adjoint_gradient(prob, x, p)
    assert np.linalg.norm(g - g_ref) <= 1e-12 * np.linalg.norm(g_ref)
    assert np.linalg.norm(lam - lam_ref) <= 1e-12 * np.linalg.norm(lam_ref)

    def grad_at(pp):
        xx, info = D.equilibrium(prob, pp, x, rtol=1e-13)
        assert info.converged
        return D.adjoint_gradient(prob, xx, pp)[0]

    h = 1e-5
    fd = np.empty_like(H)
    for j in range(prob.n_p):
        e = np.zeros(prob.n_p)
        e[j] = h
        fd[:, j] = (grad_at(p + e) - grad_at(p - e)) / (2 * h)
    assert np.max(np.abs(H - fd)) <= 1e-7 * np.max(np.abs(H))
    # and it is not the Gauss-Newton Hessian: the second-order term is visible at this state
    Hgn, _ = D.dense_gn_hessian(prob, x, p)
    assert np.max(np.abs(H - Hgn)) >= 1e-2 * np.max(np.abs(H))


@pytest.mark.parametrize("delta", [0.0, 0.05])
def test_saddle_point_solve_equals_reduced_newton_step(delta):
    prob, x, p = _grid5()
    H, g, S, lam = N.reduced_newton_hessian(prob, x, p)
    nx, npar = prob.n_x, prob.n_p
    K = N.newton_matrix_sparse(prob, x, p, delta)
    b = np.concatenate([np.zeros(nx), -g, np.zeros(nx)])
    z = spla.spsolve(K.tocsc(), b)
    Hd = H + delta * (np.eye(npar) + S.T @ S)
    dp = -np.linalg.solve(Hd, g)
    assert np.linalg.norm(z[nx:nx + npar] - dp) <= 1e-9 * np.linalg.norm(dp)
    assert np.linalg.norm(z[:nx] - S @ dp) <= 1e-9 * np.linalg.norm(S @ dp)
    # dense inertia of the saddle-point matrix = (n_x, n_x, 0) + inertia(H + delta (I + S^T S))
    ev = np.linalg.eigvalsh(K.toarray())
    tol = 1e-14 * np.max(np.abs(ev))  # the smallest |eigenvalue| here is 1.8e-4 of 9.2e6
    dense = (int(np.sum(ev > tol)), int(np.sum(ev < -tol)), int(np.sum(np.abs(ev) <= tol)))
    assert dense == N.saddle_inertia(Hd, nx)


def test_inertia_correction_accepts_the_first_positive_definite_trial():
    prob, x, p = _grid5()
    st = N.inertia_corrected_step(prob, x, p)
    H, g, S, lam = N.reduced_newton_hessian(prob, x, p)
    nx, npar = prob.n_x, prob.n_p
    # at the initial parameters of this grid the Newton Hessian is indefinite
    assert np.linalg.eigvalsh(H)[0] < 0
    assert st.trials > 1 and st.delta > 0
    deltas = list(N.delta_trials(0.0))[: st.trials]
    assert deltas[-1] == st.delta
    for d in deltas[:-1]:
        assert np.linalg.eigvalsh(H + d * (np.eye(npar) + S.T @ S))[0] < 0
    assert np.linalg.eigvalsh(H + st.delta * (np.eye(npar) + S.T @ S))[0] > 0
    assert st.inertia == (nx + npar, nx, 0)
    # the saddle-point solve at the accepted delta reproduces the step in all three blocks
    K = N.newton_matrix_sparse(prob, x, p, st.delta)
    z = spla.spsolve(K.tocsc(), np.concatenate([np.zeros(nx), -g, np.zeros(nx)]))
    for got, ref in ((z[:nx], st.dx), (z[nx:nx + npar], st.dp), (z[nx + npar:], st.dlam)):
        assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)
    assert g @ st.dp < 0
    # with a remembered delta the sequence restarts at a third of it
    assert list(N.delta_trials(0.3))[:3] == pytest.approx([0.0, 0.1, 0.8], rel=1e-15)


def test_newton_iterations_decrease_and_converge_quadratically():
    prob = D.setup_targets(si.problem_2d(7, seed=1))
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-12)
    assert info.converged
    trace, p1, x1 = N.newton_iterations(prob, p, x, iters=12)
    f = [t[0] for t in trace]
    gn = [t[1] for t in trace]
    assert all(b <= a for a, b in zip(f, f[1:]))
    assert trace[0][3] > 0 and trace[0][4] > 1  # regularised at the start
    assert gn[-1] <= 1e-10 * gn[0]
    # the last unregularised full steps: |g_k+1| <= C |g_k|^2
    tail = [(a, b) for (a, b, t) in zip(gn, gn[1:], trace) if t[3] == 0.0 and t[2] == 1.0 and a < 1e-4]
    assert len(tail) >= 2
    assert all(b <= 1e4 * a * a for a, b in tail)  # C near 2e3 measured
    # superlinear: the contraction factor itself collapses
    assert gn[-1] <= 1e-4 * gn[-2]


def test_newton_blocks_refuse_other_parameter_kinds():
    prob = si.problem_3d(4, 2, 2, 0.5, seed=0, param_kind=si.P_REST_POS)
    x = prob.x_rest()
    with pytest.raises(ValueError):
        N.lagrangian_second_derivatives(prob, x, prob.p_init(), np.zeros(prob.n_x))
