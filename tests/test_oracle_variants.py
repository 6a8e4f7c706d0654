"""Pins of the oracle's method variants of Sec. 4 (CPU only): the block Gauss-Newton step and the
SGN-initialised L-BFGS.

Block solve (Appendix B): on rest-position problems with every free DOF a target and no
regulariser (B = C = 0, Kp square and invertible) the block step equals the dense Gauss-Newton
step in all three blocks (Theorem 1 then Appendix B); it refuses problems outside those conditions.

L-BFGS: the two-loop recursion equals the explicit BFGS inverse-Hessian update of the initial
matrix (the textbook identity behind it, written here as dense products), which satisfies the
secant condition on the newest pair; with an empty memory the direction is the Gauss-Newton step,
so the first iteration and a memory of 0 reproduce the plain SGN iterations; the objective
decreases monotonically.
"""
import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D


def _bgn_problem(seed=5):
    prob = si.problem_3d(4, 2, 2, 0.25, seed=seed, param_kind=si.P_REST_POS)
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged
    prob = prob.copy()
    prob.target_dof = np.arange(prob.n_x, dtype=np.int32)
    prob.target_val = x + 1e-3 * np.sin(np.arange(prob.n_x))
    prob.length_scale = 1.0
    prob.reg_mu = 0.0
    return prob, x, p


def test_block_step_equals_dense_gauss_newton_step():
    prob, x, p = _bgn_problem()
    st = D.dense_gn_step(prob, x, p)
    bg = D.block_gn_step(prob, x, p)
    for a, b in ((bg.dx, st.dx), (bg.dp, st.dp), (bg.dlam, st.dlam), (bg.grad, st.grad)):
        assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)
    # dx = -A^-1 df/dx^T: with A = I / ell^2 and ell = 1 this is the misfit with its sign flipped
    assert np.allclose(bg.dx, -(x - prob.target_val), rtol=0, atol=1e-15)
    # the multiplier block of the adjoint right-hand side is minus the adjoint multiplier
    assert np.linalg.norm(bg.dlam + bg.lam_adj) <= 1e-10 * np.linalg.norm(bg.lam_adj)


def test_block_step_refuses_problems_outside_its_conditions():
    prob, x, p = _bgn_problem()
    with_reg = prob.copy()
    with_reg.reg_mu = 1e-4
    with pytest.raises(ValueError):
        D.block_gn_step(with_reg, x, p)
    partial = prob.copy()
    partial.target_dof = prob.target_dof[: prob.n_x // 2].copy()
    partial.target_val = prob.target_val[: prob.n_x // 2].copy()
    with pytest.raises(ValueError):
        D.block_gn_step(partial, x, p)
    loge = si.problem_3d(4, 2, 2, 0.25, seed=5)
    loge.length_scale = 1.0
    loge.target_val = loge.x_rest()[loge.target_dof]
    with pytest.raises(ValueError):
        D.block_gn_step(loge, loge.x_rest(), loge.p_init())


def test_two_loop_recursion_equals_explicit_bfgs_update():
    rng = np.random.default_rng(0)
    n = 12
    Q = rng.standard_normal((n, n))
    H0 = Q @ Q.T + n * np.eye(n)   # initial inverse Hessian (SPD)
    Bt = rng.standard_normal((n, n))
    Bt = Bt @ Bt.T + np.eye(n)     # a curvature model: y = Bt s gives s^T y > 0
    pairs = []
    for _ in range(4):
        s = rng.standard_normal(n)
        pairs.append((s, Bt @ s))
    g = rng.standard_normal(n)
    d = D.lbfgs_direction(g, pairs, lambda q: H0 @ q)
    H = H0.copy()
    for s, y in pairs:
        rho = 1.0 / (y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    assert np.linalg.norm(d + H @ g) <= 1e-12 * np.linalg.norm(H @ g)
    s, y = pairs[-1]
    assert np.linalg.norm(H @ y - s) <= 1e-12 * np.linalg.norm(s)  # secant condition
    # empty memory: the initial matrix alone
    assert np.allclose(D.lbfgs_direction(g, [], lambda q: H0 @ q), -H0 @ g, rtol=1e-15, atol=0)


@pytest.fixture(scope="module")
def grid():
    prob = D.setup_targets(si.problem_2d(8, seed=1))
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged
    return prob, x, p


def test_lbfgs_without_memory_is_sgn(grid):
    prob, x, p = grid
    t_sgn, p_sgn, _ = D.sgn_iterations(prob, p, x, iters=4)
    t_lb, p_lb, _ = D.lbfgs_sgn_iterations(prob, p, x, iters=4, m=0)
    assert [a for *_, a in t_sgn] == [a for *_, a in t_lb]
    assert np.allclose([f for f, *_ in t_sgn], [f for f, *_ in t_lb], rtol=1e-12, atol=0)
    assert np.linalg.norm(p_lb - p_sgn) <= 1e-10 * np.linalg.norm(p_sgn)


def test_lbfgs_first_step_is_the_gauss_newton_step_and_objective_decreases(grid):
    prob, x, p = grid
    st = D.dense_gn_step(prob, x, p)
    t_lb, p1, _ = D.lbfgs_sgn_iterations(prob, p, x, iters=1, m=5)
    assert np.linalg.norm((p1 - p) / t_lb[0][2] - st.dp) <= 1e-10 * np.linalg.norm(st.dp)
    t_lb, pf, xf = D.lbfgs_sgn_iterations(prob, p, x, iters=6, m=5)
    fs = [f for f, *_ in t_lb] + [D.objective(prob, xf, pf)]
    assert all(fs[i + 1] <= fs[i] for i in range(len(fs) - 1))
    assert fs[-1] < 1e-2 * fs[0]
