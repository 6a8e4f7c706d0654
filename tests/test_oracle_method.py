"""Pins of the oracle's equilibrium, gradient and Gauss-Newton step (CPU only).

Each check is fixed by the mathematics, not by re-running the oracle's own
formula: zero load, the linear-elastic limit, Newton's quadratic rate, finite
differences of the reduced objective, Theorem 1 (Appendix A: the sparse
system's dp equals the dense GN step), the KKT form of Appendix A, the
KKT inertia, and two special cases with closed-form steps.
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg as sla

import sgn_inputs as si
from oracle import dense as D


@pytest.fixture(scope="module")
def tiny():
    return D.setup_targets(si.config_tiny())


@pytest.fixture(scope="module")
def c2d():
    return D.setup_targets(si.config_2d())


@pytest.fixture(scope="module")
def rest():
    return D.setup_targets(si.problem_3d(3, 2, 2, 1 / 3, seed=1, param_kind=si.P_REST_POS))


def _tiny3d(param_kind=si.P_LOGE, seed=3):
    return si.problem_3d(4, 2, 2, 0.25, seed=seed, param_kind=param_kind)


def _scaled_solve(K, b, sweeps=3):
    s = np.ones(K.shape[0])
    for _ in range(sweeps):
        s = s / np.sqrt(np.max(np.abs(K * s[:, None] * s[None, :]), axis=1))
    Ks = K * s[:, None] * s[None, :]
    return s * np.linalg.solve(Ks, s * b)


def test_zero_load_keeps_rest_state():
    # P(I) = 0: the rest state is an equilibrium without load (up to rounding in F = Ds Dm^-1)
    prob = si.config_tiny()
    prob.f_ext = np.zeros_like(prob.f_ext)
    h = 1.0 / 3.0
    c = D.residual(prob, prob.x_rest(), prob.p_init())
    assert np.linalg.norm(c) <= 1e-12 * prob.E0 * h
    x, info = D.equilibrium(prob, prob.p_init(), atol=1e-12 * prob.E0 * h)
    assert info.converged and info.iters == 0 and np.array_equal(x, prob.x_rest())


@pytest.mark.parametrize("mk", [si.config_tiny, _tiny3d])
def test_equilibrium_residual_and_quadratic_rate(mk):
    prob = mk()
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged
    assert np.linalg.norm(D.residual(prob, x, p)) <= 1e-11 * np.linalg.norm(D.fext_free(prob))
    # quadratic rate: |c_{k+1}| <= C |c_k|^2 over the Newton iterates (load x20 for a few steps)
    prob2 = dataclasses.replace(prob, f_ext=prob.f_ext * 20)
    xk = prob2.x_rest()
    norms = []
    for _ in range(4):
        c = D.residual(prob2, xk, p)
        norms.append(np.linalg.norm(c))
        K = D.stiffness(prob2, xk, p).toarray()
        xk = xk - np.linalg.solve(K, c)
    ratios = [norms[i + 1] / norms[i] ** 2 for i in range(len(norms) - 1) if norms[i + 1] > 1e-9 * norms[0]]
    assert len(ratios) >= 2 and max(ratios[1:]) <= 5 * ratios[0] + 1e-30


@pytest.mark.parametrize("mk", [si.config_tiny, _tiny3d])
def test_small_load_matches_linear_elasticity(mk):
    prob = mk()
    p = prob.p_init()
    K0 = D.stiffness(prob, prob.x_rest(), p).toarray()
    errs = []
    for s in (1e-3, 2e-3):
        pr = dataclasses.replace(prob, f_ext=prob.f_ext * s)
        x, info = D.equilibrium(pr, p, rtol=1e-13)
        u = x - prob.x_rest()
        ul = np.linalg.solve(K0, D.fext_free(pr))
        errs.append(np.linalg.norm(u - ul) / np.linalg.norm(ul))
    # the nonlinear correction is first order in the load: doubling the load doubles it
    assert errs[0] < 1e-3
    assert 1.7 < errs[1] / errs[0] < 2.3


@pytest.mark.parametrize("fixture", ["tiny", "c2d"])
def test_adjoint_gradient_equals_direct_sensitivity_gradient(fixture, request):
    prob = request.getfixturevalue(fixture)
    p = prob.p_init() + 0.05
    x, _ = D.equilibrium(prob, p)
    st = D.dense_gn_step(prob, x, p)
    g_adj, _ = D.adjoint_gradient(prob, x, p)
    assert np.linalg.norm(g_adj - st.grad) <= 1e-12 * np.linalg.norm(st.grad)


@pytest.mark.parametrize("mk", [si.config_tiny, lambda: _tiny3d(si.P_REST_POS)])
def test_adjoint_gradient_matches_central_differences(mk):
    prob = D.setup_targets(mk())
    rng = np.random.default_rng(7)
    p = prob.p_init() + (0.1 if prob.param_kind == si.P_LOGE else 0.002) * rng.standard_normal(prob.n_p)
    x, _ = D.equilibrium(prob, p, rtol=1e-13)
    g, _ = D.adjoint_gradient(prob, x, p)
    scale = 1.0 if prob.param_kind == si.P_LOGE else 1e-2
    for _ in range(5):
        v = rng.standard_normal(prob.n_p)
        v /= np.linalg.norm(v)
        h = 5e-5 * scale
        fp = D.objective(prob, *reversed((p + h * v, D.equilibrium(prob, p + h * v, x, rtol=1e-14)[0])))
        fm = D.objective(prob, *reversed((p - h * v, D.equilibrium(prob, p - h * v, x, rtol=1e-14)[0])))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * max(abs(g @ v), 1e-3 * np.linalg.norm(g))


@pytest.mark.parametrize("fixture", ["tiny", "c2d", "rest"])
def test_theorem1_sparse_system_reproduces_dense_gn_step(fixture, request):
    prob = request.getfixturevalue(fixture)
    p = prob.p_init()
    x, _ = D.equilibrium(prob, p)
    st = D.dense_gn_step(prob, x, p)
    K = D.sgn_matrix_dense(prob, x, p)
    b = D.sgn_rhs(prob, x, p)
    z = _scaled_solve(K, b)
    nx, npar = prob.n_x, prob.n_p
    assert np.linalg.norm(z[nx:nx + npar] - st.dp) <= 1e-9 * np.linalg.norm(st.dp)
    assert np.linalg.norm(z[:nx] - st.dx) <= 1e-9 * np.linalg.norm(st.dx)
    assert np.linalg.norm(z[nx + npar:] - st.dlam) <= 1e-9 * np.linalg.norm(st.dlam)


def test_kkt_right_hand_side_shifts_multiplier_by_adjoint(tiny):
    prob = tiny
    p = prob.p_init()
    x, _ = D.equilibrium(prob, p)
    st = D.dense_gn_step(prob, x, p)
    K = D.sgn_matrix_dense(prob, x, p)
    z = _scaled_solve(K, D.sgn_rhs(prob, x, p, "kkt"))
    nx, npar = prob.n_x, prob.n_p
    assert np.linalg.norm(z[nx:nx + npar] - st.dp) <= 1e-9 * np.linalg.norm(st.dp)
    assert np.linalg.norm(z[nx + npar:] - st.dlam - st.lam_adj) <= 1e-9 * np.linalg.norm(st.lam_adj)


@pytest.mark.parametrize("fixture", ["tiny", "c2d", "rest"])
def test_kkt_inertia(fixture, request):
    prob = request.getfixturevalue(fixture)
    p = prob.p_init()
    x, _ = D.equilibrium(prob, p)
    ev = np.linalg.eigvalsh(D.sgn_matrix_dense(prob, x, p))
    assert ((ev > 0).sum(), (ev < 0).sum(), (ev == 0).sum()) == (prob.n_x + prob.n_p, prob.n_x, 0)


def _all_dof_targets(prob, x):
    prob = prob.copy()
    prob.target_dof = np.arange(prob.n_x, dtype=np.int32)
    prob.target_val = x + 1e-3 * np.sin(np.arange(prob.n_x))
    prob.length_scale = 1.0
    prob.reg_mu = 0.0
    return prob


def test_nodal_force_parameters_step_is_minus_stiffness_times_misfit():
    # c = grad E - f_ext - p, so Kp = -I and S = Kx^-1; with A = I and no regulariser
    # the GN step is dp = -(S^T S)^-1 S^T (x - t) = -Kx (x - t).
    prob = si.problem_2d(5, seed=2, param_kind=si.P_NODAL_FORCE)
    p = np.zeros(prob.n_x)
    x, _ = D.equilibrium(prob, p)
    prob = _all_dof_targets(prob, x)
    prob.p_ref = np.zeros(prob.n_x)
    st = D.dense_gn_step(prob, x, p)
    Kx = D.stiffness(prob, x, p).toarray()
    ref = -Kx @ (x - prob.target_val)
    assert np.linalg.norm(st.dp - ref) <= 1e-9 * np.linalg.norm(ref)


def test_block_solve_closed_form_for_rest_positions():
    # B = C = 0, Kp invertible: dp = Kp^-1 Kx A^-1 df/dx^T (Appendix B, final form).
    prob = _tiny3d(si.P_REST_POS, seed=5)
    p = prob.p_init()
    x, _ = D.equilibrium(prob, p)
    prob = _all_dof_targets(prob, x)
    prob.p_ref = p.copy()
    st = D.dense_gn_step(prob, x, p)
    Kx = D.stiffness(prob, x, p).toarray()
    Kp = D.param_jacobian(prob, x, p).toarray()
    fx, *_ = D.objective_blocks(prob, x, p)
    ref = np.linalg.solve(Kp, Kx @ fx)
    assert np.linalg.norm(st.dp - ref) <= 1e-8 * np.linalg.norm(ref)
    # the sign printed in the body of Sec. 4 (dp = -Kp^-1 Kx dy) is the opposite one
    assert np.linalg.norm(st.dp + ref) > 1.0 * np.linalg.norm(ref)


def test_gn_iterations_decrease_objective(tiny):
    prob = tiny
    p = prob.p_init()
    x, _ = D.equilibrium(prob, p)
    trace, pf, xf = D.sgn_iterations(prob, p, x, iters=5)
    fs = [t[0] for t in trace] + [D.objective(prob, xf, pf)]
    assert all(fs[i + 1] < fs[i] for i in range(len(fs) - 1))
    assert trace[-1][1] < 1e-2 * trace[0][1]


@pytest.mark.parametrize("fixture", ["tiny", "rest"])
def test_sparse_sgn_matrix_equals_dense_and_solves_theorem1_step(fixture, request):
    """The sparse assembly of K_SGN (eq. sparseSystemGN) is entry for entry the dense one, and the dense
    Gauss-Newton step [dx; dp; dlam] (Theorem 1) solves it to rounding in the equilibrated measure."""
    prob = request.getfixturevalue(fixture)
    p = prob.p_init()
    x, _ = D.equilibrium(prob, p)
    Ks = D.sgn_matrix_sparse(prob, x, p)
    assert np.array_equal(Ks.toarray(), D.sgn_matrix_dense(prob, x, p))
    st = D.dense_gn_step(prob, x, p)
    z = np.concatenate([st.dx, st.dp, st.dlam])
    b = D.sgn_rhs(prob, x, p)
    assert D.equilibrated_residual(Ks, z, b) <= 1e-10
    assert D.equilibrated_residual(Ks, np.zeros_like(z), b) == pytest.approx(1.0, rel=1e-15)


def test_equilibrated_residual_hand_example():
    """K = [[4, 1], [1, 9]]: row maxima 4 and 9, S = diag(1/2, 1/3); for b = (2, 3) and z = (1/2, 0)
    the residual is (0, 5/2), scaled (0, 5/6), over |(1, 1)| = sqrt(2)."""
    import scipy.sparse as sp
    K = sp.csr_matrix(np.array([[4.0, 1.0], [1.0, 9.0]]))
    got = D.equilibrated_residual(K, np.array([0.5, 0.0]), np.array([2.0, 3.0]))
    assert got == pytest.approx((5.0 / 6.0) / np.sqrt(2.0), rel=1e-15)
    ext = D.equilibrated_residual_extended(K, np.array([0.5, 0.0]), np.array([2.0, 3.0]))
    assert ext == pytest.approx((5.0 / 6.0) / np.sqrt(2.0), rel=1e-15)
    # invariant under a common scale of matrix and right-hand side
    assert D.equilibrated_residual(7.0 * K, np.array([0.5, 0.0]), np.array([14.0, 21.0])) == pytest.approx(got, rel=1e-14)


def test_no_targets_gives_the_regulariser_step():
    """No targets: A = 0 and df/dx = 0, the reduced Hessian is C = mu I and g = mu (p - p_ref), so the
    dense Gauss-Newton step is dp = p_ref - p exactly."""
    prob = si.problem_2d(5, seed=4)
    prob.target_dof = np.zeros(0, np.int32)
    prob.target_val = np.zeros(0)
    prob.length_scale = 1.0
    p = 0.1 * np.random.default_rng(5).standard_normal(prob.n_p)
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged
    st = D.dense_gn_step(prob, x, p)
    assert np.linalg.norm(st.dp - (prob.p_ref - p)) <= 1e-12 * np.linalg.norm(p)


def test_extended_refinement_reaches_the_rounded_exact_solution():
    """Refinement with extended-precision residuals converges to the exact solution of the stored
    (FP64) system to u_64 + cond u_ext (Wilkinson's bound for a residual carried in a precision u_ext):
    on the 8 x 8 Hilbert matrix (cond 1.5e10) against the exact solution computed in rational arithmetic
    from the FP64 entries, while one LU solve is off by about cond u_64."""
    from fractions import Fraction
    import scipy.sparse as sp
    n = 8
    H = np.array([[1.0 / (i + j + 1) for j in range(n)] for i in range(n)])
    b = H @ np.ones(n)
    # exact rational solution of the FP64 system (Gauss-Jordan on Fractions)
    M = [[Fraction(float(H[i, j])) for j in range(n)] + [Fraction(float(b[i]))] for i in range(n)]
    for k in range(n):
        piv = max(range(k, n), key=lambda r: abs(M[r][k]))
        M[k], M[piv] = M[piv], M[k]
        for r in range(n):
            if r != k and M[r][k] != 0:
                f = M[r][k] / M[k][k]
                M[r] = [a - f * c for a, c in zip(M[r], M[k])]
    exact = np.array([float(M[i][n] / M[i][i]) for i in range(n)])
    z0 = np.linalg.solve(H, b)
    z, hist = D.refine_extended(sp.csr_matrix(H), b, z0, sweeps=4)
    err0 = np.linalg.norm(z0 - exact) / np.linalg.norm(exact)
    err = np.linalg.norm(z - exact) / np.linalg.norm(exact)
    bound = 4 * np.finfo(np.float64).eps + 10 * np.linalg.cond(H) * np.finfo(np.longdouble).eps
    assert err0 > 1e-9            # a plain solve carries cond * u
    assert err <= bound, (err, bound)
    assert err <= 0.1 * err0


def test_polished_step_is_the_dense_step_on_a_small_problem(tiny):
    prob = tiny
    p = prob.p_init()
    x, _ = D.equilibrium(prob, p, rtol=1e-11)
    st = D.dense_gn_step(prob, x, p)
    b = D.sgn_rhs(prob, x, p)
    z0 = np.concatenate([st.dx, st.dp, st.dlam])
    z, hist = D.polish_sgn_solution(prob, x, p, z0, b, sweeps=2)
    ref = np.linalg.solve(D.sgn_matrix_dense(prob, x, p), b)
    for sl in (slice(0, prob.n_x), slice(prob.n_x, prob.n_x + prob.n_p)):
        assert np.linalg.norm(z[sl] - ref[sl]) <= 1e-9 * np.linalg.norm(ref[sl])
    assert hist[-1] <= hist[0] and hist[-1] <= 1e-12
