"""Pins of the oracle's BiCGSTAB and stabilised matrix (CPU only): what linear algebra fixes."""
import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D
from oracle import krylov as KR


def test_bicgstab_solves_random_nonsymmetric_systems():
    rng = np.random.default_rng(0)
    for n in (5, 40, 120):
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        b = rng.standard_normal(n)
        x, it, hist = KR.bicgstab(A, b, lambda v: v, tol=1e-13)
        ref = np.linalg.solve(A, b)
        assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
        assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
        assert it <= n


def test_bicgstab_with_exact_preconditioner_takes_one_iteration():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 30)) + 5 * np.eye(30)
    b = rng.standard_normal(30)
    Ainv = np.linalg.inv(A)
    x, it, _ = KR.bicgstab(A, b, lambda v: Ainv @ v, tol=1e-12)
    assert it == 1
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-12 * np.linalg.norm(x)


@pytest.mark.parametrize("eps", [1e-6, 1e2])
def test_stabilised_preconditioner_recovers_the_gauss_newton_step(eps):
    prob = D.setup_targets(si.config_tiny())
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged
    K = D.sgn_matrix_dense(prob, x, p)
    Ke = KR.stabilised_sgn_matrix(prob, x, p, eps, eps)
    nx, npar = prob.n_x, prob.n_p
    # the stabilisation sits on the diagonal of the x and multiplier blocks only
    d = np.diag(Ke - K)
    ulp = 4e-16 * np.abs(np.diag(K))  # rounding of eps added to the target diagonal A
    assert np.all(np.abs(d[:nx] - eps) <= ulp[:nx] + 1e-15 * eps)
    assert np.all(d[nx:nx + npar] == 0) and np.all(d[nx + npar:] == -eps)
    assert np.array_equal(Ke - np.diag(np.diag(Ke)), K - np.diag(np.diag(K)))
    b = D.sgn_rhs(prob, x, p)
    st = D.dense_gn_step(prob, x, p)
    # row-equilibrated system (the scaling the library solves in), preconditioned by the stabilised LU
    s = 1.0 / np.sqrt(np.max(np.abs(K), axis=1))
    A = K * s[:, None] * s[None, :]
    Ae = Ke * s[:, None] * s[None, :]
    z, it, hist = KR.bicgstab(A, s * b, lambda v: np.linalg.solve(Ae, v), tol=1e-12)
    z = s * z
    dp = z[nx:nx + npar]
    assert np.linalg.norm(dp - st.dp) <= 1e-9 * np.linalg.norm(st.dp)
    # the stabilised matrix alone gives another step (by the stabilisation's effect)
    dp_e = np.linalg.solve(Ke, b)[nx:nx + npar]
    gap = np.linalg.norm(dp_e - st.dp) / np.linalg.norm(st.dp)
    assert gap > 1e-13
    assert it >= (3 if eps >= 1e2 else 1)
