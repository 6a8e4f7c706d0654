"""GPU parity of the BiCGSTAB solve preconditioned by the LDL^T of the stabilised matrix (Sec. 5,
"Solving the saddle point problem": eps_x, eps_lambda added to the x and multiplier diagonals of
the factorised matrix, BiCGSTAB on the unstabilised system).

The expected step is the oracle's dense Gauss-Newton step (Theorem 1 of Appendix A): BiCGSTAB
must recover it whatever the stabilisation, while the stabilised factor's own refined solve gives
the step of the stabilised matrix, which the oracle's dense solve of that matrix fixes.
"""
import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D
from oracle import krylov as KR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_03285_amd import sgn  # noqa: E402


def _cuda(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    return t.detach().cpu().numpy()


_MK = {
    "tiny": si.config_tiny,
    "grid21": si.config_2d,
    "cant4x2x2": lambda: si.problem_3d(4, 2, 2, 0.25, seed=1),
    "rest3x2x2": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=1, param_kind=si.P_REST_POS),
}
_CASES = {}


def _case(name):
    if name not in _CASES:
        prob = D.setup_targets(_MK[name]())
        p = prob.p_init()
        x, info = D.equilibrium(prob, p, rtol=1e-11)
        assert info.converged
        _CASES[name] = (prob, p, x, D.dense_gn_step(prob, x, p))
    return _CASES[name]


def _solve(prob, x, p, **opt):
    ctx = sgn.Context(prob, sgn.default_options(newton_rtol=1e-11, **opt)).allocate()
    N = 2 * prob.n_x + prob.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    xd, pd = _cuda(x), _cuda(p)
    ctx.equilibrium(pd, xd)  # at the oracle's equilibrium: leaves the Kx factor the adjoint form needs
    ctx.assemble(xd, pd, rhs)
    ctx.factor()
    info = ctx.solve(rhs, sol)
    return info, _host(sol), _host(rhs)


@pytest.mark.parametrize("precision", [sgn.SGN_FP64, sgn.SGN_FP32_IR])
@pytest.mark.parametrize("name", list(_MK))
def test_bicgstab_with_paper_stabilisation_gives_the_gauss_newton_step(name, precision):
    prob, p, x, st = _case(name)
    info, z, _ = _solve(prob, x, p, precision=precision, solver=sgn.SGN_BICGSTAB, eps_x=1e-6, eps_lambda=1e-6)
    assert info.rel_res <= 1e-10 and info.gmres_iters == 0
    assert 1 <= info.sweeps <= 10, info.sweeps
    nx, npar = prob.n_x, prob.n_p
    tol = 1e-9 if precision == sgn.SGN_FP64 else 1e-8
    for got, ref in ((z[nx:nx + npar], st.dp), (z[:nx], st.dx), (z[nx + npar:], st.dlam)):
        assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["tiny", "cant4x2x2"])
def test_bicgstab_recovers_the_unstabilised_step_from_a_strong_stabilisation(name):
    prob, p, x, st = _case(name)
    eps = 1e2  # far above the paper's 1e-6: the factor is of a visibly different matrix
    nx, npar = prob.n_x, prob.n_p
    # the stabilised factor's own refined solve converges to the stabilised matrix's step
    info_s, z_s, b = _solve(prob, x, p, eps_x=eps, eps_lambda=eps)
    Ke = KR.stabilised_sgn_matrix(prob, x, p, eps, eps)
    ze = np.linalg.solve(Ke, b)
    assert np.linalg.norm(z_s - ze) <= 1e-8 * np.linalg.norm(ze)
    gap = np.linalg.norm(z_s[nx:nx + npar] - st.dp) / np.linalg.norm(st.dp)
    assert gap > 1e-6, gap
    # BiCGSTAB on the unstabilised system recovers the Gauss-Newton step: it solves the oracle's
    # unstabilised system to the tolerance, and the solution agrees with the dense solve to what that
    # residual allows: in the equilibrated variables w = S^-1 z the relative forward error is at most
    # cond(S K S) times the equilibrated relative residual (the 4 x 4 grid's is 4e7)
    info, z, b2 = _solve(prob, x, p, solver=sgn.SGN_BICGSTAB, eps_x=eps, eps_lambda=eps)
    assert info.rel_res <= 1e-10
    assert info.sweeps >= 2
    K = D.sgn_matrix_sparse(prob, x, p)
    res = D.equilibrated_residual(K, z, b2)
    assert res <= 1e-10
    Kd = K.toarray()
    sc = 1.0 / np.sqrt(np.abs(Kd).max(axis=1))
    kappa = np.linalg.cond(sc[:, None] * Kd * sc[None, :])
    zref = np.linalg.solve(Kd, b2)
    assert np.linalg.norm(zref[nx:nx + npar] - st.dp) <= 1e-9 * np.linalg.norm(st.dp)  # the same system
    bound = kappa * (res + 1e-15)  # plus the dense solve's own rounding
    assert np.linalg.norm((z - zref) / sc) <= bound * np.linalg.norm(zref / sc)


def test_outer_step_with_bicgstab_matches_ldlt():
    prob = D.setup_targets(si.problem_2d(8, seed=1))
    res = {}
    for solver in (sgn.SGN_LDLT, sgn.SGN_BICGSTAB):
        ctx = sgn.Context(prob, sgn.default_options(solver=solver, eps_x=1e-6, eps_lambda=1e-6)
                          if solver == sgn.SGN_BICGSTAB else sgn.default_options()).allocate()
        p = _cuda(prob.p_init())
        x = _cuda(prob.x_rest())
        ctx.equilibrium(p, x)
        tr = [ctx.step(p, x) for _ in range(3)]
        res[solver] = ([(i.alpha, i.f1) for i in tr], _host(p))
    (t0, p0), (t1, p1) = res[sgn.SGN_LDLT], res[sgn.SGN_BICGSTAB]
    assert [a for a, _ in t0] == [a for a, _ in t1]
    assert np.allclose([f for _, f in t0], [f for _, f in t1], rtol=1e-9)
    assert np.linalg.norm(p1 - p0) <= 1e-8 * np.linalg.norm(p0)


def test_invalid_bicgstab_options_are_rejected():
    prob, *_ = _case("tiny")
    with pytest.raises(sgn.SgnError):
        sgn.Context(prob, sgn.default_options(solver=sgn.SGN_BICGSTAB, max_bicgstab=0))
    with pytest.raises(sgn.SgnError):
        sgn.Context(prob, sgn.default_options(solver=7))
    with pytest.raises(sgn.SgnError):
        sgn.Context(prob, sgn.default_options(eps_x=-1.0))
