"""The allocation-free solve (sgn_solve_static, C ABI) against sgn_solve on the same factor.

Two calls in a row share the library's static scratch array: first the 21 x 21 grid, then the
smaller 4 x 4 grid, each compared with sgn_solve of its own context to the solve tolerance's
consequence for the solution (and both with the oracle's dense Gauss-Newton step); a system whose
solve needs more than the array holds is rejected with SGN_E_NOMEM before any device work.
"""
import ctypes as C

import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_03285_amd import sgn  # noqa: E402


def _cuda(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _factored(prob, precision):
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged
    ctx = sgn.Context(prob, sgn.default_options(precision=precision, newton_rtol=1e-11)).allocate()
    N = 2 * prob.n_x + prob.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
    xd, pd = _cuda(x), _cuda(p)
    ctx.equilibrium(pd, xd)  # at the oracle's equilibrium: leaves the Kx factor the adjoint form needs
    ctx.assemble(xd, pd, rhs)
    ctx.factor()
    return ctx, rhs, D.dense_gn_step(prob, x, p)


@pytest.mark.parametrize("precision", [sgn.SGN_FP64, sgn.SGN_FP32_IR])
def test_static_solve_matches_solve_on_two_calls(precision):
    lib = sgn.load_library()
    for prob in (D.setup_targets(si.config_2d()), D.setup_targets(si.config_tiny())):  # second one smaller
        ctx, rhs, st = _factored(prob, precision)
        N = 2 * prob.n_x + prob.n_p
        ref = torch.zeros(N, dtype=torch.float64, device="cuda")
        ctx.solve(rhs, ref)
        # NaN in the output buffer: every entry must be written by the call
        out = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
        info = sgn.sgn_solve_info()
        st_code = lib.sgn_solve_static(ctx.h, C.c_void_p(rhs.data_ptr()), C.c_void_p(out.data_ptr()), C.byref(info))
        assert st_code == sgn.SGN_OK, ctx.last_error()
        assert info.rel_res <= 1e-10 and info.gmres_iters == 0
        got, want = _host(out), _host(ref)
        assert np.all(np.isfinite(got))
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
        dp = got[prob.n_x:prob.n_x + prob.n_p]
        tol = 1e-9 if precision == sgn.SGN_FP64 else 1e-8
        assert np.linalg.norm(dp - st.dp) <= tol * np.linalg.norm(st.dp)
        # the context keeps working on its own workspace afterwards
        again = torch.zeros(N, dtype=torch.float64, device="cuda")
        ctx.solve(rhs, again)
        assert np.array_equal(_host(again), want)


def test_static_solve_rejects_a_system_beyond_the_array():
    probs = si.batch_problems(256)
    for q in probs:
        q.length_scale = 1.0
        q.target_val = q.x_rest()[q.target_dof]
    u = si.union_problem(probs)  # N = 1,330,780: its solve needs about 163 MB of scratch
    ctx = sgn.Context(u, sgn.default_options()).allocate()
    N = 2 * u.n_x + u.n_p
    v = torch.zeros(N, dtype=torch.float64, device="cuda")
    info = sgn.sgn_solve_info()
    st = sgn.load_library().sgn_solve_static(ctx.h, C.c_void_p(v.data_ptr()), C.c_void_p(v.data_ptr()), C.byref(info))
    assert st == sgn.SGN_E_NOMEM
    assert "bytes of scratch" in ctx.last_error()
