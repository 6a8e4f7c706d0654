"""The factorisation reads no workspace memory it has not written (on an MI355X, through the C ABI).

Each factorisation zeroes only the fronts' lower triangles and a band above the diagonal, and the
trailing update of a block runs partly on a second stream beside the next block's panels.  A
workspace filled with NaN bytes before set-up must therefore give bitwise the step of a zeroed one:
any read of an entry that was never written would turn the result into NaN.
"""
import ctypes as C

import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_03285_amd import sgn  # noqa: E402


def _context(prob, opts, fill_byte):
    ctx = sgn.Context(prob, opts)
    nbytes = ctx.workspace_size()
    ws = torch.full((nbytes + 256,), fill_byte, dtype=torch.uint8, device="cuda")
    aligned = (int(ws.data_ptr()) + 255) & ~255
    ctx._check(ctx.lib.sgn_set_workspace(ctx.h, C.c_void_p(aligned), C.c_size_t(nbytes)))
    ctx.workspace = ws
    return ctx


def _step(prob, x, p, opts, fill_byte):
    ctx = _context(prob, opts, fill_byte)
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    N = 2 * prob.n_x + prob.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.assemble(xd, pd, rhs)
    ctx.factor()
    info = ctx.solve(rhs, sol)
    assert info.rel_res <= 1e-10
    return sol.cpu().numpy()


PROBLEMS = {
    "cant8x3x3": (lambda: si.problem_3d(8, 3, 3, 1 / 3, seed=2), None),
    # one-panel delayed-update spans: every block's update splits into the next block's columns and the
    # columns beyond, the latter on the second stream beside the next panels
    "cant20x5x5_span1": (lambda: si.problem_3d(20, 5, 5, 0.2, seed=4), {"outer_panels": [1, 1, 1], "seq_panels": 0}),
}


@pytest.mark.parametrize("precision", [sgn.SGN_FP64, sgn.SGN_FP32_IR])
@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_nan_filled_workspace_gives_the_zeroed_step_bitwise(name, precision):
    mk, tuning = PROBLEMS[name]
    prob = D.setup_targets(mk())
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged
    opts = sgn.default_options(precision=precision, rhs_kind=sgn.SGN_RHS_KKT)
    if tuning:
        opts = sgn.apply_tuning(opts, tuning)
    zeroed = _step(prob, x, p, opts, 0)
    nan_filled = _step(prob, x, p, opts, 0xFF)
    assert np.all(np.isfinite(nan_filled))
    assert np.array_equal(zeroed, nan_filled)


def _outer_step(prob, opts, fill_byte):
    ctx = _context(prob, opts, fill_byte)
    p = torch.tensor(prob.p_init(), dtype=torch.float64, device="cuda")
    x = torch.tensor(prob.x_rest(), dtype=torch.float64, device="cuda")
    ctx.equilibrium(p, x)
    info = ctx.step(p, x)
    return info.alpha, info.halvings, info.f1, p.cpu().numpy(), x.cpu().numpy()


@pytest.mark.parametrize("rhs_kind", [sgn.SGN_RHS_ADJOINT, sgn.SGN_RHS_KKT])
def test_prefilled_workspace_gives_the_zeroed_outer_step_bitwise(rhs_kind):
    """The outer iteration from rest (Newton equilibria with their Kx factorisations, the step, the
    backtracking trials) reads nothing it has not written either: workspaces prefilled with NaN bytes
    or with a finite pattern give bitwise the iterate of a zeroed one."""
    prob = D.setup_targets(si.problem_3d(4, 2, 2, 0.25, seed=1))
    opts = sgn.default_options(rhs_kind=rhs_kind)
    ref = _outer_step(prob, opts, 0)
    for fill in (0xFF, 0x40):
        got = _outer_step(prob, opts, fill)
        assert got[:3] == ref[:3], (fill, got[:3], ref[:3])
        assert np.array_equal(got[3], ref[3]) and np.array_equal(got[4], ref[4])
