"""Schedule blocking and its autotuner on an MI355X (through the C ABI).

The blocking (delayed-update span per front-size bucket, the sequential-solve threshold) regroups
launches and the order of the trailing update's k-sums only, so every setting must give the
oracle's Gauss-Newton step; the autotuner must return a valid setting whose step is the default
setting's.  Expected values come from ``oracle/`` only.
"""
import json

import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_03285_amd import sgn  # noqa: E402

SETTINGS = [
    {"outer_panels": [1, 1, 1], "seq_panels": -1},  # every panel's update right away, every solve pipelined
    {"outer_panels": [8, 8, 8], "seq_panels": 2},
    {"outer_panels": [2, 16, 1], "seq_panels": 8},
]


def _cuda(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _state(prob):
    prob = D.setup_targets(prob)
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged
    return prob, p, x


def _step(prob, x, p, opts):
    ctx = sgn.Context(prob, opts).allocate()
    xd, pd = _cuda(x), _cuda(p)
    ctx.equilibrium(pd, xd)
    N = 2 * prob.n_x + prob.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.assemble(xd, pd, rhs)
    ctx.factor()
    info = ctx.solve(rhs, sol)
    assert info.rel_res <= 1e-10
    return _host(xd), _host(sol)


@pytest.mark.parametrize("precision", [sgn.SGN_FP64, sgn.SGN_FP32_IR])
@pytest.mark.parametrize("k", range(len(SETTINGS)))
def test_every_blocking_gives_the_dense_gauss_newton_step(k, precision):
    # 8 x 3 x 3 cantilever: fronts of up to three panels, so spans 1, 2 and 8 regroup real updates
    prob, p, x = _state(si.problem_3d(8, 3, 3, 1 / 3, seed=2))
    opts = sgn.apply_tuning(sgn.default_options(precision=precision, newton_rtol=1e-11), SETTINGS[k])
    xg, sol = _step(prob, x, p, opts)
    st = D.dense_gn_step(prob, xg, p)
    nx, npar = prob.n_x, prob.n_p
    tol = 1e-9 if precision == sgn.SGN_FP64 else 1e-8
    assert _rel(sol[nx:nx + npar], st.dp) <= tol
    assert _rel(sol[:nx], st.dx) <= tol
    assert _rel(sol[nx + npar:], st.dlam) <= tol


def test_autotune_returns_a_valid_setting_with_the_same_step(tmp_path):
    # 20 x 5 x 5 cantilever (2,500 tets): fronts in the two lower buckets, chains long enough for
    # the pipelined solve
    prob, p, x = _state(si.problem_3d(20, 5, 5, 0.2, seed=4))
    base = sgn.default_options(precision=sgn.SGN_FP32_IR, newton_rtol=1e-11)
    xd, pd = _cuda(x), _cuda(p)
    path = tmp_path / "tuning.json"
    rec = sgn.autotune(prob, xd, pd, base, reps=1, path=str(path))
    assert rec == json.loads(path.read_text())
    assert len(rec["candidate_ms"]) == 18 and all(v > 0 for v in rec["candidate_ms"])
    assert all(v in (0, 1, 2, 4, 8, 16) for v in rec["outer_panels"])
    assert rec["seq_panels"] in (0, -1, 2, 4, 8)
    tuned = sgn.apply_tuning(sgn.default_options(precision=sgn.SGN_FP32_IR, newton_rtol=1e-11), rec)
    _, s_tuned = _step(prob, x, p, tuned)
    _, s_base = _step(prob, x, p, base)
    assert _rel(s_tuned, s_base) <= 1e-9
    # the record round-trips into options
    assert rec["panel_waves"] in (0, 4, 8)
    assert sgn.tuning_of(tuned) == {"outer_panels": rec["outer_panels"], "seq_panels": rec["seq_panels"],
                                    "panel_waves": rec["panel_waves"]}
