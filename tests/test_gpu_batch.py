"""GPU parity of the batched form: a disjoint union of independent 2D problems in one context,
its level-batched factorisation, and the step captured into a HIP graph and replayed.

Every problem's dp block of the union's step must equal that problem's own dense Gauss-Newton step
from the oracle (Theorem 1 of Appendix A; the KKT right-hand side of the graph step gives the same dp,
Appendix A, Theorem 2).  The problems share one length scale ell (the batch's), which the oracle uses
too.  Graph replays are checked against the eager path, with eager work between replays.
"""
import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_03285_amd import sgn  # noqa: E402


def _d(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _h(t):
    return t.detach().cpu().numpy()


_BATCH = {}


def _batch(count=6, lo=5, hi=9):
    key = (count, lo, hi)
    if key not in _BATCH:
        probs = [D.setup_targets(q) for q in si.batch_problems(count, base_seed=10000, lo=lo, hi=hi)]
        ell = max(q.length_scale for q in probs)
        for q in probs:
            q.length_scale = ell
        u = si.union_problem(probs)
        refs = []
        for q in probs:
            p0 = q.p_init()
            x0, info = D.equilibrium(q, p0, rtol=1e-11)
            assert info.converged
            refs.append((x0, D.dense_gn_step(q, x0, p0).dp))
        _BATCH[key] = (probs, u, refs)
    return _BATCH[key]


def _offsets(probs):
    return np.concatenate([[0], np.cumsum([q.n_p for q in probs])]), np.concatenate([[0], np.cumsum([q.n_x for q in probs])])


@pytest.mark.parametrize("precision", [sgn.SGN_FP64, sgn.SGN_FP32_IR])
def test_union_step_matches_each_problem(precision):
    probs, u, refs = _batch()
    ctx = sgn.Context(u, sgn.default_options(precision=precision, rhs_kind=sgn.SGN_RHS_KKT)).allocate()
    p = _d(u.p_init())
    x = _d(np.concatenate([r[0] for r in refs]))
    N = 2 * u.n_x + u.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.assemble(x, p, rhs)
    ctx.factor()
    ctx.solve(rhs, sol)
    dp = _h(sol)[u.n_x:u.n_x + u.n_p]
    po, _ = _offsets(probs)
    for i, (q, (x0, dref)) in enumerate(zip(probs, refs)):
        got = dp[po[i]:po[i + 1]]
        assert np.linalg.norm(got - dref) <= 1e-8 * np.linalg.norm(dref), q.name


@pytest.mark.parametrize("precision", [sgn.SGN_FP64, sgn.SGN_FP32_IR])
def test_large_union_one_wavefront_forms_match_each_problem(precision):
    """96 membranes of 8..16 nodes per side: the union's leaf level has 1,670 one-panel fronts with
    at most 128 rows below the pivots and 1,358 panels of at most 32 columns (host analysis of this
    union), past the 1,024 from which the solves take one wavefront per front and the narrow panels
    one wavefront each, so both forms run here (the smaller unions above keep the level kernels).
    Every problem's dp must still be its own dense Gauss-Newton step, and the solve's residual
    small."""
    probs, u, refs = _batch(96, 8, 16)
    ctx = sgn.Context(u, sgn.default_options(precision=precision, rhs_kind=sgn.SGN_RHS_KKT)).allocate()
    p = _d(u.p_init())
    x = _d(np.concatenate([r[0] for r in refs]))
    N = 2 * u.n_x + u.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.assemble(x, p, rhs)
    fi = ctx.factor()
    assert (fi.n_pos, fi.n_neg, fi.n_zero) == (u.n_x + u.n_p, u.n_x, 0)
    info = ctx.solve(rhs, sol)
    assert info.rel_res <= 1e-10
    dp = _h(sol)[u.n_x:u.n_x + u.n_p]
    po, _ = _offsets(probs)
    tol = 1e-9 if precision == sgn.SGN_FP64 else 1e-8
    for i, (q, (x0, dref)) in enumerate(zip(probs, refs)):
        got = dp[po[i]:po[i + 1]]
        assert np.linalg.norm(got - dref) <= tol * np.linalg.norm(dref), q.name


@pytest.mark.parametrize("precision", [sgn.SGN_FP64, sgn.SGN_FP32_IR])
def test_graph_step_replays_match_eager(precision):
    probs, u, refs = _batch()
    o = sgn.default_options(precision=precision, rhs_kind=sgn.SGN_RHS_KKT)
    ctx = sgn.Context(u, o).allocate()
    eager = sgn.Context(u, o).allocate()
    x = _d(np.concatenate([r[0] for r in refs]))
    p = _d(u.p_init())
    N = 2 * u.n_x + u.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    erhs = torch.zeros_like(rhs)
    esol = torch.zeros_like(sol)
    n_ir = 0 if precision == sgn.SGN_FP64 else 3
    po, _ = _offsets(probs)
    first = None
    for rep in range(4):
        # between replays: eager work on other buffers, a synchronisation, and (from the third
        # replay on) new parameter values behind the same pointer
        if rep == 2:
            p.add_(0.01)
        rel = ctx.graph_step(x, p, rhs, sol, n_ir)
        eager.assemble(x, p, erhs)
        eager.factor()
        eager.solve(erhs, esol)
        torch.cuda.synchronize()
        assert rel <= 1e-10
        assert np.array_equal(_h(rhs), _h(erhs))
        assert np.linalg.norm(_h(sol) - _h(esol)) <= 1e-9 * np.linalg.norm(_h(esol))
        if rep == 0:
            first = _h(sol).copy()
            dp = first[u.n_x:u.n_x + u.n_p]
            for i, (q, (x0, dref)) in enumerate(zip(probs, refs)):
                assert np.linalg.norm(dp[po[i]:po[i + 1]] - dref) <= 1e-8 * np.linalg.norm(dref)
        elif rep == 1:
            assert np.array_equal(_h(sol), first)  # a replay is bitwise the first run
        else:
            assert not np.array_equal(_h(sol), first)  # new p: a new step


def test_component_validation():
    probs, u, refs = _batch()
    bad = si.union_problem(probs)
    bad.components = bad.components.copy()
    bad.components[1] += 1  # an element now spans two components
    with pytest.raises(sgn.SgnError):
        sgn.Context(bad, sgn.default_options())


def test_graph_is_recaptured_after_new_targets_or_workspace():
    """The captured step holds ell and mu by value and every workspace address: after sgn_set_targets
    or sgn_set_workspace the next graph step must be captured anew and equal the eager step.  Both
    contexts get the same new targets (the eager one needs no recapture)."""
    probs, u, refs = _batch()
    o = sgn.default_options(precision=sgn.SGN_FP32_IR, rhs_kind=sgn.SGN_RHS_KKT)
    ctx = sgn.Context(u, o).allocate()
    eager = sgn.Context(u, o).allocate()
    x = _d(np.concatenate([r[0] for r in refs]))
    p = _d(u.p_init())
    N = 2 * u.n_x + u.n_p
    rhs, sol = (torch.zeros(N, dtype=torch.float64, device="cuda") for _ in range(2))
    erhs, esol = (torch.zeros(N, dtype=torch.float64, device="cuda") for _ in range(2))

    def check():
        rel = ctx.graph_step(x, p, rhs, sol, 3)
        eager.assemble(x, p, erhs)
        eager.factor()
        eager.solve(erhs, esol)
        torch.cuda.synchronize()
        assert rel <= 1e-10
        assert np.array_equal(_h(rhs), _h(erhs))
        assert np.linalg.norm(_h(sol) - _h(esol)) <= 1e-9 * np.linalg.norm(_h(esol))
        return _h(sol).copy()

    first = check()
    # new targets and a new length scale on both contexts: a stale graph would keep the old ell and mu
    tv = u.target_val + 0.1 * u.length_scale
    for c in (ctx, eager):
        c.set_targets(tv, 2.0 * u.length_scale)
    second = check()
    assert not np.array_equal(first, second)
    # a new workspace (the old one stays allocated, so nothing can touch freed memory): a stale graph
    # would run in the old workspace while the call reads the residual and the done flag from the new
    old_ws = ctx.workspace
    ctx.allocate()
    third = check()
    assert np.linalg.norm(third - second) <= 1e-9 * np.linalg.norm(second)
    del old_ws


def test_batch_create_builds_the_union():
    """sgn_batch_create gives the same system as the union built by hand: same symbolic structure,
    bitwise the same assembled values and step."""
    probs, u, refs = _batch()
    o = sgn.default_options(precision=sgn.SGN_FP32_IR, rhs_kind=sgn.SGN_RHS_KKT)
    a = sgn.Context.from_batch(probs, o).allocate()
    b = sgn.Context(u, o).allocate()
    for s1, s2 in zip(a.symbolic(), b.symbolic()):
        assert np.array_equal(s1, s2)
    x = _d(np.concatenate([r[0] for r in refs]))
    p = _d(u.p_init())
    N = 2 * u.n_x + u.n_p
    out = []
    for ctx in (a, b):
        rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
        sol = torch.zeros(N, dtype=torch.float64, device="cuda")
        ctx.assemble(x, p, rhs)
        ctx.factor()
        ctx.solve(rhs, sol)
        out.append((ctx.values(), _h(rhs), _h(sol)))
    for v1, v2 in zip(out[0], out[1]):
        assert np.array_equal(v1, v2)


@pytest.mark.parametrize("rhs_kind", [sgn.SGN_RHS_KKT, sgn.SGN_RHS_ADJOINT])
def test_batch_step_follows_each_problem_outer_iteration(rhs_kind):
    """Two sgn_batch_step calls: every problem's accepted step length and objective must follow its
    own oracle iterations (dense Gauss-Newton step, Armijo backtracking, at the batch's ell)."""
    probs, u, refs = _batch()
    ctx = sgn.Context.from_batch(probs, sgn.default_options(rhs_kind=rhs_kind, newton_rtol=1e-11)).allocate()
    ps = [_d(q.p_init()) for q in probs]
    xs = [_d(r[0]) for r in refs]
    infos = [ctx.batch_step(ps, xs) for _ in range(2)]
    for i, q in enumerate(probs):
        trace, p_ref, x_ref = D.sgn_iterations(q, q.p_init(), refs[i][0], iters=2)
        for it in range(2):
            f_ref, g_ref, a_ref = trace[it]
            assert infos[it][i].alpha == a_ref, (q.name, it)
            # the first step moves f by orders of magnitude: later values agree to the step's accuracy
            # relative to the starting objective
            assert infos[it][i].f0 == pytest.approx(f_ref, rel=1e-9, abs=1e-9 * trace[0][0]), (q.name, it)
        assert np.linalg.norm(_h(ps[i]) - p_ref) <= 1e-8 * max(np.linalg.norm(p_ref), 1e-12)
        u_ref = x_ref - q.x_rest()
        assert np.linalg.norm(_h(xs[i]) - x_ref) <= 1e-8 * np.linalg.norm(u_ref)
