"""GPU parity of the node-block preconditioner and the MINRES solve (C ABI, MI355X).

Expected values come from ``oracle/precond.py`` (dense FP64 restricted-pivoting
LDL^T, the preconditioner written out, complex-step gradients) and from dense
solves of the oracle's K_SGN.  The states (x, p) are the oracle's equilibria, so
both sides factor the same matrix.  Tolerances: the restricted pivoting leaves
the factor's L badly conditioned (cond(L) reaches 1e11 on the 4x4 grid), so
element-wise comparisons of forward results scale with the oracle's estimate
cond(L) * 1e-15; the preconditioner application is also checked through its
normwise backward error on the oracle's M, which holds at any conditioning.
"""
import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D
from oracle import precond as PC

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_03285_amd import sgn  # noqa: E402


def _cuda(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _host(t):
    return t.detach().cpu().numpy().astype(np.float64)


_MK = {
    "tiny": si.config_tiny,
    "loge3x2x2": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=2),
    "rest3x2x2": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=1, param_kind=si.P_REST_POS),
}
_CASES = {}


def _case(name):
    """(prob, p, x, K, oracle preconditioner) at an oracle equilibrium with perturbed p."""
    if name not in _CASES:
        prob = D.setup_targets(_MK[name]())
        p = prob.p_init() + 0.05 * np.random.default_rng(7).standard_normal(prob.n_p)
        x, info = D.equilibrium(prob, p, rtol=1e-11)
        assert info.converged
        K = PC.sgn_matrix(prob, x, p)
        _CASES[name] = (prob, p, x, K, PC.Preconditioner(prob, K))
    return _CASES[name]


def _ctx(prob, **opt):
    return sgn.Context(prob, sgn.default_options(**opt)).allocate()


def _corr(prob, seed, scale=0.2):
    rng = np.random.default_rng(seed)
    nb = 2 * prob.dim
    cn = (scale * rng.standard_normal(prob.n_nodes * nb * (nb + 1) // 2)).astype(np.float32)
    cp = (scale * rng.standard_normal(prob.n_p)).astype(np.float32)
    return cn, cp


def _factored(name, **opt):
    prob, p, x, K, P = _case(name)
    ctx = _ctx(prob, **opt)
    ctx.assemble(_cuda(x), _cuda(p))
    ctx.factor()
    return prob, p, x, K, P, ctx


def _cond_tol(P):
    return max(1e-12, 1e-15 * np.linalg.cond(P.L))


@pytest.mark.parametrize("name", list(_MK))
def test_forward_result_matches_oracle(name):
    prob, p, x, K, P, ctx = _factored(name)
    N = K.shape[0]
    v = np.random.default_rng(1).standard_normal(N)
    fwd = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.pc_forward(_cuda(v), fwd)
    ref = P.forward(v)
    err = np.linalg.norm(_host(fwd) - ref) / np.linalg.norm(ref)
    assert err <= _cond_tol(P), err


@pytest.mark.parametrize("name", list(_MK))
@pytest.mark.parametrize("with_corr", [False, True])
def test_pc_apply_matches_oracle(name, with_corr):
    prob, p, x, K, P, ctx = _factored(name)
    N = K.shape[0]
    cn, cp = _corr(prob, 4) if with_corr else (None, None)
    if with_corr:
        dcn, dcp = _cuda(cn, torch.float32), _cuda(cp, torch.float32)
        ctx.set_pc_correction(dcn, dcp)
    v = np.random.default_rng(2).standard_normal(N)
    out = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.pc_apply(_cuda(v), out)
    z = _host(out)
    cn64 = None if cn is None else cn.astype(np.float64)
    cp64 = None if cp is None else cp.astype(np.float64)
    ref = P.apply(v, cn64, cp64)
    assert np.linalg.norm(z - ref) <= _cond_tol(P) * np.linalg.norm(ref)
    # normwise backward error on the oracle's M
    M = P.matrix(cn64, cp64)
    be = np.linalg.norm(M @ z - v) / (np.linalg.norm(M, 2) * np.linalg.norm(z) + np.linalg.norm(v))
    assert be <= 1e-13, be
    # symmetry of the applied operator: u^T M^-1 v = v^T M^-1 u
    u = np.random.default_rng(3).standard_normal(N)
    out2 = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.pc_apply(_cuda(u), out2)
    a, b = u @ z, v @ _host(out2)
    assert abs(a - b) <= 1e-9 * (abs(a) + abs(b)) + 1e-300


@pytest.mark.parametrize("name", list(_MK))
def test_pc_grad_matches_complex_step(name):
    prob, p, x, K, P, ctx = _factored(name)
    N = K.shape[0]
    cn, cp = _corr(prob, 5)
    dcn, dcp = _cuda(cn, torch.float32), _cuda(cp, torch.float32)
    ctx.set_pc_correction(dcn, dcp)
    rng = np.random.default_rng(6)
    a, b = rng.standard_normal(N), rng.standard_normal(N)
    fa = torch.zeros(N, dtype=torch.float64, device="cuda")
    fb = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.pc_forward(_cuda(a), fa)
    ctx.pc_forward(_cuda(b), fb)
    gn = torch.zeros_like(dcn)
    gp = torch.zeros_like(dcp)
    ctx.pc_grad(fa, fb, 1.0, gn, gp)
    ctx.pc_grad(fa, fb, 0.5, gn, gp)  # accumulates: 1.5 x the gradient
    rn, rp = P.bilinear_grad(P.forward(a), P.forward(b), cn.astype(np.float64), cp.astype(np.float64))
    tol = 1e-5 + 10 * _cond_tol(P)  # FP32 gradient storage
    assert np.linalg.norm(_host(gn) - 1.5 * rn) <= tol * np.linalg.norm(1.5 * rn)
    assert np.linalg.norm(_host(gp) - 1.5 * rp) <= tol * np.linalg.norm(1.5 * rp)


def _dense_solve(K, b):
    s = 1.0 / np.sqrt(np.max(np.abs(K), axis=1))
    return s * np.linalg.solve(K * s[:, None] * s[None, :], s * b)


@pytest.mark.parametrize("name", list(_MK))
@pytest.mark.parametrize("precision", [sgn.SGN_FP64, sgn.SGN_FP32_IR])
def test_minres_with_exact_reference_converges_fast(name, precision):
    prob, p, x, K, P, ctx = _factored(name, precision=precision)
    N = K.shape[0]
    b = np.random.default_rng(8).standard_normal(N)
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    info = ctx.solve_minres(_cuda(b), sol)
    assert info.fallback == 0
    assert info.rel_res <= 1e-10
    # M^-1 K has the two eigenvalues +-1 (up to the factor's rounding, amplified by cond(L))
    assert info.sweeps <= (6 if precision == sgn.SGN_FP64 else 20), info.sweeps
    ref = _dense_solve(K, b)
    assert np.linalg.norm(_host(sol) - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", list(_MK))
def test_minres_with_stale_reference_and_fallback(name):
    prob, p, x, K, P, ctx = _factored(name)
    # a later state: p moved, new equilibrium; the reference factor is the old one
    # a small move (1% of log E per element, 3% of an edge for rest positions): the old factor still
    # clusters the spectrum of M^-1 K1 (oracle: within [0.36, 2.6] on loge3x2x2); on the 4x4 grid the
    # badly conditioned factor spreads it to [0.008, 32], so MINRES may stagnate and fall back there
    p1 = p + 0.01 * np.random.default_rng(9).standard_normal(prob.n_p)
    x1, info = D.equilibrium(prob, p1, x0=x, rtol=1e-11)
    assert info.converged
    K1 = PC.sgn_matrix(prob, x1, p1)
    ctx.assemble(_cuda(x1), _cuda(p1))
    N = K.shape[0]
    b = np.random.default_rng(10).standard_normal(N)
    ref = _dense_solve(K1, b)
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    info = ctx.solve_minres(_cuda(b), sol)
    assert info.rel_res <= 1e-10
    assert info.fallback == 0 or name == "tiny"
    assert np.linalg.norm(_host(sol) - ref) <= 1e-8 * np.linalg.norm(ref)
    if info.fallback == 0:  # the direct solve refuses the stale factor
        with pytest.raises(sgn.SgnError):
            ctx.solve(_cuda(b), sol)
    else:  # the fallback factor is of the current matrix
        ctx.solve(_cuda(b), sol)
        assert np.linalg.norm(_host(sol) - ref) <= 1e-8 * np.linalg.norm(ref)
    # a one-iteration budget forces the fallback: exact factor of K1, refined solve
    ctx2 = _ctx(prob, max_minres=1)
    ctx2.assemble(_cuda(x), _cuda(p))
    ctx2.factor()
    ctx2.assemble(_cuda(x1), _cuda(p1))
    sol2 = torch.zeros(N, dtype=torch.float64, device="cuda")
    info2 = ctx2.solve_minres(_cuda(b), sol2)
    assert info2.fallback == 1 and info2.rel_res <= 1e-10
    assert np.linalg.norm(_host(sol2) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_minres_without_reference_falls_back_and_spmv_matches():
    prob, p, x, K, P = _case("loge3x2x2")
    ctx = _ctx(prob)
    ctx.assemble(_cuda(x), _cuda(p))
    N = K.shape[0]
    v = np.random.default_rng(12).standard_normal(N)
    out = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.spmv(_cuda(v), out)
    assert np.linalg.norm(_host(out) - K @ v) <= 1e-13 * np.linalg.norm(K @ v)
    with pytest.raises(sgn.SgnError):
        _ctx(prob).pc_apply(_cuda(v), out)  # no reference factor
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    info = ctx.solve_minres(_cuda(v), sol)
    assert info.fallback == 1
    assert np.linalg.norm(_host(sol) - _dense_solve(K, v)) <= 1e-8 * np.linalg.norm(_dense_solve(K, v))


def test_outer_iterations_with_minres_match_direct():
    """Three SGN iterations: MINRES (reference = the last exact factor, refreshed on fallback) against
    the direct solver: same step lengths and iterates."""
    prob = D.setup_targets(si.problem_3d(4, 2, 2, 0.25, seed=1))
    traces = {}
    for solver in (sgn.SGN_LDLT, sgn.SGN_MINRES_LEARNED):
        ctx = _ctx(prob, solver=solver)
        p = _cuda(prob.p_init())
        x = _cuda(prob.x_rest())
        ctx.equilibrium(p, x)
        tr = []
        for _ in range(3):
            info = ctx.step(p, x)
            tr.append((info.alpha, info.f1, info.solve.fallback))
        traces[solver] = (tr, _host(p))
    (t0, p0), (t1, p1) = traces[sgn.SGN_LDLT], traces[sgn.SGN_MINRES_LEARNED]
    assert [a for a, _, _ in t0] == [a for a, _, _ in t1]
    assert t1[0][2] == 1  # no reference before the first step
    assert np.allclose([f for _, f, _ in t0], [f for _, f, _ in t1], rtol=1e-8)
    assert np.linalg.norm(p1 - p0) <= 1e-8 * np.linalg.norm(p0)


def test_training_loss_and_gradient_match_oracle():
    """The library's training loss and its weight gradient against the oracle (complex step)."""
    from oracle import gnn as G
    prob, p, x, K, P, ctx = _factored("loge3x2x2")
    p1 = p + 0.01 * np.random.default_rng(9).standard_normal(prob.n_p)
    x1, info = D.equilibrium(prob, p1, x0=x, rtol=1e-11)
    assert info.converged
    K1 = PC.sgn_matrix(prob, x1, p1)
    ctx.assemble(_cuda(x1), _cuda(p1))
    rng = np.random.default_rng(21)
    w = (0.05 * rng.standard_normal(ctx.gnn_num_weights())).astype(np.float32)
    probes = rng.standard_normal((2, K.shape[0]))
    wd = _cuda(w, torch.float32)
    gw = torch.zeros_like(wd)
    loss = ctx.pc_train_loss(wd, _cuda(probes), gw)
    state = (x, p, x1, p1, prob.length_scale)
    ref = G.train_loss(prob, P, K1, w.astype(np.float64), state, probes)
    assert abs(loss - ref) <= 1e-3 * ref
    u = rng.standard_normal(w.size)
    h = 1e-30
    dd = G.train_loss(prob, P, K1, w.astype(np.float64) + 1j * h * u, state, probes).imag / h
    g = _host(gw)
    assert abs(g @ u - dd) <= 2e-3 * np.sum(np.abs(g * u)) + 1e-3 * abs(dd)
    # the network's corrections drive MINRES when the weights are set
    ctx.set_pc_weights(wd)
    b = rng.standard_normal(K.shape[0])
    sol = torch.zeros(K.shape[0], dtype=torch.float64, device="cuda")
    info = ctx.solve_minres(_cuda(b), sol)
    assert info.rel_res <= 1e-10
    ref_sol = _dense_solve(K1, b)
    assert np.linalg.norm(_host(sol) - ref_sol) <= 1e-8 * np.linalg.norm(ref_sol)


def test_trained_network_gain_on_held_out_pairs(capsys):
    """What the trained network gains: a small logged set (SGN runs on a 12 x 3 x 3 cantilever, the
    reference factor at iterate k and the matrix a fraction t along the step to k + 1), a few epochs of
    the library's own training (network forward/backward, spectral loss, Adam on the GPU), then on a
    held-out seed the spectral loss and the MINRES iterations and fallbacks with and without the
    network.  Training must lower the held-out loss; every solve, with or without the network, must
    reach the tolerance (MINRES or its exact fallback); the iteration and fallback counts are the gain,
    reported whatever their sign."""
    from paper_2107_03285_amd import learned_pc as LP
    mesh = [(12, 3, 3, 1 / 3)]
    train = LP.build_pairs(mesh, [0, 1], 3, "cuda", fractions=(0.05, 0.25))
    held = LP.build_pairs(mesh, [1000], 3, "cuda", fractions=(0.05, 0.25))
    assert len(train) >= 4 and len(held) >= 2
    tr = LP.Trainer(train[0][0], seed=0, lr=1e-3)

    def held_loss():
        r = np.random.default_rng(12345)
        return float(np.exp(np.mean([np.log(tr.loss(p, a, b, nprobe=4, accumulate=False, rng=r))
                                     for p, a, b, _ in held])))

    before = held_loss()
    base = [tr.minres_iterations(p, a, b, False) for p, a, b, _ in held]
    rng = np.random.default_rng(0)
    for _ in range(6):
        for i in rng.permutation(len(train)):
            p, a, b, _ = train[i]
            tr.loss(p, a, b, nprobe=2)
            tr.step()
    after = held_loss()
    net = [tr.minres_iterations(p, a, b, True) for p, a, b, _ in held]
    with capsys.disabled():
        print(f"\n[learned-PC gain] held-out spectral loss {before:.4f} -> {after:.4f}; MINRES iterations "
              f"without / with the network per pair: {[(w0[0], w1[0]) for w0, w1 in zip(base, net)]}; fallbacks "
              f"{sum(w[1] for w in base)} -> {sum(w[1] for w in net)} of {len(held)}")
    assert after < before
    for iters, fb, rel in base + net:
        assert rel <= 1e-10


@pytest.mark.parametrize("name", list(_MK))
def test_block_diagonal_pc_matches_oracle(name):
    """The block-diagonal ablation (pc_kind = SGN_PC_BLOCK: |B_i|^-1 of the node groups' diagonal blocks
    of the current equilibrated matrix, no reference factor) against the oracle's eigendecomposition."""
    prob, p, x, K, P = _case(name)
    ctx = _ctx(prob, pc_kind=sgn.SGN_PC_BLOCK)
    ctx.assemble(_cuda(x), _cuda(p))
    bp = PC.BlockDiagonalPreconditioner(prob, K)
    N = K.shape[0]
    v = np.random.default_rng(5).standard_normal(N)
    out = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.pc_apply(_cuda(v), out)
    z = _host(out)
    ref = bp.apply(v)
    # two eigensolvers agree on |B_i|^-1 to the conditioning of the blocks (the smallest eigenvalues
    # carry an absolute error near eps |B_i|)
    kappa = max(np.abs(lam).max() / np.abs(lam).min() for _, _, _, lam in bp.blocks)
    assert np.linalg.norm(z - ref) <= max(1e-12, 1e-15 * kappa) * np.linalg.norm(ref)
    M = bp.matrix()
    be = np.linalg.norm(M @ z - v) / (np.linalg.norm(M, 2) * np.linalg.norm(z) + np.linalg.norm(v))
    assert be <= 1e-13, be


@pytest.mark.parametrize("name", list(_MK))
def test_minres_with_block_diagonal_pc_solves_or_falls_back(name):
    """MINRES preconditioned by the block-diagonal ablation: whichever way the solve ends (MINRES to the
    tolerance, or the exact factorisation after stagnation), the step solves the oracle's system."""
    prob, p, x, K, P = _case(name)
    ctx = _ctx(prob, pc_kind=sgn.SGN_PC_BLOCK, solve_rtol=1e-10, rhs_kind=sgn.SGN_RHS_KKT)
    N = K.shape[0]
    rhs = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.assemble(_cuda(x), _cuda(p), rhs)
    sol = torch.zeros(N, dtype=torch.float64, device="cuda")
    info = ctx.solve_minres(rhs, sol)
    z = _host(sol)
    b = _host(rhs)
    ref = np.linalg.solve(K, b)
    assert np.linalg.norm(z - ref) <= 1e-8 * np.linalg.norm(ref)
    assert info.fallback in (0, 1) and info.sweeps >= 1
