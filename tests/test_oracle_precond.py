"""Pins of the oracle's node-block preconditioner (CPU only).

Each check is fixed by linear algebra rather than by re-running the oracle's
formula: the factor reproduces the equilibrated, permuted matrix; pivots stay in
their node group; Sylvester's law fixes the inertia; with zero corrections the
preconditioned matrix squares to the identity; every correction keeps M
symmetric positive definite; a uniform correction scales M by exp(2c); the 2x2
eigen-convention yields eigenpairs, larger eigenvalue first; complex-step
gradients agree with central differences.
"""
import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D
from oracle import precond as PC


def _state(prob):
    prob = D.setup_targets(prob)
    p = prob.p_init() + 0.05 * np.random.default_rng(7).standard_normal(prob.n_p)
    x, info = D.equilibrium(prob, p)
    assert info.converged
    return prob, x, p


@pytest.fixture(scope="module", params=["tiny", "loge3d", "rest3d"])
def case(request):
    mk = {"tiny": si.config_tiny,
          "loge3d": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=2),
          "rest3d": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=1, param_kind=si.P_REST_POS)}[request.param]
    prob, x, p = _state(mk())
    K = PC.sgn_matrix(prob, x, p)
    return prob, x, p, K, PC.Preconditioner(prob, K)


def _rand_corr(prob, rng, scale=0.3):
    nb = 2 * prob.dim
    cn = scale * rng.standard_normal(prob.n_nodes * nb * (nb + 1) // 2)
    cp = scale * rng.standard_normal(prob.n_p)
    return cn, cp


def test_factor_reproduces_matrix_and_groups(case):
    prob, x, p, K, P = case
    Kn = K[np.ix_(P.perm, P.perm)]
    A = P.S[:, None] * Kn * P.S[None, :]
    rec = P.L @ P.D @ P.L.T
    # componentwise backward error against |L| |D| |L|^T (restricted pivoting does not bound |L|)
    bound = np.abs(P.L) @ np.abs(P.D) @ np.abs(P.L).T
    assert np.all(np.abs(rec - A[np.ix_(P.piv, P.piv)]) <= 1e-11 * bound + 1e-15)
    # every pivot position holds a variable of its own node group
    grp = np.repeat(np.arange(len(P.nodes)), np.diff(P.starts))
    assert np.array_equal(grp[P.piv], grp)
    # |K_ij| S_i S_j <= sqrt(|K_ij| / max_k |K_ik|) sqrt(|K_ij| / max_k |K_kj|) <= 1
    assert np.abs(A).max() <= 1.0 + 1e-15
    # the saddle point needs 2x2 pivots somewhere
    assert np.any(P.kinds == 1)


def test_inertia_is_sylvester(case):
    prob, x, p, K, P = case
    assert P.inertia() == (prob.n_x + prob.n_p, prob.n_x, 0)


def test_zero_correction_squares_to_identity(case):
    prob, x, p, K, P = case
    # M^-1 K = S P^T L^-T |D|^-1 D L^T P S^-1: similar to |D|^-1 D, whose eigenvalues are +-1
    ev = np.linalg.eigvals(P.apply(K))
    assert np.allclose(np.abs(ev), 1.0, atol=1e-6)
    assert np.sum(ev.real > 0) == prob.n_x + prob.n_p and np.sum(ev.real < 0) == prob.n_x
    # the dense M and the factored application agree on a well-scaled vector
    v = np.random.default_rng(5).standard_normal(K.shape[0])
    Mv = P.matrix() @ P.apply(v)
    assert np.linalg.norm(Mv - v) <= 1e-6 * np.linalg.norm(v)


def test_corrections_keep_spd_and_uniform_scales(case):
    prob, x, p, K, P = case
    rng = np.random.default_rng(3)
    cn, cp = _rand_corr(prob, rng)
    M = P.matrix(cn, cp)
    assert np.allclose(M, M.T, atol=1e-10 * np.abs(M).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    # uniform corrections: C = exp(c) I, so M = exp(2c) M_0
    c = 0.37
    nb = 2 * prob.dim
    tri = nb * (nb + 1) // 2
    cn_u = np.zeros(prob.n_nodes * tri)
    for v in range(prob.n_nodes):
        for i in range(nb):
            cn_u[v * tri + i * (i + 1) // 2 + i] = c
    cp_u = np.full(prob.n_p, c)
    assert np.allclose(P.matrix(cn_u, cp_u), np.exp(2 * c) * P.matrix(), rtol=1e-10,
                       atol=1e-12 * np.abs(M).max())


def test_eig2_convention():
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, b, e = rng.standard_normal(3) * np.exp(rng.uniform(-3, 3))
        Q, lam = PC.eig2(a, b, e)
        A = np.array([[a, b], [b, e]])
        assert np.allclose(A @ Q, Q * lam[None, :], atol=1e-12 * np.abs(A).max())
        assert lam[0] >= lam[1] - 1e-12 * np.abs(A).max()
        assert np.allclose(Q.T @ Q, np.eye(2), atol=1e-14)
    # b = 0 keeps the axes
    Q, lam = PC.eig2(-2.0, 0.0, 5.0)
    assert np.allclose(np.abs(Q), [[0, 1], [1, 0]]) and np.allclose(lam, [5.0, -2.0])


def test_bilinear_gradient_matches_central_differences(case):
    prob, x, p, K, P = case
    rng = np.random.default_rng(11)
    cn, cp = _rand_corr(prob, rng, 0.2)
    ya = P.forward(rng.standard_normal(K.shape[0]))
    yb = P.forward(rng.standard_normal(K.shape[0]))
    gn, gp = P.bilinear_grad(ya, yb, cn, cp)
    h = 1e-6
    nb = 2 * prob.dim
    tri = nb * (nb + 1) // 2
    v = int(P.nodes[len(P.nodes) // 2])
    for t in (0, 1, tri - 1):
        i = v * tri + t
        cp_ = cn.copy()
        cp_[i] += h
        cm_ = cn.copy()
        cm_[i] -= h
        fd = (P.bilinear(ya, yb, cp_, cp) - P.bilinear(ya, yb, cm_, cp)) / (2 * h)
        assert abs(fd - gn[i]) <= 1e-6 * max(1.0, abs(fd))
    for i in (0, prob.n_p - 1):
        pp = cp.copy()
        pp[i] += h
        pm = cp.copy()
        pm[i] -= h
        fd = (P.bilinear(ya, yb, cn, pp) - P.bilinear(ya, yb, cn, pm)) / (2 * h)
        assert abs(fd - gp[i]) <= 1e-6 * max(1.0, abs(fd))
    # nodes without a group (fixed) get no gradient
    fixed = np.nonzero(prob.fixed)[0]
    if fixed.size:
        assert np.all(gn.reshape(prob.n_nodes, tri)[fixed] == 0)


def test_block_diagonal_ablation(case):
    """The block-diagonal preconditioner without a reference factor: |B_i|^2 = B_i^2 and |B_i| is
    positive definite for every group (the eigen-absolute value), M is SPD, apply() is M^-1, and on a
    matrix that is block diagonal over the groups M^-1 K has only the eigenvalues +-1."""
    prob, x, p, K, _ = case
    bp = PC.BlockDiagonalPreconditioner(prob, K)
    perm = bp.perm
    Kn = K[np.ix_(perm, perm)]
    Ks = bp.S[:, None] * Kn * bp.S[None, :]
    for g in range(len(bp.blocks)):
        a, b = bp.blocks[g][:2]
        Bg = Ks[a:b, a:b]
        Ag = bp.abs_block(g)
        assert np.allclose(Ag @ Ag, Bg @ Bg, rtol=0, atol=1e-12 * max(1.0, np.abs(Bg).max() ** 2))
        assert np.linalg.eigvalsh(Ag).min() > 0
    M = bp.matrix()
    assert np.allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())
    assert np.linalg.eigvalsh(M).min() > 0
    rng = np.random.default_rng(3)
    v = rng.standard_normal(K.shape[0])
    z = bp.apply(v)
    assert np.linalg.norm(M @ z - v) <= 1e-13 * np.linalg.norm(M, 2) * np.linalg.norm(z)
    # K restricted to the group blocks (in new order) gives M^-1 K = blockdiag(|B_i|^-1 B_i): +-1
    Kb = np.zeros_like(Kn)
    for a, b, _, _ in bp.blocks:
        Kb[a:b, a:b] = Kn[a:b, a:b]
    Ku = np.zeros_like(Kb)
    Ku[np.ix_(perm, perm)] = Kb
    bp2 = PC.BlockDiagonalPreconditioner(prob, Ku)
    ev = np.linalg.eigvals(np.linalg.solve(bp2.matrix(), Ku))
    assert np.allclose(np.abs(ev.real), 1.0, atol=1e-8) and np.allclose(ev.imag, 0.0, atol=1e-8)
