"""Pins of the oracle's preconditioner network (CPU only).

Zero decoders give zero corrections; a rigid translation of mesh and states
leaves the outputs unchanged; relabelling the nodes permutes the outputs the same
way; complex-step weight gradients agree with central differences; the weight
count follows the layer list.  The training loss: at the reference matrix with
zero corrections its symmetric operator squares to the identity; its spectrum is
that of M^-1 K with M assembled densely from the reference factor; the best-scale
substitution makes the loss vanish for uniform corrections and leaves it unchanged
when the matrix is scaled; its complex-step derivative agrees with central
differences.
"""
import dataclasses

import numpy as np
import pytest

import sgn_inputs as si
from oracle import gnn as G


def _setup(kind):
    prob = {"loge": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=2),
            "rest": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=1, param_kind=si.P_REST_POS),
            "tiny": si.config_tiny}[kind]()
    rng = np.random.default_rng(0)
    x_ref = prob.x_rest() + 0.01 * rng.standard_normal(prob.n_x)
    x = x_ref + 0.01 * rng.standard_normal(prob.n_x)
    p_ref = 0.1 * rng.standard_normal(prob.n_p)
    p = p_ref + 0.05 * rng.standard_normal(prob.n_p)
    w = 0.2 * rng.standard_normal(G.num_weights(prob))
    return prob, w, (x_ref, p_ref, x, p, 0.05)


@pytest.mark.parametrize("kind", ["loge", "rest", "tiny"])
def test_zero_decoder_gives_zero(kind):
    prob, w, st = _setup(kind)
    L = G.unpack(prob, w)
    for name in ("dec_node", "dec_elem"):
        Wd, bd = L[name]
        Wd[...] = 0
        bd[...] = 0
    cn, cp = G.forward(prob, w, *st)
    assert np.all(cn == 0) and np.all(cp == 0)


@pytest.mark.parametrize("kind", ["loge", "rest"])
def test_translation_invariance(kind):
    prob, w, st = _setup(kind)
    cn, cp = G.forward(prob, w, *st)
    t = np.array([0.3, -1.7, 2.5])[:prob.dim]
    moved = dataclasses.replace(prob, rest_pos=prob.rest_pos + t)
    x_ref, p_ref, x, p, ell = st
    shift = np.tile(t, prob.n_x // prob.dim)
    cn2, cp2 = G.forward(moved, w, x_ref + shift, p_ref, x + shift, p, ell)
    assert np.allclose(cn, cn2, atol=1e-12) and np.allclose(cp, cp2, atol=1e-12)


def test_node_relabelling_permutes_outputs():
    prob, w, st = _setup("loge")
    x_ref, p_ref, x, p, ell = st
    rng = np.random.default_rng(5)
    # relabel the nodes, keeping the relative order of the free nodes (so the DOF vectors keep their order)
    n = prob.n_nodes
    free = np.nonzero(~prob.fixed.astype(bool))[0]
    fixed = np.nonzero(prob.fixed.astype(bool))[0]
    new_pos = np.empty(n, dtype=np.int64)
    slots = np.sort(rng.choice(n, size=free.size, replace=False))
    new_pos[free] = slots
    new_pos[fixed] = np.setdiff1d(np.arange(n), slots)
    old_of_new = np.argsort(new_pos)
    moved = dataclasses.replace(prob, rest_pos=prob.rest_pos[old_of_new], elems=new_pos[prob.elems].astype(np.int32),
                                fixed=prob.fixed[old_of_new], f_ext=prob.f_ext[old_of_new],
                                grid=prob.grid)
    cn, cp = G.forward(prob, w, *st)
    cn2, cp2 = G.forward(moved, w, *st)
    tri = 21
    assert np.allclose(cn.reshape(n, tri)[old_of_new], cn2.reshape(n, tri), atol=1e-12)
    assert np.allclose(cp, cp2, atol=1e-12)


@pytest.mark.parametrize("kind", ["loge", "rest"])
def test_complex_step_matches_central_differences(kind):
    prob, w, st = _setup(kind)
    rng = np.random.default_rng(3)
    cn, cp = G.forward(prob, w, *st)
    gn, gp = rng.standard_normal(cn.shape), rng.standard_normal(cp.shape)
    idx = rng.choice(w.size, size=12, replace=False)
    cs = G.grad_complex_step(prob, w, gn, gp, st, idx)
    h = 1e-6
    for k, i in enumerate(idx):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (G.loss_dot(prob, wp, gn, gp, *st) - G.loss_dot(prob, wm, gn, gp, *st)) / (2 * h)
        assert abs(fd - cs[k]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, cs[k])
    u = rng.standard_normal(w.size)
    dd = G.directional_complex_step(prob, w, gn, gp, st, u)
    fd = (G.loss_dot(prob, w + h * u, gn, gp, *st) - G.loss_dot(prob, w - h * u, gn, gp, *st)) / (2 * h)
    assert abs(fd - dd) <= 1e-5 * max(1.0, abs(fd))


def test_weight_count():
    prob = si.problem_3d(3, 2, 2, 1 / 3, seed=2)
    H = 64
    expect = (9 + 1) * H + (6 + 1) * H + 3 * ((3 * H + 1) * H + (2 * H + 1) * H) + (H + 1) * 21 + (H + 1) * 1
    assert G.num_weights(prob) == expect


# ---- the training loss and its symmetric operator ------------------------------------------------
# T = (R C)^-1 L^-1 Q K Q^T L^-T (R C)^-T is similar to M^-1 K (M the preconditioner of the same
# reference factor and corrections), symmetric, and equal to R^-1 D R^-T (eigenvalues +-1) when K is
# the reference matrix and the corrections vanish.  The loss substitutes the best scale gamma, so a
# uniform correction (M -> e^{2c} M) leaves it at zero and scaling K leaves it unchanged.

from oracle import dense as D  # noqa: E402
from oracle import precond as PC  # noqa: E402


@pytest.fixture(scope="module", params=["tiny", "loge3d", "rest3d"])
def ref_case(request):
    mk = {"tiny": si.config_tiny,
          "loge3d": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=2),
          "rest3d": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=1, param_kind=si.P_REST_POS)}[request.param]
    prob = D.setup_targets(mk())
    rng = np.random.default_rng(7)
    p = prob.p_init() + 0.05 * rng.standard_normal(prob.n_p)
    x, info = D.equilibrium(prob, p)
    assert info.converged
    K = PC.sgn_matrix(prob, x, p)
    P = PC.Preconditioner(prob, K)
    # a second state near the reference one (the matrices the loss sees in training)
    p2 = p + 0.02 * rng.standard_normal(prob.n_p)
    x2, info2 = D.equilibrium(prob, p2)
    assert info2.converged
    K2 = PC.sgn_matrix(prob, x2, p2)
    return prob, x, p, K, P, x2, p2, K2


def _tri(prob):
    nb = 2 * prob.dim
    return nb * (nb + 1) // 2


def _uniform_weights(prob, c):
    """Network weights whose corrections are exactly c on every diagonal position and 0 elsewhere."""
    w = np.zeros(G.num_weights(prob))
    L = G.unpack(prob, w)
    nb = 2 * prob.dim
    _, bn = L["dec_node"]
    for i in range(nb):
        bn[i * (i + 1) // 2 + i] = c
    if prob.param_kind == si.P_LOGE:
        L["dec_elem"][1][:] = c
    else:
        bn[_tri(prob):] = c
    return w


def test_symmetric_operator_at_reference_squares_to_identity(ref_case):
    prob, x, p, K, P, *_ = ref_case
    n = K.shape[0]
    T = G.symmetric_operator(prob, P, K, np.zeros(prob.n_nodes * _tri(prob)), np.zeros(prob.n_p))
    # T = R^-1 D R^-T: block diagonal with eigenvalues exactly +-1, so T^2 = I up to cond(L) rounding
    assert np.abs(T - T.T).max() <= 1e-9
    assert np.abs(T @ T - np.eye(n)).max() <= 1e-8
    ev = np.linalg.eigvalsh(0.5 * (T + T.T))
    assert np.sum(ev > 0) == prob.n_x + prob.n_p and np.sum(ev < 0) == prob.n_x


def test_symmetric_operator_spectrum_is_that_of_preconditioned_matrix(ref_case):
    prob, x, p, K, P, x2, p2, K2 = ref_case
    rng = np.random.default_rng(11)
    cn = 0.3 * rng.standard_normal(prob.n_nodes * _tri(prob))
    cp = 0.3 * rng.standard_normal(prob.n_p)
    T = G.symmetric_operator(prob, P, K2, cn, cp)
    scale = np.abs(T).max()
    assert np.abs(T - T.T).max() <= 1e-9 * scale
    ev_t = np.sort(np.linalg.eigvalsh(0.5 * (T + T.T)))
    # M assembled densely from the reference factor (L B L^T, B = R C C^T R^T), then M^-1 K directly
    M = P.matrix(cn, cp)
    ev_m = np.linalg.eigvals(np.linalg.solve(M, K2))
    assert np.abs(ev_m.imag).max() <= 1e-6 * np.abs(ev_m).max()   # similar to a symmetric matrix
    ev_m = np.sort(ev_m.real)
    assert np.abs(ev_t - ev_m).max() <= 1e-6 * np.abs(ev_t).max(), np.abs(ev_t - ev_m).max()


def test_train_loss_vanishes_at_reference_for_uniform_corrections(ref_case):
    prob, x, p, K, P, *_ = ref_case
    rng = np.random.default_rng(2)
    probes = [rng.standard_normal(K.shape[0]) for _ in range(3)]
    state = (x, p, x, p, 0.05)
    for c in (0.0, 0.7):
        w = _uniform_weights(prob, c)
        cn, cp = G.forward(prob, w, *state)
        nb = 2 * prob.dim
        diag = np.array([i * (i + 1) // 2 + i for i in range(nb)])
        cnr = cn.reshape(prob.n_nodes, -1)
        assert np.all(cnr[:, diag] == c) and np.all(np.delete(cnr, diag, axis=1) == 0) and np.all(cp == c)
        # C = e^c I, so T = e^{-2c} T0 and T^2 = e^{-4c} I: the best scale gamma = e^{4c} makes every
        # probe's residual vanish (without gamma the loss would be (e^{-4c} - 1)^2)
        T = G.symmetric_operator(prob, P, K, cn, cp)
        assert np.abs(T @ T - np.exp(-4 * c) * np.eye(K.shape[0])).max() <= 1e-8
        assert G.train_loss(prob, P, K, w, state, probes) <= 1e-14


def test_train_loss_is_invariant_to_scaling_the_matrix(ref_case):
    prob, x, p, K, P, x2, p2, K2 = ref_case
    rng = np.random.default_rng(4)
    probes = [rng.standard_normal(K.shape[0]) for _ in range(2)]
    w = 0.05 * rng.standard_normal(G.num_weights(prob))
    state = (x, p, x2, p2, 0.05)
    l1 = G.train_loss(prob, P, K2, w, state, probes)
    l2 = G.train_loss(prob, P, 3.0 * K2, w, state, probes)
    assert 0.0 < l1 < 1.0
    assert abs(l1 - l2) <= 1e-10 * l1
    # one probe by hand: gamma = u.b / b.b with b = T^2 u minimises |gamma b - u|^2
    u = probes[0]
    cn, cp = G.forward(prob, w, *state)
    T = G.symmetric_operator(prob, P, K2, cn, cp)
    b = T @ (T @ u)
    gam = (u @ b) / (b @ b)
    best = np.sum((gam * b - u) ** 2) / (u @ u)
    for g in (0.9 * gam, 1.1 * gam):
        assert np.sum((g * b - u) ** 2) / (u @ u) > best
    assert abs(G.train_loss(prob, P, K2, w, state, [u]) - best) <= 1e-12 * best


def test_train_loss_complex_step_matches_central_differences(ref_case):
    prob, x, p, K, P, x2, p2, K2 = ref_case
    rng = np.random.default_rng(6)
    probes = [rng.standard_normal(K.shape[0]) for _ in range(2)]
    w = 0.05 * rng.standard_normal(G.num_weights(prob))
    state = (x, p, x2, p2, 0.05)
    u = rng.standard_normal(w.size)
    h = 1e-30
    cs = G.train_loss(prob, P, K2, w.astype(np.complex128) + 1j * h * u, state, probes).imag / h
    hd = 1e-5
    fd = (G.train_loss(prob, P, K2, w + hd * u, state, probes)
          - G.train_loss(prob, P, K2, w - hd * u, state, probes)) / (2 * hd)
    assert abs(cs - fd) <= 1e-5 * max(abs(fd), 1e-8), (cs, fd)
    assert abs(fd) > 0
