"""Pins of the oracle's preconditioner network (CPU only).

Zero decoders give zero corrections; a rigid translation of mesh and states
leaves the outputs unchanged; relabelling the nodes permutes the outputs the same
way; complex-step weight gradients agree with central differences; the weight
count follows the layer list.
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
