"""Pins of the oracle's symbolic analysis (CPU only)."""
import os

import numpy as np
import pytest

import sgn_inputs as si
from oracle import dense as D
from oracle import symbolic as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    rows = [l for l in open(os.path.join(GOLD, name)) if not l.startswith("#")]
    return np.array(" ".join(rows).split(), dtype=np.int64)


def test_nd_order_matches_hand_derivation():
    assert np.array_equal(S.nd_node_order(si.config_tiny()), _load("nd_order_grid2d_4x4.txt"))


@pytest.mark.parametrize("mk", [si.config_tiny,
                                lambda: si.problem_3d(4, 2, 2, 0.25, seed=1),
                                lambda: si.problem_3d(2, 2, 1, 0.5, seed=1, param_kind=si.P_REST_POS)])
def test_three_etree_algorithms_agree(mk):
    prob = mk()
    rp, ci = S.permuted_lower_csr(prob)
    e1 = S.etree_liu(rp, ci)
    assert np.array_equal(e1, S.etree_by_columns(rp, ci))
    if rp.size < 800:
        assert np.array_equal(e1, S.etree_dense(rp, ci))


def test_etree_definition_on_2d_config():
    prob = si.config_2d()
    rp, ci = S.permuted_lower_csr(prob)
    assert np.array_equal(S.etree_liu(rp, ci), S.etree_by_columns(rp, ci))


@pytest.mark.parametrize("mk", [si.config_tiny, lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=4),
                                lambda: si.problem_3d(2, 2, 2, 0.5, seed=1, param_kind=si.P_REST_POS),
                                lambda: si.problem_2d(4, seed=1, param_kind=si.P_NODAL_FORCE)])
def test_pattern_is_support_of_numeric_matrix(mk):
    # structural pattern = nonzeros of the numeric K_SGN at a generic state, plus every diagonal
    prob = mk()
    prob.length_scale = 1.0
    prob.target_val = np.zeros(prob.target_dof.size)
    rng = np.random.default_rng(0)
    x = prob.x_rest() + 1e-3 * rng.standard_normal(prob.n_x)
    p = prob.p_init() + (1e-3 if prob.param_kind == si.P_REST_POS else 0.2) * rng.standard_normal(prob.n_p)
    K = D.sgn_matrix_dense(prob, x, p)
    r, c = S.pattern_pairs(prob)
    M = np.zeros_like(K, dtype=bool)
    M[r, c] = True
    M[c, r] = True
    nz = K != 0
    nz[np.arange(K.shape[0]), np.arange(K.shape[0])] = True
    assert np.array_equal(M, nz)


@pytest.mark.parametrize("mk", [si.config_2d, lambda: si.problem_3d(6, 3, 3, 1 / 3, seed=4)])
def test_variable_order_is_permutation_with_contiguous_node_groups(mk):
    prob = mk()
    perm = S.variable_order(prob)
    N = 2 * prob.n_x + prob.n_p
    assert np.array_equal(np.sort(perm), np.arange(N))
    d, nx, npar = prob.dim, prob.n_x, prob.n_p
    pos = np.empty(N, dtype=np.int64)
    pos[perm] = np.arange(N)
    for k in range(0, nx, d):
        xs = pos[k:k + d]
        ls = pos[nx + npar + k:nx + npar + k + d]
        assert np.array_equal(xs, xs[0] + np.arange(d))
        assert np.array_equal(ls, xs[-1] + 1 + np.arange(d))


def test_csr_is_lower_sorted_and_complete():
    prob = si.config_2d()
    rp, ci = S.permuted_lower_csr(prob)
    N = rp.size - 1
    for i in range(N):
        row = ci[rp[i]:rp[i + 1]]
        assert row[-1] == i and np.all(np.diff(row) > 0)
    # Closed-form count for the 21 x 21 grid (rows 1..20 free, 420 nodes):
    # free-free edges 20*20 (horizontal) + 19*21 (vertical) + 19*20 (diagonal) = 1179;
    # Kx: d^2 (1 + deg) per free node = 4 * (420 + 2 * 1179); Kp: d per free incidence,
    # 800 * 3 - 60 fixed incidences; plus all N = 2480 diagonals.
    assert rp[-1] == 4 * (420 + 2 * 1179) + 2 * (800 * 3 - 60) + 2480
