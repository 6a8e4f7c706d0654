"""Host-side checks of libsgn through its C ABI (no GPU needed): exported symbols,
argument validation, and bit-exact symbolic parity with the oracle."""
import os
import re

import numpy as np
import pytest

import sgn_inputs as si
from oracle import symbolic as S

sgn = pytest.importorskip("paper_2107_03285_amd.sgn")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        return sgn.load_library()
    except RuntimeError as e:  # not built in this checkout
        pytest.skip(str(e))


def test_library_exports_every_declared_symbol():
    lib = _lib()
    header = open(os.path.join(ROOT, "include", "sgn.h")).read()
    names = set(re.findall(r"\b(sgn_[a-z_0-9]+)\s*\(", header))
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names <= set(sgn.EXPORTS) | {"sgn_default_options"}


def test_create_rejects_invalid_problems():
    _lib()
    prob = si.config_tiny()
    bad = prob.copy()
    bad.elems = prob.elems.copy()
    bad.elems[0, 0] = prob.n_nodes + 5
    with pytest.raises(sgn.SgnError) as e:
        sgn.Context(bad)
    assert e.value.status == sgn.SGN_E_ARG
    bad = prob.copy()
    bad.nu = 0.5
    with pytest.raises(sgn.SgnError):
        sgn.Context(bad)
    bad = prob.copy()
    bad.target_dof = np.array([prob.n_x + 3], dtype=np.int32)
    with pytest.raises(sgn.SgnError):
        sgn.Context(bad)


def test_create_rejects_invalid_schedule_blocking():
    _lib()
    prob = si.config_tiny()
    for kw in ({"outer_panels": (17, 0, 0)}, {"outer_panels": (0, -1, 0)}, {"seq_panels": 9},
               {"seq_panels": -2}):
        o = sgn.default_options()
        if "outer_panels" in kw:
            for b, v in enumerate(kw["outer_panels"]):
                o.outer_panels[b] = v
        else:
            o.seq_panels = kw["seq_panels"]
        with pytest.raises(sgn.SgnError) as e:
            sgn.Context(prob, o)
        assert e.value.status == sgn.SGN_E_ARG


def test_schedule_blocking_leaves_the_symbolic_structure_unchanged():
    """The tuned blocking only regroups launches: ordering, pattern and elimination tree are those of
    the default schedule (and the oracle's)."""
    _lib()
    prob = si.config_cantilever_small()
    ref = sgn.Context(prob).symbolic(sgn.SGN_SYS_SGN)
    for tun in ({"outer_panels": [1, 2, 8], "seq_panels": -1, "panel_waves": 0},
                {"outer_panels": [8, 1, 2], "seq_panels": 2, "panel_waves": 4}):
        ctx = sgn.Context(prob, sgn.apply_tuning(sgn.default_options(), tun))
        for a, b in zip(ctx.symbolic(sgn.SGN_SYS_SGN), ref):
            assert np.array_equal(a, b)
        assert sgn.tuning_of(ctx.options) == tun


def test_device_calls_before_workspace_are_state_errors():
    _lib()
    ctx = sgn.Context(si.config_tiny())
    st, _ = ctx.factor_status()
    assert st == sgn.SGN_E_STATE


CASES = {
    "tiny": si.config_tiny,
    "grid21": si.config_2d,
    "cant4x2x2": lambda: si.problem_3d(4, 2, 2, 0.25, seed=1),
    "rest3x2x2": lambda: si.problem_3d(3, 2, 2, 1 / 3, seed=1, param_kind=si.P_REST_POS),
    "force5": lambda: si.problem_2d(5, seed=1, param_kind=si.P_NODAL_FORCE),
    "cant40x10x10": si.config_cantilever_small,
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_symbolic_structure_is_bit_exact(name):
    _lib()
    prob = CASES[name]()
    ctx = sgn.Context(prob)
    perm, etree, rowptr, colind = ctx.symbolic(sgn.SGN_SYS_SGN)
    operm = S.variable_order(prob)
    orp, oci = S.permuted_lower_csr(prob, operm)
    assert np.array_equal(perm, operm)
    assert np.array_equal(rowptr, orp)
    assert np.array_equal(colind, oci)
    assert np.array_equal(etree, S.etree_liu(orp, oci))
    sz = ctx.sizes()
    assert sz["n"] == 2 * prob.n_x + prob.n_p and sz["nnz"] == orp[-1]


@pytest.mark.parametrize("name", ["grid21", "cant4x2x2"])
def test_newton_form_structure_is_bit_exact(name):
    """The Newton form (hessian = SGN_HESSIAN_NEWTON) adds the x-x and x-p couplings of every element
    to the pattern without changing the variable order; its supernodal structure still holds it
    (sgn_create would fail on a missing slot)."""
    _lib()
    prob = CASES[name]()
    ctx = sgn.Context(prob, sgn.default_options(hessian=sgn.SGN_HESSIAN_NEWTON))
    perm, etree, rowptr, colind = ctx.symbolic(sgn.SGN_SYS_SGN)
    operm = S.variable_order(prob)
    orp, oci = S.permuted_lower_csr(prob, operm, newton=True)
    assert np.array_equal(perm, operm)
    assert np.array_equal(rowptr, orp) and np.array_equal(colind, oci)
    assert np.array_equal(etree, S.etree_liu(orp, oci))
    grp, _ = S.permuted_lower_csr(prob, operm)
    assert orp[-1] > grp[-1]
    # the Kx system is the same as in the Gauss-Newton form
    gn = sgn.Context(prob)
    for a, b in zip(ctx.symbolic(sgn.SGN_SYS_KX), gn.symbolic(sgn.SGN_SYS_KX)):
        assert np.array_equal(a, b)


@pytest.mark.slow
def test_symbolic_structure_is_bit_exact_at_200k_dof():
    _lib()
    prob = si.config_cantilever_200k()
    ctx = sgn.Context(prob)
    perm, etree, rowptr, colind = ctx.symbolic(sgn.SGN_SYS_SGN)
    operm = S.variable_order(prob)
    orp, oci = S.permuted_lower_csr(prob, operm)
    assert np.array_equal(perm, operm) and np.array_equal(rowptr, orp) and np.array_equal(colind, oci)
    assert np.array_equal(etree, S.etree_liu(orp, oci))
    assert rowptr[-1] == 12_043_982


def test_union_orders_each_problem_on_its_own():
    """A batch (disjoint union) is ordered problem by problem: the union's perm restricted to each
    problem is that problem's own perm shifted into the union's numbering (block order
    [x; p; lambda] of the union), and the elimination tree is a forest with one root per problem."""
    _lib()
    probs = si.batch_problems(5, base_seed=10000, lo=4, hi=9)
    u = si.union_problem(probs)
    cu = sgn.Context(u)
    pu, eu, _, _ = cu.symbolic()
    nxu, npu = u.n_x, u.n_p
    xo = np.concatenate([[0], np.cumsum([q.n_x for q in probs])])
    po = np.concatenate([[0], np.cumsum([q.n_p for q in probs])])
    pos = 0
    for i, q in enumerate(probs):
        pq, eq, _, _ = sgn.Context(q).symbolic()
        nx, npar = q.n_x, q.n_p
        # map the problem's old index (block order) into the union's old index
        mapped = np.where(pq < nx, pq + xo[i],
                          np.where(pq < nx + npar, nxu + po[i] + (pq - nx), nxu + npu + xo[i] + (pq - nx - npar)))
        n = pq.size
        assert np.array_equal(pu[pos:pos + n], mapped)
        e_local = np.where(eq >= 0, eq + pos, -1)
        assert np.array_equal(eu[pos:pos + n], e_local)
        pos += n
    assert pos == pu.size
    assert int(np.sum(eu < 0)) == len(probs)


def test_single_component_is_the_plain_problem():
    _lib()
    q = si.config_2d()
    a = sgn.Context(q).symbolic()
    q1 = q.copy()
    q1.components = np.array([0, q.n_nodes], dtype=np.int32)
    b = sgn.Context(q1).symbolic()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
