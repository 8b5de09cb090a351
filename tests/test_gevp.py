"""Correlation matrices for the GEVP (Eqs. E1-E3): host side. The union table
must hold exactly every element's own table, and evaluated on the oracle's
blocks it must give the oracle's C_ij for every element."""
import numpy as np
import pytest

import oracle
import paper_2411_08962_amd as W
import wick_inputs as wi
from oracle import operators as ops
from tests.helpers import (eval_table, gevp_element, oracle_compact_blocks, plan_kind_order, sorted_entries,
                           table_entries, to_wick)


def deuteron_basis():
    return [ops.deuteron(+1), ops.deuteron(-1), ops.deuteron(0)]


def union_entries(op_elem, g):
    """The union table with indices in the oracle's encoding of op_elem's kinds."""
    bp = g.blocks_plan()
    kidx, coef = g.table()
    order = np.array(plan_kind_order(op_elem, bp), dtype=np.int64)
    from tests.helpers import pair_index
    dec = np.zeros(792, dtype=np.int64)
    for i3 in range(12):
        for i1 in range(i3):
            for i2 in range(12):
                dec[pair_index(i1, i3) * 12 + i2] = i1 * 144 + i2 * 12 + i3
    k = kidx.astype(np.int64)
    return (order[k // 792] * 1728 + dec[k % 792]).T, coef


@pytest.mark.parametrize("basis", ["2H3", "3He-J"])
def test_union_table_holds_every_element_table(basis):
    op_list = deuteron_basis() if basis == "2H3" else [ops.helium3(0), ops.helium3(1)]
    g = W.gevp_plan([to_wick(o) for o in op_list])
    info = g.info()
    n = len(op_list)
    total = 0
    # every element of the deuteron basis; one off-diagonal element of the 3He pair
    compare = {(i, j) for i in range(n) for j in range(n)} if basis == "2H3" else {(0, 1)}
    for i in range(n):
        for j in range(n):
            el = gevp_element(op_list, i, j)
            pe = W.plan(**to_wick(el))
            total += pe.n_terms
            if (i, j) not in compare:
                continue
            ent, coef = table_entries(el, pe)
            uent, ucoef = union_entries(el, g)
            pos = {t: m for m, t in enumerate(sorted_entries(uent))}
            idx = np.array([pos[t] for t in sorted_entries(ent)])
            assert np.array_equal(ucoef[idx, i, j], coef)
            others = np.ones(len(ucoef), dtype=bool)
            others[idx] = False
            assert np.all(ucoef[others, i, j] == 0)
    assert info["n_element_terms"] == total
    assert info["n_terms"] <= total
    if basis == "2H3":
        assert info["n_terms"] < total / 4  # the elements share most monomials


def test_union_table_gives_every_element_correlator():
    op_list = deuteron_basis()
    g = W.gevp_plan([to_wick(o) for o in op_list])
    Su, Sd = wi.propagator_pair(981, 0, (3, 2, 1, 1))
    kidx, coef = g.table()
    for i in range(3):
        for j in range(3):
            el = gevp_element(op_list, i, j)
            Bc = oracle_compact_blocks(el, plan_kind_order(el, g.blocks_plan()), Su[0], Sd[0])
            got, mag = eval_table(kidx, coef[:, i, j], Bc)
            ref = el.scale * oracle.sum_dp(el, oracle.blocks_raw(el, Su[0], Sd[0]))
            assert abs(got - ref) <= 1e-12 * mag


def test_single_operator_matrix_is_the_plain_plan():
    op = ops.deuteron()
    g = W.gevp_plan([to_wick(op)])
    pl = W.plan_std("2H")
    e1, c1 = table_entries(op, pl)
    e2, c2 = union_entries(op, g)
    m1 = dict(zip(sorted_entries(e1), c1))
    m2 = dict(zip(sorted_entries(e2), c2[:, 0, 0]))
    assert m1 == m2


def test_gevp_rejects_bad_bases():
    d = to_wick(ops.deuteron())
    with pytest.raises(W.WickError):
        W.gevp_plan([d, to_wick(ops.helium3())])          # different A
    with pytest.raises(W.WickError):
        W.gevp_plan([dict(d, scale=-1.0)])                # negative scale
    with pytest.raises(W.WickError):
        W.gevp_plan([d] * 5)                               # more than four operators
    with pytest.raises(W.WickError):
        W.gevp_plan([])


def test_builtin_basis_and_pair_plans_match_general_operators():
    bas = deuteron_basis()
    names = ["2H", "2H-", "2H0"]
    g1 = W.gevp_plan_std(names)
    g2 = W.gevp_plan([to_wick(o) for o in bas])
    assert g1.info() == g2.info()
    for a, b in zip(g1.table(), g2.table()):
        assert np.array_equal(a, b)
    for i in range(3):
        for j in range(3):
            el = gevp_element(bas, i, j)
            e1, c1 = table_entries(el, W.plan_std_pair(names[i], names[j]))
            e2, c2 = table_entries(el, W.plan(**to_wick(el)))
            assert dict(zip(sorted_entries(e1), c1)) == dict(zip(sorted_entries(e2), c2))
    with pytest.raises(W.WickError):
        W.plan_std_pair("2H", "3He")
