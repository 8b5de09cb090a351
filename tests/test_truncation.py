"""Important-term truncation (Sec. 5 "distributions of terms", App. D).

The oracle builds its own list of block-form terms (one per canonical slot
assignment of the antisymmetrised source, merged by monomial) and its own
selection. Pins of those two pieces come first (sums against the other oracle
routes, counts, a worked example, brute force over subsets, invariances);
then the library's wick_plan_truncate is compared with them on the host.
"""
import ctypes
import itertools
import math

import numpy as np
import pytest

import oracle
import paper_2411_08962_amd as W
import wick_inputs as wi
from oracle import operators as ops
from tests.helpers import oracle_compact_blocks, plan_kind_order, row_index, table_entries, to_wick


def props(V, wid, t=(0,)):
    Su, Sd = wi.propagator_pair(wid, 0, (V, 1, 1, max(t) + 1), t_slices=list(t))
    return [(Su[i], Sd[i]) for i in range(len(t))]


def eq24_blocks(op, slices):
    return np.stack([np.stack([oracle.block_eq24(k, Su, Sd) for k in op.kinds]) for Su, Sd in slices])


# ----------------------------------------------------- oracle term list pins
@pytest.mark.parametrize("make", [lambda: ops.proton(1), ops.deuteron, ops.helium3, lambda: ops.triton(1)])
def test_oracle_term_list_sums_to_the_correlator(make):
    # summed on Eq. 2.4 blocks, the list equals the DP route on raw blocks
    op = make()
    (Su, Sd), = props(3, 911)
    ent, c = oracle.term_list(op)
    v = oracle.term_values(ent, c, eq24_blocks(op, [(Su, Sd)]))[0]
    ref = oracle.sum_dp(op, oracle.blocks_raw(op, Su, Sd))
    assert abs(v.sum() - ref) <= 1e-13 * np.abs(v).sum()
    keys, cm = oracle.merged_terms(op)
    vm = oracle.term_values(keys, cm, eq24_blocks(op, [(Su, Sd)]))[0]
    assert abs(vm.sum() - op.scale * ref) <= 1e-13 * np.abs(vm).sum()


def test_oracle_term_list_matches_full_route_on_sparse_helium4():
    op = ops.sparsify(ops.helium4(), 3, np.random.default_rng(5), keep_patterns=2)
    (Su, Sd), = props(2, 912)
    ent, c = oracle.term_list(op)
    v = oracle.term_values(ent, c, eq24_blocks(op, [(Su, Sd)]))[0]
    ref = oracle.sum_full(op, oracle.blocks_raw(op, Su, Sd))
    assert len(c) > 0
    assert abs(v.sum() - ref) <= 1e-12 * np.abs(v).sum()


@pytest.mark.parametrize("name", ["2H", "3He"])
def test_oracle_term_count_is_one_per_assignment_class(name):
    # n_u! n_d! assignments per (group, pattern), 2^A of them per class (Sec. 2.2 counting)
    op = ops.by_name(name)
    fl = ops.flavor_listing(op, op.snk[0][0])
    nu, nd = fl.count(0), fl.count(1)
    ent, _ = oracle.term_list(op)
    per = math.factorial(nu) * math.factorial(nd) // 2 ** op.A
    assert len(ent) == oracle.source_group_count(op) * len(op.snk) * per
    assert np.all(ent % 1728 // 144 < ent % 12)  # i1 < i3 in every block


# ------------------------------------------------------ selection: pins
def test_selection_worked_example():
    # four one-block terms on two slices, values written out by hand:
    # slice 0: 4, -1, 0.5, 2 (max 4); slice 1: 0.1, 3, 0.2, -0.3 (max 3)
    # scores: max(4/4, .1/3)=1, max(1/4, 3/3)=1, max(.5/4, .2/3)=.125, max(2/4, .3/3)=.5
    B = np.zeros((2, 1, 12, 12, 12), dtype=np.complex128)
    flat = B.reshape(2, -1)
    keys = np.array([[1], [2], [3], [4]], dtype=np.int32)
    flat[0, 1:5] = [4, -1, 0.5, 2]
    flat[1, 1:5] = [0.1, 3, 0.2, -0.3]
    coef = np.ones(4, dtype=np.complex128)
    kept, score, dropped = oracle.important_terms(keys, coef, B, 0.5)
    assert np.allclose(score, [1, 1, 0.125, 0.5])
    assert kept.tolist() == [True, True, False, False]
    assert np.allclose(dropped, [2.5, 0.5])
    kept, _, dropped = oracle.important_terms(keys, coef, B, 0.75)
    assert kept.tolist() == [True, True, False, True]
    assert np.allclose(dropped, [0.5, 0.2])
    kept, _, dropped = oracle.important_terms(keys, coef, B, 0.01)
    assert kept.sum() == 1 and kept[0]  # one term at least; equal scores: lower index first
    assert oracle.keep_count(1000, 0.05) == 50 and oracle.keep_count(7, 1.0) == 7


def test_selection_is_the_best_subset_by_brute_force():
    rng = np.random.default_rng(3)
    K, A, N, S = 1, 2, 9, 3
    B = (rng.standard_normal((S, K, 12, 12, 12)) + 1j * rng.standard_normal((S, K, 12, 12, 12)))
    keys = rng.integers(0, 1728, size=(N, A)).astype(np.int32)
    coef = rng.integers(-3, 4, size=N) + 0j
    coef[coef == 0] = 1
    mag = np.abs(oracle.term_values(keys, coef, B))
    norm = mag / mag.max(axis=1, keepdims=True)
    for keep in (0.2, 0.45, 0.7):
        kept, _, dropped = oracle.important_terms(keys, coef, B, keep)
        M = oracle.keep_count(N, keep)
        best = max(itertools.combinations(range(N), M), key=lambda sub: sum(norm[:, list(sub)].max(axis=0)))
        assert sorted(np.flatnonzero(kept).tolist()) == sorted(best)
        assert np.allclose(dropped, mag[:, ~kept].sum(axis=1))


def test_selection_invariances_and_error_bound():
    op = ops.deuteron()
    keys, coef = oracle.merged_terms(op)
    Beq = eq24_blocks(op, props(3, 913, t=(0, 1, 2)))
    kept, score, dropped = oracle.important_terms(keys, coef, Beq, 0.1)
    # per-slice normalisation: scaling one slice's blocks changes nothing
    B2 = Beq.copy()
    B2[1] *= 7.5
    k2, s2, _ = oracle.important_terms(keys, coef, B2, 0.1)
    assert np.array_equal(kept, k2) and np.allclose(score, s2, rtol=1e-13)
    # reordering the table reorders the selection
    perm = np.random.default_rng(1).permutation(len(coef))
    k3, _, _ = oracle.important_terms(keys[perm], coef[perm], Beq, 0.1)
    assert np.array_equal(kept[perm], k3)
    # nested fractions
    k4, _, _ = oracle.important_terms(keys, coef, Beq, 0.3)
    assert np.all(k4[kept])
    # |C_full - C_kept| <= sum of |dropped terms| on every slice
    v = oracle.term_values(keys, coef, Beq)
    assert np.all(np.abs(v.sum(axis=1) - v[:, kept].sum(axis=1)) <= dropped * (1 + 1e-12))
    # keeping everything
    kall, _, d0 = oracle.important_terms(keys, coef, Beq, 1.0)
    assert kall.all() and np.all(d0 == 0)


# ------------------------------------------------ the library vs the oracle
@pytest.mark.parametrize("name", ["2H", "3He"])
def test_plan_table_equals_oracle_merged_terms(name):
    # the planner's F_p merge and the oracle's exact monomial merge give the same table
    op = ops.by_name(name)
    pl = W.plan_std(name)
    ent, coef = table_entries(op, pl)
    keys, cm = oracle.merged_terms(op)
    assert len(coef) == len(cm)
    idx = row_index(keys)
    pos = np.array([idx[tuple(r)] for r in np.sort(ent, axis=1).tolist()])
    assert np.array_equal(np.sort(pos), np.arange(len(cm)))
    assert np.array_equal(coef, cm[pos])


def check_truncation(op, pl, slices, keep):
    order = plan_kind_order(op, pl)
    Bc = np.stack([oracle_compact_blocks(op, order, Su, Sd) for Su, Sd in slices])
    keys, cm = oracle.merged_terms(op)
    kept, score, dropped = oracle.important_terms(keys, cm, eq24_blocks(op, slices), keep)
    tp, dp = pl.truncate(Bc, keep)
    M = oracle.keep_count(len(cm), keep)
    assert tp.n_terms == M
    # a sub-table of the full one, in table order, coefficients unchanged
    fe, fc = table_entries(op, pl)
    te, tc = table_entries(op, tp)
    fidx = row_index(fe)
    fpos = np.array([fidx[tuple(r)] for r in np.sort(te, axis=1).tolist()])
    assert np.all(np.diff(fpos) > 0) and np.array_equal(tc, fc[fpos])
    # the same selection as the oracle's, up to (near-)equal scores at the edge
    idx = row_index(keys)
    opos = np.array([idx[tuple(r)] for r in np.sort(te, axis=1).tolist()])
    tau = np.sort(score)[::-1][M - 1]
    assert np.all(score[opos] >= tau * (1 - 1e-12))
    must = np.flatnonzero(score > tau * (1 + 1e-12))
    assert set(must.tolist()) <= set(opos.tolist())
    total = np.abs(oracle.term_values(keys, cm, eq24_blocks(op, slices))).sum(axis=1)
    assert np.all(np.abs(dp - dropped) <= 1e-12 * total)
    return tp, kept, keys, cm


@pytest.mark.parametrize("name,keep,nt", [("2H", 0.05, 1), ("2H", 0.3, 3), ("3He", 0.01, 2), ("3H", 0.2, 1)])
def test_truncate_matches_oracle_selection(name, keep, nt):
    op = ops.by_name(name)
    pl = W.plan_std(name)
    tp, kept, keys, cm = check_truncation(op, pl, props(2, 914, t=tuple(range(nt))), keep)
    assert tp.n_kinds == pl.n_kinds and tp.A == pl.A


def test_truncate_sparse_helium4_and_general_plan():
    op = ops.sparsify(ops.helium4(), 4, np.random.default_rng(8), keep_patterns=3)
    pl = W.plan(**to_wick(op))
    check_truncation(op, pl, props(2, 915, t=(0, 1)), 0.15)


def test_truncate_keep_all_is_the_identity_and_is_deterministic(tmp_path):
    op = ops.deuteron()
    pl = W.plan_std("2H")
    Bc = oracle_compact_blocks(op, plan_kind_order(op, pl), *props(2, 916)[0])
    full_k, full_c = pl.table()
    t1, d1 = pl.truncate(Bc, 1.0)
    k1, c1 = t1.table()
    assert np.array_equal(k1, full_k) and np.array_equal(c1, full_c) and np.all(d1 == 0)
    a, da = pl.truncate(Bc, 0.2)
    b, db = pl.truncate(Bc, 0.2)
    assert np.array_equal(a.table()[0], b.table()[0]) and np.array_equal(da, db)
    a.save(tmp_path / "t.plan")
    c = W.Plan.load(tmp_path / "t.plan")
    assert np.array_equal(c.table()[0], a.table()[0]) and np.array_equal(c.table()[1], a.table()[1])
    # zero calibration blocks: every score is 0, the first terms in table order are kept
    z, dz = pl.truncate(np.zeros_like(Bc), 0.1)
    assert np.array_equal(z.table()[0], full_k[:, :z.n_terms]) and np.all(dz == 0)


def test_truncate_rejects_bad_arguments():
    pl = W.plan_std("2H")
    B = np.zeros((1, pl.n_kinds, 792, 2))
    for keep in (0.0, -0.1, 1.5, float("nan")):
        with pytest.raises(W.WickError) as e:
            pl.truncate(B, keep)
        assert e.value.status == W.EINVAL
    bad = B.copy()
    bad[0, 0, 5, 1] = np.inf
    with pytest.raises(W.WickError):
        pl.truncate(bad, 0.5)
    with pytest.raises(ValueError):
        pl.truncate(np.zeros((1, pl.n_kinds + 1, 792, 2)), 0.5)
    L = W.lib()
    h = ctypes.c_void_p()
    assert L.wick_plan_truncate(pl.handle, B.ctypes.data_as(ctypes.c_void_p), 0, 0.5, ctypes.byref(h), None) == W.EINVAL
    assert L.wick_plan_truncate(pl.handle, None, 1, 0.5, ctypes.byref(h), None) == W.EINVAL
    assert L.wick_plan_truncate(None, B.ctypes.data_as(ctypes.c_void_p), 1, 0.5, ctypes.byref(h), None) == W.EINVAL
    assert L.wick_plan_truncate(pl.handle, B.ctypes.data_as(ctypes.c_void_p), 1, 0.5, None, None) == W.EINVAL


def test_truncate_complex_coefficient_plan():
    # complex couplings: the kept coefficients stay complex and the selection matches the oracle's
    op = ops.deuteron()
    snk = [(k, (c[0] - 2 * c[1], 2 * c[0] + c[1])) for k, c in op.snk]
    src = [(k, (2 * c[0] + c[1], -c[0] + 2 * c[1])) for k, c in op.src]
    opc = ops.Operator(op.A, op.kinds, snk, src, op.scale, "2H-complex")
    pl = W.plan(**to_wick(opc))
    tp, kept, keys, cm = check_truncation(opc, pl, props(2, 917, t=(0, 1)), 0.25)
    assert np.any(tp.table()[1].imag != 0)
