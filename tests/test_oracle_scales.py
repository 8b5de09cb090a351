"""Pins of the oracle's error scales and of its flat-table evaluator.

``oracle.point_det_magnitude`` is the absolute-term scale of the determinant
form of a point-sink correlator (Eq. 2.9, the weighted double sum of App. A,
Eq. A1); ``oracle.table_sum`` evaluates a flat list of block-entry products
(Eq. 2.6 written term by term). Each is checked against something other than
itself: a closed form, the block-form DP route of the oracle, a triangle
inequality, and the single-nucleon expression written out quark by quark.
"""
import itertools

import numpy as np
import pytest

import oracle
import wick_inputs as wi
from oracle import operators as ops


# ------------------------------------------------------------ table_sum
def _merged(op):
    keys, coef = oracle.merged_terms(op)
    return keys.T.astype(np.uint16), coef


@pytest.mark.parametrize("make", [lambda: ops.proton(1), ops.deuteron, ops.helium3])
def test_table_sum_of_the_merged_terms_equals_the_dp_route(make):
    # the oracle's own merged term list, evaluated as a flat table, against the
    # subset DP over antisymmetrised source groups (a different algorithm)
    op = make()
    kidx, coef = _merged(op)
    Su, Sd = wi.propagator_pair(961, 0, (2, 1, 1, 2))
    sets, refs = [], []
    for t in range(2):
        Be = np.stack([oracle.block_eq24(k, Su[t], Sd[t]) for k in op.kinds])
        sets.append(Be.reshape(-1))
        refs.append(op.scale * oracle.sum_dp(op, oracle.blocks_raw(op, Su[t], Sd[t])))
    got = oracle.table_sum(kidx, coef, np.stack(sets))
    mag = oracle.table_sum(kidx, np.abs(coef), np.abs(np.stack(sets))).real
    for t in range(2):
        assert abs(got[t] - refs[t]) <= 1e-12 * mag[t], (t, got[t], refs[t])
        assert abs(got[t]) <= mag[t] * (1 + 1e-12)


def test_table_sum_homogeneity_and_empty_table():
    op = ops.deuteron()
    kidx, coef = _merged(op)
    rng = np.random.default_rng(5)
    B = rng.standard_normal(len(op.kinds) * 1728) + 1j * rng.standard_normal(len(op.kinds) * 1728)
    a = oracle.table_sum(kidx, coef, B[None])[0]
    b = oracle.table_sum(kidx, coef, 2 * B[None])[0]
    # A = 2: scaling every entry by 2 scales each term by 4 exactly (the
    # threads' partial sums may combine in another order, hence the tolerance)
    assert abs(b - 4 * a) <= 1e-13 * abs(b)
    # a coefficient vector with one nonzero entry selects that term alone
    n = len(coef) // 2
    one = np.zeros_like(coef)
    one[n] = 1.0
    v = oracle.table_sum(kidx, one, B[None])[0]
    assert abs(v - B[kidx[0, n]] * B[kidx[1, n]]) <= 1e-15 * abs(v)
    empty = oracle.table_sum(np.zeros((2, 0), np.uint16), np.zeros(0, np.complex128), B[None])
    assert empty[0] == 0


# --------------------------------------------------- point_det_magnitude
def _diag_props(rng, V, T, positive):
    S = np.zeros((T, 1, 1, V, 12, 12), dtype=np.complex128)
    for t in range(T):
        for x in range(V):
            d = rng.uniform(0.5, 2.0, 12) if positive else np.ones(12)
            S[t, 0, 0, x] = np.diag(d)
    return S


@pytest.mark.parametrize("make", [ops.deuteron, ops.helium3])
def test_point_det_magnitude_identity_closed_form(make):
    # S = 1: det S[R; K] = [R == K], so every surviving term is W_g^2 >= 0 and
    # the scale equals |C| = |scale| V sum_g W_g^2, here from the DP route
    op = make()
    V = 3
    S = _diag_props(None, V, 1, positive=False)
    mag = oracle.point_det_magnitude(op, S, S)[0]
    c = oracle.point_correlator(op, S, S)[0]
    assert abs(mag - abs(c)) <= 1e-12 * mag
    _, w = oracle.source_groups(op)
    assert abs(mag - abs(op.scale) * V * np.sum(np.abs(w) ** 2)) <= 1e-12 * mag


@pytest.mark.parametrize("make", [ops.deuteron, ops.helium3])
def test_point_det_magnitude_positive_diagonal(make):
    # S(x) diagonal with positive entries: det S[R; K] = prod_R d if R == K else 0,
    # so again no term can cancel and the scale equals |C| of the DP route
    op = make()
    rng = np.random.default_rng(11)
    Su = _diag_props(rng, 2, 2, positive=True)
    Sd = _diag_props(rng, 2, 2, positive=True)
    mag = oracle.point_det_magnitude(op, Su, Sd)
    c = oracle.point_correlator(op, Su, Sd)
    for t in range(2):
        assert abs(mag[t] - abs(c[t])) <= 1e-12 * mag[t], t


@pytest.mark.parametrize("make", [ops.deuteron, ops.helium3])
def test_point_det_magnitude_bounds_the_correlator(make):
    op = make()
    Su, Sd = wi.propagator_pair(962, 0, (2, 1, 1, 2))
    mag = oracle.point_det_magnitude(op, Su, Sd)
    c = oracle.point_correlator(op, Su, Sd)
    assert np.all(np.abs(c) <= mag * (1 + 1e-12))
    assert np.all(mag > 0)


def test_point_det_magnitude_single_proton_by_hand():
    # A = 1: the two-term expression of the single proton (App. B), summed with
    # absolute values over antisymmetrised sink and source index sets
    op = ops.proton(0)
    w = np.zeros((12, 12, 12))
    for j1, j2, j3, re, im in op.kinds[0].w:
        w[j1, j2, j3] = re
    Su, Sd = wi.propagator_pair(963, 0, (2, 1, 1, 1))
    su, sd = Su[0].reshape(-1, 12, 12), Sd[0].reshape(-1, 12, 12)
    ref = 0.0
    sets = [(a, c, b) for a, b in itertools.combinations(range(12), 2) for c in range(12)]
    W = {(a, c, b): w[a, c, b] - w[b, c, a] for a, c, b in sets}
    nz = [s for s in sets if W[s] != 0]
    for x in range(su.shape[0]):
        for (a, c, b) in nz:
            for (i, k, j) in nz:
                det = su[x, a, i] * su[x, b, j] - su[x, a, j] * su[x, b, i]
                ref += abs(W[(a, c, b)]) * abs(W[(i, k, j)]) * abs(det) * abs(sd[x, c, k])
    mag = oracle.point_det_magnitude(op, Su, Sd)[0]
    assert abs(mag - ref) <= 1e-12 * ref
