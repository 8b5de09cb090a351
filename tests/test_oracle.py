"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: they check it against values the
paper prints (term counts, permutation counts, the single-proton expression),
closed forms, algebraic invariances and independent formulations.
"""
import math
import os

import numpy as np
import pytest

import oracle
import wick_inputs as wi
from oracle import conventions as cv
from oracle import operators as ops

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_gold(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.split("#")[0].strip()
        if line:
            rows.append(line.split())
    return rows


def small(V=2, T=1, wid=900, cfg=0):
    return wi.propagator_pair(wid, cfg, (V, 1, 1, T))


def su3(rng):
    z = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    q, r = np.linalg.qr(z)
    q = q * (np.diag(r) / abs(np.diag(r)))
    return q / np.linalg.det(q) ** (1 / 3)


def close(a, b, scale, tol=1e-12):
    return abs(a - b) <= tol * max(scale, 1e-300)


# --------------------------------------------------------------------------
# Conventions
# --------------------------------------------------------------------------
def test_gamma_algebra():
    g = cv.gammas()
    for m in range(4):
        for n in range(4):
            ac = g[m] @ g[n] + g[n] @ g[m]
            assert np.allclose(ac, 2 * np.eye(4) * (m == n))
        assert np.allclose(g[m], g[m].conj().T)          # Euclidean: hermitian
        assert np.allclose(g[4] @ g[m] + g[m] @ g[4], 0)  # gamma_5 anticommutes
    C = cv.charge_conjugation()
    Ci = np.linalg.inv(C)
    for m in range(4):
        assert np.allclose(C @ g[m] @ Ci, -g[m].T)          # charge conjugation
    M = cv.cg5()
    assert np.array_equal(M, -M.T)                           # C g5 antisymmetric
    for s in (+1, -1):
        P = cv.proj(s)
        assert np.array_equal(P @ P, P)
    assert np.array_equal(cv.proj(1) + cv.proj(-1), np.eye(4, dtype=np.int64))
    e = cv.levi_civita()
    assert e[0, 1, 2] == 1 and e[1, 0, 2] == -1 and np.count_nonzero(e) == 6


def test_nucleon_weights_count():
    # 6 colour orderings times the nonzeros of the diquark matrix (Sec. 2: one
    # eps and one gamma matrix per nucleon: 6 and 4 entries).
    assert len(ops.nucleon_kind("p", 0, 0).w) == 24
    assert len(ops.nucleon_kind("n", +1, 1).w) == 12


# --------------------------------------------------------------------------
# Counts the paper prints
# --------------------------------------------------------------------------
def test_operator_term_counts_match_paper():
    for name, J, count in _read_gold("operator_term_counts.txt"):
        if name == "3He":
            op = ops.helium3(int(J))
        else:
            op = ops.by_name(name)
        assert oracle.source_group_count(op) == int(count), name


def test_nperm_table1():
    for name, nu, nd, nperm in _read_gold("table1_nperm.txt"):
        nu, nd = int(nu), int(nd)
        f = [0] * nu + [1] * nd
        g = list(f)
        np.random.default_rng(nu * 7 + nd).shuffle(g)
        assert oracle.count_bijections(f, g) == int(nperm) == math.factorial(nu) * math.factorial(nd)
    # and the listings of the built operators carry those flavor contents
    assert ops.deuteron().n_u == 3 and ops.helium3().n_u == 5 and ops.helium4().n_u == 6


# --------------------------------------------------------------------------
# Blocks
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [ops.nucleon_kind("p", 0, 1), ops.nucleon_kind("n", -1, 2)])
def test_block_identity_propagator_closed_form(kind):
    # S = 1 at every site: B[i1,i2,i3] = V w(i1,i2,i3).
    V = 5
    S = np.broadcast_to(np.eye(12, dtype=np.complex128), (V, 12, 12)).copy()
    B = oracle.block_raw(kind, S, S)
    W = np.zeros((12, 12, 12), dtype=np.complex128)
    for j1, j2, j3, a, b in kind.w:
        W[j1, j2, j3] = a + 1j * b
    assert np.array_equal(B, V * W)


def test_block_sink_colour_rotation_invariance():
    # S(x) -> (1 x Omega(x)) S(x) at the sink leaves every block unchanged
    # (each nucleon is an eps singlet at its sink site).
    rng = np.random.default_rng(3)
    Su, Sd = small(V=3)
    Su2, Sd2 = Su[0].reshape(-1, 12, 12).copy(), Sd[0].reshape(-1, 12, 12).copy()
    for x in range(3):
        R = np.kron(np.eye(4), su3(rng))
        Su2[x] = R @ Su2[x]
        Sd2[x] = R @ Sd2[x]
    for kind in (ops.nucleon_kind("p", 0, 0), ops.nucleon_kind("n", +1, 3)):
        B1 = oracle.block_raw(kind, Su[0], Sd[0])
        B2 = oracle.block_raw(kind, Su2, Sd2)
        assert np.max(abs(B1 - B2)) <= 1e-12 * np.max(abs(B1))


def test_block_eq24_is_antisymmetrised_raw_block():
    Su, Sd = small(V=3)
    kind = ops.nucleon_kind("p", -1, 1)
    R = oracle.block_raw(kind, Su[0], Sd[0])
    E = oracle.block_eq24(kind, Su[0], Sd[0])
    ref = R - R.transpose(2, 1, 0)
    assert np.max(abs(E - ref)) <= 1e-13 * np.max(abs(R))
    assert np.max(abs(E + E.transpose(2, 1, 0))) <= 1e-13 * np.max(abs(R))


# --------------------------------------------------------------------------
# The single-proton expression printed in App. B
# --------------------------------------------------------------------------
@pytest.mark.parametrize("a_snk,a_src", [(0, 0), (1, 1), (2, 3), (3, 1)])
def test_single_proton_matches_printed_two_term_expression(a_snk, a_src):
    Su, Sd = small(V=3)
    su = Su[0].reshape(-1, 4, 3, 4, 3)  # [x, spin, colour, spin', colour']
    sd = Sd[0].reshape(-1, 4, 3, 4, 3)
    eps = cv.levi_civita().astype(float)
    C = cv.cg5().astype(float)
    qf = [su, su, sd]  # sink quarks 0 = (i, alpha) u, 1 = (j, beta) u, 2 = (k, gamma) d
    total = 0.0
    for sign, *pairs in _read_gold("single_proton_two_terms.txt"):
        p = [int(v) for v in pairs]
        # source quark labels: 0 -> (I, A'), 1 -> (J, B'), 2 -> (K, G')
        src = {0: "IA", 1: "JB", 2: "KG"}
        subs = []
        for q, (lab_c, lab_s) in enumerate([("i", "a"), ("j", "b"), ("k", "g")]):
            sc, ss = src[p[q]]
            subs.append(f"x{lab_s}{lab_c}{ss}{sc}")
        expr = "ijk,bg,IJK,BG," + ",".join(subs) + "->xaA"
        val = np.einsum(expr, eps, C, eps, C, *qf, optimize=True).sum(axis=0)
        total = total + (1 if sign == "+" else -1) * val
    ref = total[a_snk, a_src]
    op = ops.proton_pair(a_snk, a_src)
    for route in ("bruteforce", "full", "dp"):
        got = oracle.correlator(op, Su, Sd, route=route)[0]
        assert close(got, ref, abs(ref) + 1.0, 1e-12), (route, got, ref)


# --------------------------------------------------------------------------
# Independent routes agree
# --------------------------------------------------------------------------
def _routes(op, Su, Sd, by_flavor_only=False):
    B = oracle.blocks_raw(op, Su, Sd)
    bf, mag = oracle.bruteforce(op, Su, Sd, by_flavor=True, with_magnitude=True)
    out = {"dp": oracle.sum_dp(op, B), "bf_flavor": bf}
    if not by_flavor_only:
        out["bf"] = oracle.bruteforce(op, Su, Sd)
        out["full"] = oracle.sum_full(op, B)
    return out, mag


@pytest.mark.parametrize("name", ["p", "2H"])
def test_routes_agree_full_operators(name):
    op = ops.proton() if name == "p" else ops.deuteron()
    Su, Sd = small(V=2)
    r, mag = _routes(op, Su[0], Sd[0])
    ref = r["bf"]
    assert abs(ref) > 1e-6 * mag
    for k, v in r.items():
        assert close(v, ref, mag, 1e-13), (k, v, ref)


@pytest.mark.parametrize("name,keep,pats", [("3He", 4, 2), ("3H", 4, 2), ("4He", 2, 5)])
def test_routes_agree_sparsified(name, keep, pats):
    # first seed whose sparsified operator is not a pure Pauli zero
    for seed in range(200):
        op = ops.sparsify(ops.by_name(name), keep, np.random.default_rng(seed), keep_patterns=pats)
        if oracle.source_group_count(op) > 0:
            break
    Su, Sd = small(V=2)
    r, mag = _routes(op, Su[0], Sd[0], by_flavor_only=(name == "4He"))
    ref = r["bf_flavor"]
    assert abs(ref) > 1e-6 * mag
    for k, v in r.items():
        assert close(v, ref, mag, 1e-13), (k, v, ref)


def test_full_equals_dp_3He_full_operator():
    Su, Sd = small(V=2)
    op = ops.helium3()
    B = oracle.blocks_raw(op, Su[0], Sd[0])
    a, b = oracle.sum_full(op, B), oracle.sum_dp(op, B)
    assert close(a, b, abs(a), 1e-12)


# --------------------------------------------------------------------------
# Pauli zeros
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["2H", "3He", "4He"])
def test_rank_one_u_propagator_gives_zero(name):
    # S_u(x) = a(x) b^T with b fixed: every u determinant vanishes (>= 2 u quarks).
    rng = np.random.default_rng(5)
    Su, Sd = small(V=2)
    b = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    a = rng.standard_normal((2, 12)) + 1j * rng.standard_normal((2, 12))
    Su1 = np.einsum("xj,i->xji", a, b)
    op = ops.by_name(name)
    # entries of Su1 have the same magnitude as those of the generic Su
    c0 = oracle.sum_dp(op, oracle.blocks_raw(op, Su1, Sd[0]))
    cg = oracle.sum_dp(op, oracle.blocks_raw(op, Su[0], Sd[0]))
    assert abs(cg) > 0
    assert abs(c0) <= 1e-10 * abs(cg)


def test_repeated_source_index_gives_exact_zero():
    # a source in which the two u quarks of every nucleon carry the same index
    op = ops.deuteron()
    kinds = []
    for k in op.kinds:
        w = [(j1, j2, j1, a, b) for (j1, j2, j3, a, b) in k.w]
        kinds.append(ops.Kind(k.flavors, w, k.label))
    src_kinds = [ops.Kind(k.flavors, k.w, k.label) for k in kinds]
    op2 = ops.Operator(2, op.kinds + src_kinds, op.snk,
                       [(tuple(i + len(op.kinds) for i in p), c) for p, c in op.src])
    assert oracle.source_group_count(op2) == 0
    Su, Sd = small(V=2)
    c, mag = oracle.bruteforce(op2, Su[0], Sd[0], with_magnitude=True)
    assert mag > 0 and abs(c) <= 1e-14 * mag      # pairs cancel up to rounding
    assert oracle.sum_dp(op2, oracle.blocks_raw(op2, Su[0], Sd[0])) == 0


# --------------------------------------------------------------------------
# Grassmann signs
# --------------------------------------------------------------------------
def _swap13(k):
    return ops.Kind(k.flavors, [(j3, j2, j1, a, b) for (j1, j2, j3, a, b) in k.w], k.label)


def test_swapping_two_source_quarks_flips_sign():
    op = ops.deuteron()
    Su, Sd = small(V=2)
    c1 = oracle.bruteforce(op, Su[0], Sd[0])
    K = len(op.kinds)
    src_kinds = [_swap13(k) for k in op.kinds]
    # swap the two same-flavor quarks of the first source nucleon only
    src = [((p[0] + K, p[1]), c) for p, c in op.src]
    op2 = ops.Operator(2, op.kinds + src_kinds, op.snk, src)
    c2 = oracle.bruteforce(op2, Su[0], Sd[0])
    assert close(c2, -c1, abs(c1), 1e-12)
    B = oracle.blocks_raw(op2, Su[0], Sd[0])
    assert close(oracle.sum_dp(op2, B), -c1, abs(c1), 1e-12)


@pytest.mark.parametrize("name", ["2H", "3He"])
def test_swapping_two_sink_nucleons_flips_sign(name):
    op = ops.by_name(name)
    Su, Sd = small(V=2)
    B = oracle.blocks_raw(op, Su[0], Sd[0])
    c1 = oracle.sum_dp(op, B)
    swap = lambda p: (p[1], p[0]) + tuple(p[2:])
    op2 = ops.Operator(op.A, op.kinds, [(swap(p), c) for p, c in op.snk], op.src)
    op3 = ops.Operator(op.A, op.kinds, [(swap(p), c) for p, c in op.snk],
                       [(swap(p), c) for p, c in op.src])
    assert close(oracle.sum_dp(op2, B), -c1, abs(c1), 1e-12)
    assert close(oracle.sum_dp(op3, B), c1, abs(c1), 1e-12)
    if name == "2H":
        assert close(oracle.bruteforce(op2, Su[0], Sd[0]), -c1, abs(c1), 1e-12)


# --------------------------------------------------------------------------
# Colour invariance at the source
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["2H", "3He", "4He"])
def test_source_colour_rotation_invariance(name):
    rng = np.random.default_rng(8)
    Su, Sd = small(V=2)
    R = np.kron(np.eye(4), su3(rng).conj().T)
    op = ops.by_name(name)
    B1 = oracle.blocks_raw(op, Su[0], Sd[0])
    B2 = oracle.blocks_raw(op, Su[0] @ R, Sd[0] @ R)
    c1, c2 = oracle.sum_dp(op, B1), oracle.sum_dp(op, B2)
    assert abs(c1) > 0
    assert close(c1, c2, abs(c1), 1e-11)
