"""Host-side tests of the planner and the C ABI (no GPU needed).

The table is evaluated here with the oracle's blocks and compared with the
oracle's correlator, so the planner is checked against an independent
computation of the same C(t).
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import paper_2411_08962_amd as W
import wick_inputs as wi
from oracle import operators as ops
from tests.helpers import (eval_table, header_symbols, oracle_compact_blocks, plan_kind_order, sink_kind_order,
                           to_wick)


def small(V=3, wid=901):
    Su, Sd = wi.propagator_pair(wid, 0, (V, 1, 1, 1))
    return Su[0], Sd[0]


def check_plan(op, pl, Su, Sd, tol=1e-12):
    kidx, coef = pl.table()
    Bc = oracle_compact_blocks(op, plan_kind_order(op, pl), Su, Sd)
    got, mag = eval_table(kidx, coef, Bc)
    ref = op.scale * oracle.sum_dp(op, oracle.blocks_raw(op, Su, Sd))
    assert mag > 0
    assert abs(got - ref) <= tol * mag, (got, ref, mag)
    return got, mag


# ------------------------------------------------------------------ exports
def test_library_exports_every_header_symbol():
    L = W.lib()
    syms = header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(W.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", W.wick.LIB_PATH], capture_output=True, text=True).stdout
    for s in syms:
        assert f" T {s}\n" in out or f" T {s}" in out, s


def test_version_and_no_error():
    assert "gfx950" in W.version()


# ------------------------------------------------------------ vs the oracle
@pytest.mark.parametrize("name,J", [("2H", 0), ("3He", 0), ("3He", 1), ("3H", 0)])
def test_std_plan_matches_oracle(name, J):
    op = ops.helium3(J) if name == "3He" else ops.by_name(name)
    pl = W.plan_std(name, J)
    Su, Sd = small()
    check_plan(op, pl, Su, Sd)


def test_helium4_full_plan_matches_oracle():
    # the full 4He operator (2716 patterns, 88M table terms; about a minute of
    # planning on 8 cores); its kinds are numbered by first use in the built-in
    # operator's pattern order, which differs from the oracle's
    op = ops.helium4()
    pl = W.plan_std("4He")
    assert plan_kind_order(op, pl) != sink_kind_order(op)
    assert sorted(plan_kind_order(op, pl)) == list(range(len(op.kinds)))
    check_plan(op, pl, *small(V=2))
    # its term sum takes the factored form: the 364752 prefixes of the best
    # leading pair share 28751 lists, so the words are far fewer than the terms
    w = pl.sum_work()
    assert w["form"] == "factored"
    assert 0 < w["words2"] + w["words1"] < pl.n_terms // 10 and w["segments"] > 0


@pytest.mark.parametrize("seed", range(4))
def test_random_segmented_tables_hold_every_term_once(seed):
    # sparsified A = 3 operators (irregular node and segment structure, a
    # rational unit): the segmented integer-word table holds every term in
    # exactly one word slot, and every segment has at least one word
    rng = np.random.default_rng(7000 + seed)
    base = [ops.helium3, lambda: ops.triton(1)][seed % 2]()
    op = ops.sparsify(base, int(rng.integers(3, 7)), rng, keep_patterns=int(rng.integers(1, 5)))
    pl = W.plan(**to_wick(op))
    if pl.n_terms == 0:
        pytest.skip("the sparsified operator has no terms")
    w = pl.sum_work()
    assert w["form"] == "segmented"
    assert 2 * w["words2"] + w["words1"] == pl.n_terms
    assert 0 < w["segments"] <= w["words2"] + w["words1"]


def test_rational_unit_tables_take_the_integer_word_forms():
    # with the operator scaled by 1/24 the table's coefficients are multiples
    # of 1/24, not integers: the A = 4 table still takes the factored form and
    # the A = 3 one the segmented integer form, with the same word counts as
    # the unscaled operator's
    for base, form in ((ops.helium4, "factored"), (ops.helium3, "segmented")):
        op = ops.sparsify(base(), 4, np.random.default_rng(5001), keep_patterns=2)
        args = to_wick(op)
        pl1 = W.plan(**args)
        pl24 = W.plan(**dict(args, scale=args["scale"] / 24))
        _, coef = pl24.table()
        assert pl24.n_terms > 0 and not np.all(coef.real == np.round(coef.real))
        assert pl24.sum_work()["form"] == form
        assert pl24.sum_work() == pl1.sum_work()


@pytest.mark.parametrize("name,form", [("2H", "packed"), ("3He", "segmented"), ("3H", "segmented")])
def test_term_sum_work_accounts_for_every_term(name, form):
    # every term sits in exactly one word slot of the unfactored forms (a
    # two-leaf word holds two terms), and every segment is a lane with work
    pl = W.plan_std(name)
    w = pl.sum_work()
    assert w["form"] == form
    assert 2 * w["words2"] + w["words1"] == pl.n_terms
    if form == "segmented":
        assert 0 < w["segments"] <= w["words2"] + w["words1"]


@pytest.mark.parametrize("a", [0, 1, 2, 3])
def test_proton_plan_matches_oracle(a):
    op = ops.proton(a)
    pl = W.plan_std("1H", a)
    check_plan(op, pl, *small())
    # the printed single-proton expression has two terms per source index set
    assert pl.stats()["n_enumerated"] == pl.stats()["n_groups"]


def test_general_plan_equals_std_plan():
    op = ops.deuteron()
    p1 = W.plan(**to_wick(op))
    p2 = W.plan_std("2H")
    k1, c1 = p1.table()
    k2, c2 = p2.table()
    Su, Sd = small()
    v1 = eval_table(k1, c1, oracle_compact_blocks(op, plan_kind_order(op, p1), Su, Sd))[0]
    v2 = eval_table(k2, c2, oracle_compact_blocks(op, plan_kind_order(op, p2), Su, Sd))[0]
    assert abs(v1 - v2) <= 1e-13 * abs(v1)


@pytest.mark.parametrize("name,keep,pats,seed", [("3He", 6, 3, 1), ("4He", 6, 4, 2), ("3H", 8, 4, 3)])
def test_sparse_plan_matches_oracle(name, keep, pats, seed):
    for s in range(seed, seed + 200):
        op = ops.sparsify(ops.by_name(name), keep, np.random.default_rng(s), keep_patterns=pats)
        if oracle.source_group_count(op) > 0:
            break
    pl = W.plan(**to_wick(op))
    assert pl.n_terms > 0
    check_plan(op, pl, *small(V=2))


def test_sink_nucleon_swap_flips_sign():
    op = ops.helium3()
    swap = lambda p: (p[1], p[0], p[2])
    op2 = ops.Operator(3, op.kinds, [(swap(p), c) for p, c in op.snk], op.src)
    Su, Sd = small()
    v1, m1 = check_plan(op, W.plan(**to_wick(op)), Su, Sd)
    v2, _ = check_plan(op2, W.plan(**to_wick(op2)), Su, Sd)
    assert abs(v1 + v2) <= 1e-12 * m1


# ---------------------------------------------------------- counts / dedup
def test_deuteron_nine_assignment_classes():
    # n_u! n_d! / 2^A = 9 independent terms per index set (Sec. 4, TF deuteron)
    st = W.plan_std("2H").stats()
    assert st["n_groups"] == 356
    assert st["n_enumerated"] == st["n_groups"] * 2 * 9


def test_helium3_assignment_classes():
    st = W.plan_std("3He").stats()
    assert st["n_groups"] == 1026
    assert st["n_enumerated"] == 1026 * 4 * (math.factorial(5) * math.factorial(4) // 8)


def test_plan_independent_of_hash_seed_and_toy_lattice():
    # the minimal set depends on neither the propagator nor the lattice (Sec. 3.2)
    op = ops.deuteron()
    a = W.plan(**to_wick(op), hash_seed=11, hash_sites=8)
    b = W.plan(**to_wick(op), hash_seed=12345, hash_sites=27, hash_trials=3)
    ka, ca = a.table()
    kb, cb = b.table()
    assert np.array_equal(ka, kb) and np.array_equal(ca, cb)
    assert a.stats()["false_merge_bound"] < 1e-20


P61 = (1 << 61) - 1


def _fp_blocks(op, order, rng, V=3):
    """F_p blocks (Eq. 2.4 form, compact) from random F_p propagators; python ints."""
    S = [rng.integers(0, 2**61 - 1, size=(V, 12, 12), dtype=np.int64).astype(object) for _ in range(2)]
    out = []
    from tests.helpers import pair_index
    for k in order:
        kd = op.kinds[k]
        B = np.zeros(792, dtype=object)
        for x in range(V):
            f, g = S[kd.flavors[0]][x], S[kd.flavors[1]][x]
            for (j1, j2, j3, wr, wi_) in kd.w:
                for i3 in range(12):
                    for i1 in range(i3):
                        uu = (f[j1, i1] * f[j3, i3] - f[j3, i1] * f[j1, i3]) * wr
                        for i2 in range(12):
                            B[pair_index(i1, i3) * 12 + i2] += uu * g[j2, i2]
        out.append(B % P61)
    return np.stack(out)


def test_dedup_equals_full_sum_exactly_in_Fp():
    """The deduplicated table and the full Wick sum agree exactly on fresh F_p propagators."""
    op = ops.deuteron()
    pl = W.plan(**to_wick(op), hash_seed=99)
    kidx, coef = pl.table()
    cint = np.round(coef.real).astype(np.int64)
    assert np.all(cint == coef.real)
    rng = np.random.default_rng(2024)
    order = plan_kind_order(op, pl)
    assert order == sink_kind_order(op)  # a general plan numbers kinds by first use at the sink
    Bp = _fp_blocks(op, order, rng).reshape(-1)
    table = 0
    for n in range(kidx.shape[1]):
        t = int(cint[n])
        for a in range(kidx.shape[0]):
            t = t * int(Bp[kidx[a, n]]) % P61
        table = (table + t) % P61
    # full sum: every source tuple, every bijection, with the full sign
    import itertools
    pos = {k: i for i, k in enumerate(order)}
    full = 0
    for psk, cs in op.snk:
        f = [fl for k in psk for fl in op.kinds[k].flavors]
        for psr, csr in op.src:
            g = [fl for k in psr for fl in op.kinds[k].flavors]
            # raw block in F_p from the compact antisymmetric one is not needed: use
            # the antisymmetrised blocks and half the bijections (slot1 < slot3 handled by sign)
            sigmas = []
            for perm in itertools.permutations(range(6)):
                if all(f[q] == g[perm[q]] for q in range(6)):
                    inv = sum(1 for i in range(6) for j in range(i + 1, 6) if perm[i] > perm[j])
                    sigmas.append((perm, -1 if inv % 2 else 1))
            w0 = op.kinds[psr[0]].w
            w1 = op.kinds[psr[1]].w
            for e0 in w0:
                for e1 in w1:
                    I = [e0[0], e0[1], e0[2], e1[0], e1[1], e1[2]]
                    wI = e0[3] * e1[3] * csr[0] * cs[0]
                    for perm, sg in sigmas:
                        t = wI * sg
                        for a in range(2):
                            i1, i2, i3 = (I[perm[3 * a]], I[perm[3 * a + 1]], I[perm[3 * a + 2]])
                            if i1 == i3:
                                t = 0
                                break
                            from tests.helpers import pair_index
                            c = pair_index(min(i1, i3), max(i1, i3)) * 12 + i2
                            v = int(Bp[pos[psk[a]] * 792 + c])
                            if i1 > i3:
                                v = -v
                            t = t * v
                        full = (full + t) % P61
    # every bijection is counted with both orders of the two same-flavor slots:
    # the antisymmetrised block counts each raw product twice
    inv4 = pow(4, P61 - 2, P61)
    assert table == full * inv4 % P61


# --------------------------------------------------------------- plan files
def test_plan_save_load_roundtrip(tmp_path):
    p = W.plan_std("3He")
    path = tmp_path / "he3.plan"
    p.save(path)
    q = W.Plan.load(path)
    k1, c1 = p.table()
    k2, c2 = q.table()
    assert np.array_equal(k1, k2) and np.array_equal(c1, c2)
    assert q.stats() == p.stats()


def test_corrupt_plan_file_is_rejected(tmp_path):
    p = W.plan_std("2H")
    path = tmp_path / "d.plan"
    p.save(path)
    raw = bytearray(path.read_bytes())
    raw[100] ^= 0xFF
    path.write_bytes(bytes(raw))
    with pytest.raises(W.WickError) as e:
        W.Plan.load(path)
    assert e.value.status == -5
    path.write_bytes(b"nonsense")
    with pytest.raises(W.WickError) as e:
        W.Plan.load(path)
    assert e.value.status == -5


# ----------------------------------------------------------- invalid input
def test_invalid_inputs_are_rejected():
    op = ops.deuteron()
    args = to_wick(op)
    with pytest.raises(W.WickError) as e:
        W.plan(**dict(args, A=0))
    assert e.value.status == -1
    bad = dict(args, snk=[((0, 99), (1, 0))])
    with pytest.raises(W.WickError) as e:
        W.plan(**bad)
    assert e.value.status == -1
    uuu = [((0, 0, 0), [(0, 1, 2, 1, 0)])]
    with pytest.raises(W.WickError) as e:
        W.plan(A=1, kinds=uuu, snk=[((0,), (1, 0))], src=[((0,), (1, 0))])
    assert e.value.status == -4
    with pytest.raises(W.WickError):
        W.plan_std("12C")
    with pytest.raises(W.WickError):
        W.plan(**dict(args, hash_sites=1))


def test_pauli_operator_gives_empty_table():
    op = ops.deuteron()
    src_kinds = [(k.flavors, [(j1, j2, j1, a, b) for (j1, j2, j3, a, b) in k.w]) for k in op.kinds]
    kinds = [(k.flavors, k.w) for k in op.kinds] + src_kinds
    K = len(op.kinds)
    src = [(tuple(i + K for i in p), c) for p, c in op.src]
    pl = W.plan(A=2, kinds=kinds, snk=op.snk, src=src)
    assert pl.n_terms == 0 and pl.stats()["n_groups"] == 0


def test_autotune_rejects_bad_arguments_and_corrupt_cache(tmp_path):
    # argument and cache-file checks come before any device work
    pl = W.plan_std("2H")
    with pytest.raises(W.WickError) as e:
        W.autotune(pl, (4, 0, 4, 8))
    assert e.value.status == W.EINVAL
    bad = tmp_path / "tune.txt"
    bad.write_text("not a tune cache\n")
    with pytest.raises(W.WickError) as e:
        W.autotune(pl, (4, 4, 4, 8), cache_path=bad)
    assert e.value.status == W.ECORRUPT
    bad.write_text("wick-tune 1\nblocks some:key 256\n")  # a field missing
    with pytest.raises(W.WickError) as e:
        W.autotune(pl, (4, 4, 4, 8), cache_path=bad)
    assert e.value.status == W.ECORRUPT
    bad.write_text("wick-tune 1\ncontract some:key -5\n")
    with pytest.raises(W.WickError) as e:
        W.autotune(pl, (4, 4, 4, 8), cache_path=bad)
    assert e.value.status == W.ECORRUPT
    bad.write_text("wick-tune 1\ncontract some:key 99999999999999\n")  # absurd slice length
    with pytest.raises(W.WickError) as e:
        W.autotune(pl, (4, 4, 4, 8), cache_path=bad)
    assert e.value.status == W.ECORRUPT


def test_complex_coefficient_plan_matches_oracle():
    op = ops.deuteron()
    snk = [(k, (c[0] - 2 * c[1], 2 * c[0] + c[1])) for k, c in op.snk]
    src = [(k, (2 * c[0] + c[1], -c[0] + 2 * c[1])) for k, c in op.src]
    opc = ops.Operator(op.A, op.kinds, snk, src, op.scale, "2H-complex")
    pl = W.plan(**to_wick(opc))
    got, mag = check_plan(opc, pl, *small())
    # the complex couplings multiply C by (1 + 2i)(2 - i) = 4 + 3i
    ref, _ = check_plan(op, W.plan_std("2H"), *small())
    assert abs(got - (4 + 3j) * ref) <= 1e-12 * 5 * mag


def _fnv1a(b):
    h = 1469598103934665603
    for c in b:
        h = ((h ^ c) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


@pytest.mark.parametrize("offset,value", [(64, 100), (52, 7), (48, 1)])
def test_plan_file_with_valid_checksum_but_bad_kind_is_rejected(tmp_path, offset, value):
    # a crafted file whose checksum matches: a spin-color index outside [0, 12),
    # a flavor outside {0, 1}, slot flavors that are not (f, g, f)
    import struct
    pl = W.plan_std("2H")
    path = tmp_path / "p.plan"
    pl.save(path)
    raw = bytearray(open(path, "rb").read())
    body = raw[8:-8]
    if offset == 64:
        body[offset] = value                    # first weight's j1
    else:
        body[offset:offset + 4] = struct.pack("<i", value)  # a slot flavor of kind 0
    out = bytes(raw[:8]) + bytes(body) + struct.pack("<Q", _fnv1a(bytes(body)))
    open(path, "wb").write(out)
    with pytest.raises(W.WickError) as e:
        W.Plan.load(path)
    assert e.value.status == W.ECORRUPT
