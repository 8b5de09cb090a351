"""Shared test helpers: operator conversion and table evaluation on the CPU."""
import re
import os

import numpy as np

import oracle
from oracle import operators as ops
from oracle.operators import gevp_element  # noqa: F401  (re-exported for the tests)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def pair_index(i1, i3):
    return i3 * (i3 - 1) // 2 + i1


def compact(Bfull):
    """[..., 12, 12, 12] antisymmetric block -> [..., 792] (c = pair(i1<i3)*12 + i2)."""
    out = np.zeros(Bfull.shape[:-3] + (792,), dtype=Bfull.dtype)
    for i3 in range(12):
        for i1 in range(i3):
            for i2 in range(12):
                out[..., pair_index(i1, i3) * 12 + i2] = Bfull[..., i1, i2, i3]
    return out


def oracle_compact_blocks(op, kind_order, Su_t, Sd_t):
    """Oracle blocks in the form of Eq. 2.4 (antisymmetrised), compact, in the plan's kind order."""
    return np.stack([compact(oracle.block_eq24(op.kinds[k], Su_t, Sd_t)) for k in kind_order])


def eval_table(kidx, coef, Bc):
    """sum_n coef_n prod_a Bc.flat[kidx[a, n]] and sum_n |coef_n prod_a ...| (FP64, numpy)."""
    flat = Bc.reshape(-1)
    prod = np.ones(kidx.shape[1], dtype=np.complex128)
    for a in range(kidx.shape[0]):
        prod = prod * flat[kidx[a].astype(np.int64)]
    terms = coef * prod
    return terms.sum(), np.abs(terms).sum()


def to_wick(op):
    """oracle Operator -> the binding's plan() arguments (the same exact integers)."""
    kinds = [(k.flavors, k.w) for k in op.kinds]
    return dict(A=op.A, kinds=kinds, snk=op.snk, src=op.src, scale=op.scale)


def sink_kind_order(op):
    """Kinds used at the sink, in order of first use (the planner's block-kind order)."""
    order = []
    for p, _ in op.snk:
        for k in p:
            if k not in order:
                order.append(k)
    return order


def plan_kind_order(op, pl):
    """For each block kind of the plan, the index of the oracle operator's kind
    with the same flavors and weights (the plan numbers kinds by first use in
    its own sink patterns, which need not follow the oracle's pattern order)."""
    def canon(fl, w):
        return tuple(int(f) for f in fl), tuple(sorted((int(a), int(b), int(c), int(x), int(y)) for a, b, c, x, y in w))
    index = {}
    for i, k in enumerate(op.kinds):
        index.setdefault(canon(k.flavors, k.w), i)
    order = []
    for k in range(pl.n_kinds):
        key = canon(*pl.kind(k))
        assert key in index, f"plan kind {k} has no counterpart in the oracle operator"
        order.append(index[key])
    return order


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "wick.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wick_[a-z_]+)\s*\(", txt)))


def table_entries(op, pl):
    """The plan's table with every index in the oracle's encoding: ent [N, A] with
    ent = oracle_kind * 1728 + i1 * 144 + i2 * 12 + i3 (i1 < i3; the compact index
    c = pair(i1, i3) * 12 + i2 of the C header decoded), rows in table order, and coef [N]."""
    kidx, coef = pl.table()
    order = np.array(plan_kind_order(op, pl), dtype=np.int64)
    dec = np.zeros(792, dtype=np.int64)
    for i3 in range(12):
        for i1 in range(i3):
            for i2 in range(12):
                dec[pair_index(i1, i3) * 12 + i2] = i1 * 144 + i2 * 12 + i3
    k = kidx.astype(np.int64)
    ent = order[k // 792] * 1728 + dec[k % 792]
    return ent.T.copy(), coef


def row_index(keys):
    """{tuple(sorted row): position} for a [N, A] key array."""
    return {tuple(r): i for i, r in enumerate(np.sort(keys, axis=1).tolist())}


def sorted_entries(ent):
    """Rows of an [N, A] oracle-encoded index array, each sorted, as tuples."""
    return [tuple(r) for r in np.sort(ent, axis=1).tolist()]
