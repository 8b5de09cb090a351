"""Seeded random scenarios through the GPU path against the oracle: sparsified
operators (any coefficient tensor is a legal operator) on random lattice shapes
and storage types through blocks + contract, and random mixes of built-in
nuclei through the batched entry point, eager and graph-replayed."""
import numpy as np
import pytest

import oracle
import wick_inputs as wi
from oracle import operators as ops
from tests.helpers import eval_table, oracle_compact_blocks, plan_kind_order, to_wick

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def W():
    import paper_2411_08962_amd as w
    return w


def props(wid, n_cfg, dims, dtype):
    torch = _torch()
    hu = np.stack([wi.propagator(wid, c, 0, dims, dtype) for c in range(n_cfg)])
    hd = np.stack([wi.propagator(wid, c, 1, dims, dtype) for c in range(n_cfg)])
    return hu, hd, torch.from_numpy(hu).cuda(), torch.from_numpy(hd).cuda()


def check(op, pl, C, hu, hd, cfg, row):
    kidx, coef = pl.table()
    for t in range(hu.shape[1]):
        su, sd = hu[cfg, t].astype(np.complex128), hd[cfg, t].astype(np.complex128)
        Bc = oracle_compact_blocks(op, plan_kind_order(op, pl), su, sd)
        _, mag = eval_table(kidx, coef, Bc)
        ref = op.scale * oracle.sum_dp(op, oracle.blocks_raw(op, su, sd))
        got = C[row, t, 0] + 1j * C[row, t, 1]
        assert abs(got - ref) <= 1e-12 * max(mag, 1e-300), (t, got, ref, mag)


@pytest.mark.parametrize("seed", range(6))
def test_random_sparse_operator(seed):
    rng = np.random.default_rng(1000 + seed)
    base = [ops.deuteron, ops.helium3, lambda: ops.triton(1), ops.helium4][seed % 4]()
    op = ops.sparsify(base, int(rng.integers(3, 9)), rng, keep_patterns=int(rng.integers(1, 4)))
    dims = tuple(int(v) for v in rng.integers(1, 5, size=3)) + (int(rng.integers(1, 3)),)
    dtype = [np.complex128, np.complex64][seed % 2]
    w = W()
    pl = w.plan(**to_wick(op))
    if pl.n_terms == 0:
        pytest.skip("the sparsified operator has no terms")
    hu, hd, du, dd = props(2000 + seed, 1, dims, dtype)
    C = w.contract(pl, w.blocks(pl, du, dd)).cpu().numpy()
    check(op, pl, C, hu, hd, 0, 0)


@pytest.mark.parametrize("seed", range(4))
def test_random_batches_of_builtin_nuclei(seed):
    rng = np.random.default_rng(3000 + seed)
    names = ["2H", "3He", "3H"]
    n_cfg = int(rng.integers(1, 4))
    dims = tuple(int(v) for v in rng.integers(2, 5, size=3)) + (int(rng.integers(1, 4)),)
    dtype = [np.complex128, np.complex64][seed % 2]
    w = W()
    plans = [w.plan_std(n) for n in names]
    makers = [ops.deuteron, ops.helium3, ops.triton]
    items = [(int(rng.integers(0, 3)), int(rng.integers(0, n_cfg))) for _ in range(int(rng.integers(1, 6)))]
    hu, hd, du, dd = props(4000 + seed, n_cfg, dims, dtype)
    for use_graph in (False, True, True):
        C = w.correlator(plans, items, du, dd, use_graph=use_graph).cpu().numpy()
        for row, (pi, cfg) in enumerate(items):
            check(makers[pi](), plans[pi], C, hu, hd, cfg, row)


@pytest.mark.parametrize("seed", [1, 3, 4, 6])
@pytest.mark.parametrize("piece", ["8", "13", "256"])
def test_random_helium4_factored_term_sum(monkeypatch, seed, piece):
    # sparsified 4He operators (A = 4, coefficients multiples of one rational
    # unit: the factored table form; 97k to 227k terms) with list pieces of 8,
    # 13 or 256 words, so that lists split into many pieces and the switch from
    # prefix-group to list words falls at many offsets of the 8-word blocks the
    # kernel prefetches; against the oracle through wick_contract, and with
    # the palette and packed forms of the same operator (the batched entry
    # point takes kinds of nucleon form only: the full 4He batch covers the
    # factored form there)
    rng = np.random.default_rng(5000 + seed)
    op = ops.sparsify(ops.helium4(), int(rng.integers(3, 6)), rng, keep_patterns=int(rng.integers(1, 4)))
    dims = (2, 2, 1, 2)
    w = W()
    monkeypatch.setenv("WICK_PIECE_WORDS", piece)
    hu, hd, du, dd = props(6000 + seed, 1, dims, np.complex128)
    for form in ("segmented", "segmented-palette", "packed"):
        monkeypatch.setenv("WICK_TABLE_FORM", form)
        pl = w.plan(**to_wick(op))  # a fresh plan: its table is built under this form
        assert pl.n_terms > 0
        work = pl.sum_work()
        assert work["form"] == {"segmented": "factored", "segmented-palette": "segmented-palette",
                                "packed": "packed"}[form]
        C = w.contract(pl, w.blocks(pl, du, dd)).cpu().numpy()
        check(op, pl, C, hu, hd, 0, 0)
