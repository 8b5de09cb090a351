"""The allocation-free term sum, wick_contract_noalloc, against wick_contract.

Both run the same kernels with the same launch shape, so their C(t) must be
bitwise equal; the second call of each pair is smaller than the first, so a
partial sum left in the static scratch array by an earlier call must not
leak into a later one.
"""
import numpy as np
import pytest

import wick_inputs as wi

pytestmark = pytest.mark.gpu


def _blocks(w, pl, wid, n_cfg, dims):
    import torch
    hu = np.stack([wi.propagator(wid, c, 0, dims) for c in range(n_cfg)])
    hd = np.stack([wi.propagator(wid, c, 1, dims) for c in range(n_cfg)])
    return w.blocks(pl, torch.from_numpy(hu).cuda(), torch.from_numpy(hd).cuda())


def test_contract_noalloc_equals_contract_on_shrinking_calls():
    import torch
    import paper_2411_08962_amd as w
    print("wick_contract_noalloc: 3He 2 cfg 4^3x6, then 3He 1 cfg 2^3x3, then 2H 1 cfg 2^3x2", flush=True)
    cases = [("3He", 31, 2, (4, 4, 4, 6)), ("3He", 32, 1, (2, 2, 2, 3)), ("2H", 33, 1, (2, 2, 2, 2))]
    plans = {}
    for name, wid, n_cfg, dims in cases:
        pl = plans.setdefault(name, w.plan_std(name))
        B = _blocks(w, pl, wid, n_cfg, dims)
        ref = w.contract(pl, B)
        out = torch.full((n_cfg, dims[3], 2), float("nan"), dtype=torch.float64, device="cuda")
        w.contract_noalloc(pl, B, out)
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(got)), name
        assert np.array_equal(got, want), (name, n_cfg, dims, np.max(np.abs(got - want)))


def test_contract_noalloc_needs_a_resident_plan():
    import torch
    import paper_2411_08962_amd as w
    pl = w.plan_std("3He")
    B = _blocks(w, pl, 34, 1, (2, 2, 2, 2))
    fresh = w.plan_std("3He")  # same table, never used on this device
    out = torch.zeros((1, 2, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(w.WickError) as e:
        w.contract_noalloc(fresh, B, out)
    assert e.value.status == w.EINVAL and "not on this device" in str(e.value)
    torch.cuda.synchronize()
    assert not torch.any(out != 0)


def test_contract_noalloc_factored_table():
    # an A = 4 table in the factored form (a sparsified 4He operator, 97 200
    # terms): the allocation-free call equals wick_contract bitwise, then again
    # on a smaller set of blocks
    import torch
    import paper_2411_08962_amd as w
    from oracle import operators as ops
    from tests.helpers import to_wick
    print("wick_contract_noalloc: sparsified 4He (factored table) 2x2x1x3, then 1x1x1x1", flush=True)
    rng = np.random.default_rng(5004)
    op = ops.sparsify(ops.helium4(), int(rng.integers(3, 6)), rng, keep_patterns=int(rng.integers(1, 4)))
    pl = w.plan(**to_wick(op))
    assert pl.sum_work()["form"] == "factored"
    for wid, dims in ((35, (2, 2, 1, 3)), (36, (1, 1, 1, 1))):
        B = _blocks(w, pl, wid, 1, dims)
        ref = w.contract(pl, B)
        out = torch.full((1, dims[3], 2), float("nan"), dtype=torch.float64, device="cuda")
        w.contract_noalloc(pl, B, out)
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(got)), dims
        assert np.array_equal(got, want), (dims, np.max(np.abs(got - want)))
