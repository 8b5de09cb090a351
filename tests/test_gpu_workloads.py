"""GPU parity at the full sizes of the benchmark workloads, on sampled outputs.

Each test runs the HIP path in the launch configuration bench.py times and
checks sampled (configuration, time slice) correlators against the oracle
(blocks by direct sums, then the subset-DP term sum), with the bound
|dC| <= tol * sum_n |term_n| (sum over the deduplicated table evaluated with
the oracle's blocks): 1e-12 for FP64 blocks, 1e-8 for FP32 and three BF16
limbs, 1e-6 for two BF16 limbs.
"""
import numpy as np
import pytest

import oracle
import wick_inputs as wi
from oracle import operators as ops
from tests.helpers import eval_table

pytestmark = pytest.mark.gpu

TOL = {"p64": 1e-12, "p32": 1e-8, "pb6": 1e-8, "pb3": 1e-6}
_PLANS = {}


def plan(name):
    import paper_2411_08962_amd as w
    if name not in _PLANS:
        _PLANS[name] = w.plan_std(name)
    return _PLANS[name]


def props(wid, n_cfg, dims, dtype=np.complex128):
    import torch
    X, Y, Z, T = dims
    hu = np.empty((n_cfg, T, Z, Y, X, 12, 12), dtype=dtype)
    hd = np.empty_like(hu)
    for c in range(n_cfg):
        hu[c] = wi.propagator(wid, c, 0, dims, dtype)
        hd[c] = wi.propagator(wid, c, 1, dims, dtype)
    return hu, hd, torch.from_numpy(hu).cuda(), torch.from_numpy(hd).cuda()


def reference(name, hu, hd, cfg, t):
    """Oracle C(t) and sum_n |term_n| of the plan's table with the oracle's blocks."""
    from tests.helpers import oracle_compact_blocks, plan_kind_order
    op = ops.by_name(name)
    su, sd = hu[cfg, t].astype(np.complex128), hd[cfg, t].astype(np.complex128)
    ref = op.scale * oracle.sum_dp(op, oracle.blocks_raw(op, su, sd))
    pl = plan(name)
    kidx, coef = pl.table()
    tab, mag = eval_table(kidx, coef, oracle_compact_blocks(op, plan_kind_order(op, pl), su, sd))
    assert abs(tab - ref) <= 1e-12 * mag  # the table itself is right (host)
    return ref, mag


def test_helium4_24cubed_x48_per_t_error():
    """4He on 24^3 x 48 (complex128): FP64, FP32, two-limb and three-limb BF16
    blocks, each followed by the FP64 term sum; per-time-slice error against
    the oracle on eight slices spanning the lattice (first and last included):
    |dC| / sum|terms| is asserted, |dC| / |C| is printed beside it."""
    import paper_2411_08962_amd as w
    pl = plan("4He")
    hu, hd, du, dd = props(3, 1, (24, 24, 24, 48))
    precs = ("p64", "p32", "pb3", "pb6")
    Cs = {p: w.contract(pl, w.blocks(pl, du, dd, p)).cpu().numpy() for p in precs}
    print("\n  t  " + "  ".join(f"{p}: dC/sum|terms|  dC/|C|  " for p in precs), flush=True)
    for t in (0, 7, 13, 20, 27, 34, 41, 47):
        ref, mag = reference("4He", hu, hd, 0, t)
        row, bad = [], []
        for p, C in Cs.items():
            d = abs(C[0, t, 0] + 1j * C[0, t, 1] - ref)
            row.append(f"{d / mag:9.2e} {d / abs(ref):9.2e}")
            if d / mag > TOL[p]:
                bad.append((p, t, d / mag))
        print(f" {t:2d}  " + "    ".join(row), flush=True)
        assert not bad, bad


def test_lithium7_clusters_32cubed_x64():
    """7Li as the product of the 4He and 3H cluster correlators on 32^3 x 64,
    both computed in one batched launch with FP32 blocks (and FP64 once)."""
    import paper_2411_08962_amd as w
    plans = [plan("4He"), plan("3H")]
    hu, hd, du, dd = props(4, 1, (32, 32, 32, 64))
    for prec in ("p32", "p64"):
        C = w.correlator(plans, [(0, 0), (1, 0)], du, dd, prec, use_graph=True).cpu().numpy()
        for t in (0, 63):
            r4, m4 = reference("4He", hu, hd, 0, t)
            r3, m3 = reference("3H", hu, hd, 0, t)
            c4 = C[0, t, 0] + 1j * C[0, t, 1]
            c3 = C[1, t, 0] + 1j * C[1, t, 1]
            assert abs(c4 - r4) <= TOL[prec] * m4, (prec, t, "4He")
            assert abs(c3 - r3) <= TOL[prec] * m3, (prec, t, "3H")
            # the cluster product inherits both bounds to first order
            bound = TOL[prec] * (m4 * abs(r3) + m3 * abs(r4)) * (1 + 1e-6)
            assert abs(c4 * c3 - r4 * r3) <= bound, (prec, t, "7Li")


def test_batch64_mixed_nuclei_c64_graph():
    """64 complex64 configurations of 16^3 x 32: 2H on 0-7, 3He on 8-31, 4He on
    32-63, one graph-captured batch with FP32 and with FP64 blocks; sampled
    items against the oracle (which reads the same complex64 values), and for
    each precision a second replay equal to the first bitwise."""
    import torch
    import paper_2411_08962_amd as w
    names = ["2H", "3He", "4He"]
    plans = [plan(n) for n in names]
    items = [(0, c) for c in range(8)] + [(1, c) for c in range(8, 32)] + [(2, c) for c in range(32, 64)]
    hu, hd, du, dd = props(5, 64, (16, 16, 16, 32), np.complex64)
    out = torch.empty((64, 32, 2), dtype=torch.float64, device="cuda")
    got = {}
    for prec in ("p32", "p64"):
        w.correlator(plans, items, du, dd, prec, use_graph=True, out=out)
        torch.cuda.synchronize()
        got[prec] = out.cpu().numpy()
        out.zero_()
        w.correlator(plans, items, du, dd, prec, use_graph=True, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), got[prec]), prec
    for i, t in ((3, 0), (3, 31), (17, 5), (40, 0), (63, 31)):
        name = names[items[i][0]]
        ref, mag = reference(name, hu, hd, items[i][1], t)
        for prec, C in got.items():
            c = C[i, t, 0] + 1j * C[i, t, 1]
            assert abs(c - ref) <= TOL[prec] * mag, (prec, i, name, t, abs(c - ref) / mag)
