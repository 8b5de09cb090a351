"""GPU parity of correlation matrices for the GEVP (Eqs. E1-E3): blocks of
the matrix's kinds (wick_blocks on the borrowed plan) and the union term sum,
every element against the oracle's correlator of that element's operator.
Bound per element and slice: 1e-12 * sum_n |term_n| of the element (the
oracle's merged terms on the oracle's blocks)."""
import numpy as np
import pytest

import oracle
import wick_inputs as wi
from oracle import operators as ops
from tests.helpers import gevp_element, to_wick

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def W():
    import paper_2411_08962_amd as w
    return w


def props(wid, dims):
    torch = _torch()
    hu = wi.propagator(wid, 0, 0, dims)[None]
    hd = wi.propagator(wid, 0, 1, dims)[None]
    return hu, hd, torch.from_numpy(hu).cuda(), torch.from_numpy(hd).cuda()


def complex_deuteron():
    op = ops.deuteron(-1)
    snk = [(p, (0, c[0])) for p, c in op.snk]  # i times the P_- operator
    return ops.Operator(2, op.kinds, snk, list(snk), 1.0, "i2H(-1)")


BASES = {
    "2H-three": lambda: [ops.deuteron(+1), ops.deuteron(-1), ops.deuteron(0)],
    "2H-four-complex": lambda: [ops.deuteron(+1), ops.deuteron(-1), ops.deuteron(0), complex_deuteron()],
    "3He-spins": lambda: [ops.helium3(0), ops.helium3(1)],
}


@pytest.mark.parametrize("name", sorted(BASES))
def test_gevp_matrix_matches_oracle(name):
    w = W()
    op_list = BASES[name]()
    n = len(op_list)
    g = w.gevp_plan([to_wick(o) for o in op_list])
    dims = (2, 2, 2, 2) if name.startswith("3He") else (3, 2, 2, 3)
    hu, hd, du, dd = props(991, dims)
    B = w.blocks(g.blocks_plan(), du, dd)
    C = w.gevp_contract(g, B).cpu().numpy()[0]
    C2 = w.gevp_contract(g, B).cpu().numpy()[0]
    assert np.array_equal(C, C2)  # deterministic
    for i in range(n):
        for j in range(n):
            el = gevp_element(op_list, i, j)
            keys, coef = oracle.merged_terms(el)
            for t in range(dims[3]):
                ref = el.scale * oracle.sum_dp(el, oracle.blocks_raw(el, hu[0, t], hd[0, t]))
                Beq = np.stack([oracle.block_eq24(k, hu[0, t], hd[0, t]) for k in el.kinds])[None]
                mag = np.abs(oracle.term_values(keys, coef, Beq)).sum()
                got = C[t, i, j, 0] + 1j * C[t, i, j, 1]
                assert abs(got - ref) <= 1e-12 * mag, (i, j, t, got, ref, mag)


def test_gevp_single_operator_equals_contract():
    w = W()
    g = w.gevp_plan([to_wick(ops.deuteron())])
    pl = w.plan_std("2H")
    hu, hd, du, dd = props(992, (4, 4, 4, 4))
    Cg = w.gevp_contract(g, w.blocks(g.blocks_plan(), du, dd)).cpu().numpy()[0, :, 0, 0]
    Cp = w.contract(pl, w.blocks(pl, du, dd)).cpu().numpy()[0]
    keys, coef = oracle.merged_terms(ops.deuteron())
    for t in range(4):
        Beq = np.stack([oracle.block_eq24(k, hu[0, t], hd[0, t]) for k in ops.deuteron().kinds])[None]
        mag = np.abs(oracle.term_values(keys, coef, Beq)).sum()
        assert abs((Cg[t, 0] - Cp[t, 0]) + 1j * (Cg[t, 1] - Cp[t, 1])) <= 2e-12 * mag


def test_gevp_contract_argument_errors():
    import ctypes
    w = W()
    torch = _torch()
    g = w.gevp_plan([to_wick(ops.deuteron(+1)), to_wick(ops.deuteron(-1))])
    K = g.info()["n_kinds"]
    B = torch.zeros((1, 2, K, 792, 2), dtype=torch.float64, device="cuda")
    C = torch.zeros((1, 2, 2, 2, 2), dtype=torch.float64, device="cuda")
    L = w.lib()
    P = ctypes.c_void_p
    s = P(torch.cuda.current_stream().cuda_stream)
    assert L.wick_gevp_contract(g.handle, P(B.data_ptr()), 1, 2, s, P(C.data_ptr())) == w.OK
    assert L.wick_gevp_contract(None, P(B.data_ptr()), 1, 2, s, P(C.data_ptr())) == w.EINVAL
    assert L.wick_gevp_contract(g.handle, None, 1, 2, s, P(C.data_ptr())) == w.EINVAL
    assert L.wick_gevp_contract(g.handle, P(B.data_ptr() + 8), 1, 2, s, P(C.data_ptr())) == w.EINVAL
    assert L.wick_gevp_contract(g.handle, P(B.data_ptr()), 0, 2, s, P(C.data_ptr())) == w.EINVAL
    torch.cuda.synchronize()
    assert np.all(C.cpu().numpy() == 0)  # zero blocks give a zero matrix
    with pytest.raises(ValueError):
        w.gevp_contract(g, torch.zeros((1, 2, K + 1, 792, 2), dtype=torch.float64, device="cuda"))
