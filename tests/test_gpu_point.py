"""GPU parity of the point-sink determinant path (Eq. 2.9, App. A Eq. A1)
against the oracle's point-sink route (one-site blocks and the DP route per
site, no determinants). Bound: |C_gpu - C_oracle| <= 1e-12 * sum over sites
of sum_{g,h} |W_g W'_h det_u det_d| (the absolute terms of the determinant
form, from numpy determinants)."""
import ctypes

import numpy as np
import pytest

import oracle
import wick_inputs as wi
from oracle import operators as ops
from tests.helpers import to_wick

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    return torch


def W():
    import paper_2411_08962_amd as w
    return w


def props(wid, n_cfg, dims, dtype=np.complex128):
    torch = _torch()
    hu = np.stack([wi.propagator(wid, c, 0, dims, dtype) for c in range(n_cfg)])
    hd = np.stack([wi.propagator(wid, c, 1, dims, dtype) for c in range(n_cfg)])
    return hu, hd, torch.from_numpy(hu).cuda(), torch.from_numpy(hd).cuda()


def check(op, pp, hu, hd, C, cfg=0):
    su, sd = hu[cfg].astype(np.complex128), hd[cfg].astype(np.complex128)
    ref = oracle.point_correlator(op, su, sd)
    mag = oracle.point_det_magnitude(op, su, sd)
    got = C[cfg, :, 0] + 1j * C[cfg, :, 1]
    rel = np.abs(got - ref) / mag
    assert np.all(rel <= TOL), (rel, got, ref)
    return rel.max()


CASES = [
    ("1H", lambda: ops.proton(1), (3, 2, 2, 3)),
    ("2H", ops.deuteron, (2, 2, 2, 2)),
    ("3He", ops.helium3, (2, 2, 1, 2)),
    ("3H", lambda: ops.triton(1), (2, 1, 1, 2)),
    ("4He", ops.helium4, (2, 1, 1, 1)),
]


@pytest.mark.parametrize("name,make,dims", CASES, ids=[c[0] for c in CASES])
def test_point_correlator_matches_oracle(name, make, dims):
    w = W()
    op = make()
    pp = w.point_plan(**to_wick(op))
    hu, hd, du, dd = props(961, 1, dims)
    C = w.point_correlator(pp, du, dd).cpu().numpy()
    check(op, pp, hu, hd, C)


def test_point_std_plan_two_configurations_and_repeatability():
    w = W()
    op = ops.deuteron()
    pp = w.point_plan_std("2H")
    hu, hd, du, dd = props(962, 2, (2, 2, 1, 3))
    C1 = w.point_correlator(pp, du, dd).cpu().numpy()
    C2 = w.point_correlator(pp, du, dd).cpu().numpy()
    assert np.array_equal(C1, C2)  # deterministic
    for cfg in range(2):
        check(op, pp, hu, hd, C1, cfg)


def test_point_complex64_storage():
    w = W()
    op = ops.deuteron()
    pp = w.point_plan_std("2H")
    hu, hd, du, dd = props(963, 1, (2, 2, 2, 2), np.complex64)
    C = w.point_correlator(pp, du, dd).cpu().numpy()
    check(op, pp, hu, hd, C)


def test_point_many_site_chunks():
    # 6^3 x 6 = 1296 site-slices: more than one chunk of the d-minor workspace for 2H
    w = W()
    op = ops.deuteron()
    pp = w.point_plan_std("2H")
    hu, hd, du, dd = props(964, 1, (6, 6, 6, 6))
    C = w.point_correlator(pp, du, dd).cpu().numpy()
    check(op, pp, hu, hd, C)


@pytest.mark.parametrize("name", ["2H", "3He", "4He"])
def test_point_equals_plane_wave_on_one_site(name):
    # on a one-site lattice a point sink and nucleon sinks at zero momentum coincide
    w = W()
    pp = w.point_plan_std(name)
    pl = w.plan_std(name)
    hu, hd, du, dd = props(965, 1, (1, 1, 1, 3))
    Cp = w.point_correlator(pp, du, dd).cpu().numpy()
    Cb = w.contract(pl, w.blocks(pl, du, dd)).cpu().numpy()
    op = ops.by_name(name)
    mag = oracle.point_det_magnitude(op, hu[0], hd[0])
    d = np.abs((Cp[0, :, 0] - Cb[0, :, 0]) + 1j * (Cp[0, :, 1] - Cb[0, :, 1]))
    assert np.all(d <= 10 * TOL * mag), (d, mag)


def test_point_single_nucleon_equals_plane_wave_on_a_lattice():
    w = W()
    pp = w.point_plan_std("1H", 2)
    pl = w.plan_std("1H", 2)
    hu, hd, du, dd = props(966, 1, (4, 4, 4, 4))
    Cp = w.point_correlator(pp, du, dd).cpu().numpy()
    Cb = w.contract(pl, w.blocks(pl, du, dd)).cpu().numpy()
    op = ops.proton(2)
    mag = oracle.point_det_magnitude(op, hu[0], hd[0])
    d = np.abs((Cp[0, :, 0] - Cb[0, :, 0]) + 1j * (Cp[0, :, 1] - Cb[0, :, 1]))
    assert np.all(d <= 10 * TOL * mag)


def test_point_pauli_operator_gives_zero():
    # every weight repeats a u index: no sink group survives, C = 0
    w = W()
    kinds = [((0, 1, 0), [(0, 1, 0, 1, 0), (3, 2, 3, 1, 0)])]
    pp = w.point_plan(A=1, kinds=kinds, snk=[((0,), (1, 0))], src=[((0,), (1, 0))])
    assert pp.info()["n_sink_groups"] == 0
    hu, hd, du, dd = props(967, 1, (2, 1, 1, 2))
    C = _torch().full((1, 2, 2), 7.0, dtype=_torch().float64, device="cuda")
    w.point_correlator(pp, du, dd, out=C)
    assert np.all(C.cpu().numpy() == 0)


def test_point_argument_errors():
    w = W()
    torch = _torch()
    pp = w.point_plan_std("2H")
    hu, hd, du, dd = props(968, 1, (2, 1, 1, 2))
    L = w.lib()
    C = torch.zeros((1, 2, 2), dtype=torch.float64, device="cuda")
    dims = (ctypes.c_int32 * 4)(2, 1, 1, 2)
    P = ctypes.c_void_p
    s = P(torch.cuda.current_stream().cuda_stream)
    ok = L.wick_point_correlator(pp.handle, P(du.data_ptr()), P(dd.data_ptr()), 0, dims, 1, s, P(C.data_ptr()))
    assert ok == w.OK
    assert L.wick_point_correlator(None, P(du.data_ptr()), P(dd.data_ptr()), 0, dims, 1, s, P(C.data_ptr())) == w.EINVAL
    assert L.wick_point_correlator(pp.handle, None, P(dd.data_ptr()), 0, dims, 1, s, P(C.data_ptr())) == w.EINVAL
    assert L.wick_point_correlator(pp.handle, P(du.data_ptr() + 8), P(dd.data_ptr()), 0, dims, 1, s,
                                   P(C.data_ptr())) == w.EINVAL
    bad = (ctypes.c_int32 * 4)(2, 0, 1, 2)
    assert L.wick_point_correlator(pp.handle, P(du.data_ptr()), P(dd.data_ptr()), 0, bad, 1, s, P(C.data_ptr())) == w.EINVAL
    assert L.wick_point_correlator(pp.handle, P(du.data_ptr()), P(dd.data_ptr()), 7, dims, 1, s, P(C.data_ptr())) == w.EINVAL
    torch.cuda.synchronize()


# ------------------------------------------------ block form (Eq. 3.1)
BLOCK_CASES = [
    ("1H", lambda: ops.proton(1), (3, 2, 2, 3)),
    ("2H", ops.deuteron, (2, 2, 2, 2)),
    ("3He", ops.helium3, (2, 2, 1, 2)),
    ("4He", ops.helium4, (2, 1, 1, 1)),
]


@pytest.mark.parametrize("name,make,dims", BLOCK_CASES, ids=[c[0] for c in BLOCK_CASES])
def test_point_block_form_matches_oracle(name, make, dims):
    w = W()
    op = make()
    pl = w.plan_std(name, 1) if name == "1H" else w.plan_std(name)
    hu, hd, du, dd = props(971, 1, dims)
    C = w.point_blocks_correlator(pl, du, dd).cpu().numpy()
    check(op, None, hu, hd, C)


def test_point_block_form_equals_determinants_on_a_lattice():
    # the two routes to the same point-sink correlator, on 4^3 x 3 (2H), 3x3x2 x 2 (3He)
    # and 2x2x2 x 2 (4He: the block form's term sum takes the factored table)
    w = W()
    for name, op, dims in (("2H", ops.deuteron(), (4, 4, 4, 3)), ("3He", ops.helium3(), (3, 3, 2, 2)),
                           ("4He", ops.helium4(), (2, 2, 2, 2))):
        hu, hd, du, dd = props(972, 1, dims)
        Cb = w.point_blocks_correlator(w.plan_std(name), du, dd).cpu().numpy()[0]
        Cd = w.point_correlator(w.point_plan_std(name), du, dd).cpu().numpy()[0]
        mag = oracle.point_det_magnitude(op, hu[0], hd[0])
        d = np.abs((Cb[:, 0] - Cd[:, 0]) + 1j * (Cb[:, 1] - Cd[:, 1]))
        assert np.all(d <= 10 * TOL * mag), (name, d, mag)


def test_point_block_form_general_plan_complex64_and_empty():
    w = W()
    op = ops.sparsify(ops.helium3(), 6, np.random.default_rng(4))
    pl = w.plan(**to_wick(op))
    hu, hd, du, dd = props(973, 1, (2, 2, 1, 2), np.complex64)
    C = w.point_blocks_correlator(pl, du, dd).cpu().numpy()
    check(op, None, hu, hd, C)
    # a plan whose table is empty gives zeros
    kinds = [((0, 1, 0), [(0, 1, 0, 1, 0), (3, 2, 3, 1, 0)])]
    pe = w.plan(A=1, kinds=kinds, snk=[((0,), (1, 0))], src=[((0,), (1, 0))])
    assert pe.n_terms == 0
    Cz = _torch().full((1, 2, 2), 5.0, dtype=_torch().float64, device="cuda")
    w.point_blocks_correlator(pe, du, dd, out=Cz)
    assert np.all(Cz.cpu().numpy() == 0)


def test_point_routes_agree_full_size():
    """Determinants and the block form on the benchmark lattice (24^3; two time
    slices, one for 4He): two independent algorithms for the same point-sink
    correlator."""
    w = W()
    for name in ("2H", "3He", "4He"):
        hu, hd, du, dd = props(974, 1, (24, 24, 24, 1 if name == "4He" else 2))
        Cd = w.point_correlator(w.point_plan_std(name), du, dd).cpu().numpy()[0]
        Cb = w.point_blocks_correlator(w.plan_std(name), du, dd).cpu().numpy()[0]
        a, b = Cd[:, 0] + 1j * Cd[:, 1], Cb[:, 0] + 1j * Cb[:, 1]
        assert np.all(np.abs(a - b) <= 1e-9 * np.abs(a)), (name, a, b)
