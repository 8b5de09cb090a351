"""Point-sink determinant path (Eq. 2.9, method B of Sec. 3.3, App. A): host
side. Pins of the oracle's point-sink route and of the planner's sizes."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2411_08962_amd as W
import wick_inputs as wi
from oracle import operators as ops
from tests.helpers import to_wick


# ------------------------------------------------------------ planner sizes
@pytest.mark.parametrize("name,groups,nu,nd", [("2H", 356, 3, 3), ("3He", 1026, 5, 4), ("4He", 2716, 6, 6)])
def test_point_plan_matches_the_paper_table(name, groups, nu, nd):
    # operator terms and determinant ranks of the method-comparison table (Sec. 3.3)
    info = W.point_plan_std(name).info()
    assert info["n_sink_groups"] == groups and info["n_src_groups"] == groups
    assert (info["n_u"], info["n_d"]) == (nu, nd)


@pytest.mark.parametrize("make", [lambda: ops.proton(0), ops.deuteron, ops.helium3, lambda: ops.triton(1)])
def test_point_plan_row_and_column_sets_match_the_oracle_groups(make):
    op = make()
    pp = W.point_plan(**to_wick(op))
    vals, w = oracle.source_groups(op)
    info = pp.info()
    nu = info["n_u"]
    assert info["n_src_groups"] == len(w) and info["n_sink_groups"] == len(w)
    assert info["n_cols_u"] == len({tuple(v[:nu]) for v in vals.tolist()})
    assert info["n_cols_d"] == len({tuple(v[nu:]) for v in vals.tolist()})
    assert info["n_rows_u"] == info["n_cols_u"] and info["n_rows_d"] == info["n_cols_d"]


def test_point_plan_rejects_bad_operators():
    op = ops.deuteron()
    d = to_wick(op)
    # a source with a different flavor content: two protons against p n
    kp = next(i for i, k in enumerate(op.kinds) if tuple(k.flavors) == (0, 1, 0))
    with pytest.raises(W.WickError) as e:
        W.point_plan(**dict(d, src=[((kp, kp), (1, 0))]))
    assert e.value.status == W.EINVAL
    # more than six quarks of one flavor: four protons
    p = ops.proton(0)
    with pytest.raises(W.WickError) as e:
        W.point_plan(A=4, kinds=[(p.kinds[0].flavors, p.kinds[0].w)], snk=[((0, 0, 0, 0), (1, 0))],
                     src=[((0, 0, 0, 0), (1, 0))])
    assert e.value.status == W.EUNSUPPORTED
    with pytest.raises(W.WickError):
        W.point_plan_std("7Be")
    L = W.lib()
    h = ctypes.c_void_p()
    assert L.wick_point_plan(None, ctypes.byref(h)) == W.EINVAL
    assert L.wick_point_info(None, None, None, None, None, None, None, None, None) == W.EINVAL


# ------------------------------------------------- oracle point route pins
def test_point_route_single_nucleon_equals_plane_wave():
    # with one nucleon the point sink and the zero-momentum nucleon sink coincide
    op = ops.proton(1)
    Su, Sd = wi.propagator_pair(952, 0, (3, 2, 1, 2))
    a = oracle.point_correlator(op, Su, Sd)
    b = oracle.correlator(op, Su, Sd)
    assert np.allclose(a, b, rtol=1e-13, atol=0)


@pytest.mark.parametrize("make", [ops.deuteron, ops.helium3])
def test_point_route_identity_propagator_closed_form(make):
    # S = 1: det S[U; U'] = [U == U'], so C = scale * V * sum_g W_g^2 (sink = source groups)
    op = make()
    V = 2
    S = np.broadcast_to(np.eye(12, dtype=np.complex128), (1, 1, 1, V, 12, 12)).copy()
    c = oracle.point_correlator(op, S, S)[0]
    _, w = oracle.source_groups(op)
    assert abs(c - op.scale * V * np.sum(w * w)) <= 1e-12 * abs(c)


def test_point_route_equals_quark_level_definition_per_site():
    # per site, Wick's theorem quark by quark on the one-site lattice
    op = ops.deuteron()
    Su, Sd = wi.propagator_pair(953, 0, (2, 1, 1, 1))
    a = oracle.point_correlator(op, Su, Sd)[0]
    su, sd = Su[0].reshape(-1, 12, 12), Sd[0].reshape(-1, 12, 12)
    b, m = 0, 0
    for x in range(2):
        c, mm = oracle.bruteforce(op, su[x:x + 1], sd[x:x + 1], with_magnitude=True)
        b += c
        m += mm
    assert abs(a - op.scale * b) <= 1e-12 * abs(op.scale) * m
