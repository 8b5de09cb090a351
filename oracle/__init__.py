"""FP64 CPU oracle for nuclear two-point correlators -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It shares no code with the GPU library
(``paper_2411_08962_amd``) and never imports it.

Routes to C(t) for one time slice (all FP64, compensated accumulation):

* ``bruteforce``: Wick's theorem quark by quark (Sec. 3.1, the expansion that
  precedes Eq. 2.8), each nucleon summed over its own site (zero-momentum
  nucleon sinks, Eqs. 2.4-2.6, App. D). The definition itself; small lattices.
* ``sum_full``: blocks (Eq. 2.4 / App. D), then every source index tuple and
  every flavor-preserving bijection with its sign (Eq. 2.6 / App. D).
* ``sum_dp``: blocks, the source antisymmetrised first (method A, Sec. 3.3),
  then a dynamic programme over used source positions.
* ``point_correlator``: a point sink (every quark of the sink at one site,
  summed over sites, Eq. 2.9): the one-site lattice's blocks and the DP route
  per site. No determinants are involved.
* ``term_list`` / ``merged_terms``: the block-form terms themselves (one per
  canonical slot assignment, then merged by monomial), the objects that the
  important-term study of Sec. 5 and App. D ranks; ``important_terms`` is that
  selection written out.

The sign of a bijection is its sign as a permutation of quark positions, so
the flavor-grouping factor eta of Eq. 2.8 is part of every term; the overall
(-1)^n / Z is dropped, as in the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import conventions, operators  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C core with gcc (-O3, OpenMP; no -ffast-math, so
    every floating-point sum keeps its written order). Not -march=native: the
    library is built on one host and may run on another."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.oracle_block_raw.argtypes = [i64, P, P, P, i32, P, P, P, P]
        L.oracle_block_eq24.argtypes = [i64, P, P, P, i32, P, P, P, P]
        kinds = [i32, P, P, P, P, P, P]
        pats = [i32, P, P, i32, P, P]
        L.oracle_bruteforce.argtypes = [i32, i64, P, P] + kinds + pats + [i32, P]
        L.oracle_count_bijections.argtypes = [i32, P, P]
        L.oracle_count_bijections.restype = ctypes.c_long
        L.oracle_sum_full.argtypes = [i32, P] + kinds + pats + [P]
        L.oracle_sum_dp.argtypes = [i32, P] + kinds + pats + [P]
        L.oracle_source_group_count.argtypes = [i32] + kinds + [i32, P, P, i32]
        L.oracle_source_group_count.restype = ctypes.c_long
        L.oracle_threads.restype = ctypes.c_int32
        L.oracle_term_list.argtypes = [i32] + kinds + pats + [P, P]
        L.oracle_source_groups.argtypes = [i32] + kinds + [i32, P, P, i32, P, P]
        L.oracle_table_sum.argtypes = [i32, i64, P, P, i32, i64, P, P]
        L.oracle_source_groups.restype = ctypes.c_long
        L.oracle_term_list.restype = ctypes.c_long
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Packed:
    """The operator as flat arrays for the C routines (keeps them alive)."""

    def __init__(self, op):
        K = len(op.kinds)
        self.flav = np.array([f for k in op.kinds for f in k.flavors], dtype=np.int32)
        self.nw = np.array([len(k.w) for k in op.kinds], dtype=np.int32)
        self.woff = np.concatenate([[0], np.cumsum(self.nw)[:-1]]).astype(np.int32)
        ws = [e for k in op.kinds for e in k.w]
        self.wj = np.array([[e[0], e[1], e[2]] for e in ws], dtype=np.int32).reshape(-1)
        self.wre = np.array([e[3] for e in ws], dtype=np.float64)
        self.wim = np.array([e[4] for e in ws], dtype=np.float64)
        self.K = K
        self.snk_k = np.array([k for p in op.snk for k in p[0]], dtype=np.int32)
        self.snk_c = np.array([c for p in op.snk for c in p[1]], dtype=np.float64)
        self.src_k = np.array([k for p in op.src for k in p[0]], dtype=np.int32)
        self.src_c = np.array([c for p in op.src for c in p[1]], dtype=np.float64)
        self.n_snk, self.n_src = len(op.snk), len(op.src)

    def kinds_args(self):
        return [self.K, _p(self.flav), _p(self.nw), _p(self.woff), _p(self.wj), _p(self.wre), _p(self.wim)]

    def pat_args(self):
        return [self.n_snk, _p(self.snk_k), _p(self.snk_c), self.n_src, _p(self.src_k), _p(self.src_c)]


def _site_major(S):
    S = np.ascontiguousarray(S, dtype=np.complex128)
    return S.reshape(-1, 12, 12)


def block_raw(kind, Su_t, Sd_t):
    """B[i1, i2, i3] of one kind at one time slice (the block formula, raw)."""
    Su, Sd = _site_major(Su_t), _site_major(Sd_t)
    flav = np.array(kind.flavors, dtype=np.int32)
    wj = np.array([[e[0], e[1], e[2]] for e in kind.w], dtype=np.int32).reshape(-1)
    wre = np.array([e[3] for e in kind.w], dtype=np.float64)
    wim = np.array([e[4] for e in kind.w], dtype=np.float64)
    B = np.zeros(1728, dtype=np.complex128)
    lib().oracle_block_raw(Su.shape[0], _p(Su), _p(Sd), _p(flav), len(kind.w), _p(wj), _p(wre), _p(wim), _p(B))
    return B.reshape(12, 12, 12)


def block_eq24(kind, Su_t, Sd_t):
    """The block of Eq. 2.4: antisymmetrised in its two same-flavor source slots (1 and 3)."""
    assert kind.flavors[0] == kind.flavors[2]
    Su, Sd = _site_major(Su_t), _site_major(Sd_t)
    flav = np.array(kind.flavors, dtype=np.int32)
    wj = np.array([[e[0], e[1], e[2]] for e in kind.w], dtype=np.int32).reshape(-1)
    wre = np.array([e[3] for e in kind.w], dtype=np.float64)
    wim = np.array([e[4] for e in kind.w], dtype=np.float64)
    B = np.zeros(1728, dtype=np.complex128)
    lib().oracle_block_eq24(Su.shape[0], _p(Su), _p(Sd), _p(flav), len(kind.w), _p(wj), _p(wre), _p(wim), _p(B))
    return B.reshape(12, 12, 12)


def blocks_raw(op, Su_t, Sd_t):
    return np.stack([block_raw(k, Su_t, Sd_t) for k in op.kinds])


def bruteforce(op, Su_t, Sd_t, by_flavor=False, with_magnitude=False):
    """C at one time slice from the quark-level definition (unscaled).

    ``by_flavor`` sums the bijections flavor by flavor (the determinant form of
    Eqs. 2.8-2.9) instead of over all positions at once. ``with_magnitude``
    also returns the sum of the absolute values of the summed products, a
    scale for rounding-level comparisons.
    """
    pk = _Packed(op)
    Su, Sd = _site_major(Su_t), _site_major(Sd_t)
    out = np.zeros(3)
    lib().oracle_bruteforce(op.A, Su.shape[0], _p(Su), _p(Sd), *pk.kinds_args(), *pk.pat_args(),
                            1 if by_flavor else 0, _p(out))
    c = complex(out[0], out[1])
    return (c, float(out[2])) if with_magnitude else c


def sum_full(op, B):
    pk = _Packed(op)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    out = np.zeros(2)
    lib().oracle_sum_full(op.A, _p(B), *pk.kinds_args(), *pk.pat_args(), _p(out))
    return complex(out[0], out[1])


def sum_dp(op, B):
    pk = _Packed(op)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    out = np.zeros(2)
    lib().oracle_sum_dp(op.A, _p(B), *pk.kinds_args(), *pk.pat_args(), _p(out))
    return complex(out[0], out[1])


def threads():
    """OpenMP threads used by the oracle's parallel loops."""
    return int(lib().oracle_threads())


def count_bijections(f, g):
    """Number of flavor-preserving bijections between two flavor listings."""
    f = np.asarray(f, dtype=np.int32)
    g = np.asarray(g, dtype=np.int32)
    return int(lib().oracle_count_bijections(len(f), _p(f), _p(g)))


def source_group_count(op):
    pk = _Packed(op)
    nu = sum(1 for f in operators.flavor_listing(op, op.snk[0][0]) if f == 0)
    return int(lib().oracle_source_group_count(op.A, *pk.kinds_args(), pk.n_src, _p(pk.src_k), _p(pk.src_c), nu))


def correlator(op, Su, Sd, route="dp", t_slices=None):
    """Scaled C(t) for the time slices of ``Su, Sd`` ([T, Z, Y, X, 12, 12])."""
    T = Su.shape[0]
    ts = range(T) if t_slices is None else t_slices
    out = np.zeros(len(ts), dtype=np.complex128)
    for n, t in enumerate(ts):
        if route == "bruteforce":
            c = bruteforce(op, Su[t], Sd[t])
        else:
            B = blocks_raw(op, Su[t], Sd[t])
            c = sum_full(op, B) if route == "full" else sum_dp(op, B)
        out[n] = op.scale * c
    return out


# ------------------------------------------------------- block-form terms
def term_list(op):
    """Unmerged block-form terms: (ent [n, A] int32, coef [n] complex128, unscaled).

    ent[:, a] = kind * 1728 + i1 * 144 + i2 * 12 + i3 with i1 < i3: the entry of
    the Eq. 2.4 block (``block_eq24``) of nucleon a, in sink order.
    """
    pk = _Packed(op)
    n = int(lib().oracle_term_list(op.A, *pk.kinds_args(), *pk.pat_args(), None, None))
    ent = np.zeros((max(n, 1), op.A), dtype=np.int32)
    coef = np.zeros((max(n, 1), 2), dtype=np.float64)
    m = int(lib().oracle_term_list(op.A, *pk.kinds_args(), *pk.pat_args(), _p(ent), _p(coef)))
    assert m == n
    return ent[:n], coef[:n, 0] + 1j * coef[:n, 1]


def merged_terms(op):
    """Terms with equal monomials merged exactly: (keys [m, A] int32, each row
    ascending, rows in lexicographic order; coef [m] complex128, scale included).
    Coefficients are sums of integers (exact in FP64); zero sums are dropped."""
    ent, c = term_list(op)
    if len(c) == 0:
        return np.zeros((0, op.A), dtype=np.int32), np.zeros(0, dtype=np.complex128)
    keys = np.sort(ent, axis=1)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    acc = np.zeros(len(uniq), dtype=np.complex128)
    np.add.at(acc, inv.reshape(-1), c)
    nz = acc != 0
    return uniq[nz], op.scale * acc[nz]


def term_values(keys, coef, B_eq24):
    """v[s, n] = coef_n prod_a B_eq24[s].flat[keys[n, a]] for blocks [S, K, 12, 12, 12]."""
    flat = np.asarray(B_eq24, dtype=np.complex128).reshape(B_eq24.shape[0], -1)
    v = np.broadcast_to(np.asarray(coef, dtype=np.complex128), (flat.shape[0], len(coef))).copy()
    for a in range(keys.shape[1]):
        v = v * flat[:, keys[:, a].astype(np.int64)]
    return v


def keep_count(n_terms, keep):
    """Number of terms kept at fraction ``keep``: ceil(keep * N) up to 1e-6, at least 1."""
    if n_terms <= 0:
        return 0
    return int(min(n_terms, max(1.0, np.ceil(keep * float(n_terms) - 1e-6))))


def important_terms(keys, coef, B_eq24, keep):
    """Important-term selection (Sec. 5, App. D): terms ranked by |value| on
    calibration blocks, each slice's values normalised by its largest one.

    Returns (kept mask [n], score [n], dropped [S]) where score_n is the largest
    |v[s, n]| / max_m |v[s, m]| over slices with a nonzero maximum, the kept
    terms are the keep_count(n, keep) largest scores (equal scores: lower index
    first) and dropped[s] is the sum of |v[s, n]| over the terms not kept.
    """
    mag = np.abs(term_values(keys, coef, B_eq24))
    n = mag.shape[1]
    score = np.zeros(n)
    for s in range(mag.shape[0]):
        m = mag[s].max() if n else 0.0
        if m > 0:
            score = np.maximum(score, mag[s] / m)
    M = keep_count(n, keep)
    order = np.lexsort((np.arange(n), -score))
    kept = np.zeros(n, dtype=bool)
    kept[order[:M]] = True
    dropped = mag[:, ~kept].sum(axis=1)
    return kept, score, dropped


# ------------------------------------------------------------- point sinks
def source_groups(op):
    """Antisymmetrised source groups: (vals [G, 3A] canonical index lists, u's
    ascending then d's ascending; W' [G] complex128, unscaled)."""
    pk = _Packed(op)
    nu = sum(1 for f in operators.flavor_listing(op, op.src[0][0]) if f == 0)
    args = [op.A, *pk.kinds_args(), pk.n_src, _p(pk.src_k), _p(pk.src_c), nu]
    n = int(lib().oracle_source_groups(*args, None, None))
    vals = np.zeros((max(n, 1), 3 * op.A), dtype=np.int32)
    w = np.zeros((max(n, 1), 2))
    lib().oracle_source_groups(*args, _p(vals), _p(w))
    return vals[:n], w[:n, 0] + 1j * w[:n, 1]


def point_correlator(op, Su, Sd, t_slices=None):
    """Scaled point-sink C(t) for propagators [T, Z, Y, X, 12, 12]: the sink's
    quarks all at one site x, summed over x (Eq. 2.9). Per site, the blocks of
    that one-site lattice and the DP route of the block form; no determinants."""
    T = Su.shape[0]
    ts = range(T) if t_slices is None else t_slices
    out = np.zeros(len(ts), dtype=np.complex128)
    for n, t in enumerate(ts):
        su = _site_major(Su[t])
        sd = _site_major(Sd[t])
        c = 0j
        for x in range(su.shape[0]):
            c += sum_dp(op, blocks_raw(op, su[x:x + 1], sd[x:x + 1]))
        out[n] = op.scale * c
    return out


def point_det_magnitude(op, Su, Sd, t_slices=None):
    """Per time slice, sum over sites of sum_{g,h} |W_g W'_h det S_u[U_g; U'_h]
    det S_d[D_g; D'_h]|: the absolute terms of the determinant form of Eq. 2.9
    (numpy determinants), the error scale of a point-sink C(t). Unscaled by
    op.scale's sign, scaled by its magnitude."""
    from .operators import Operator
    sink = Operator(op.A, op.kinds, op.snk, op.snk, op.scale, op.name)
    vs, ws = source_groups(sink)
    vh, wh = source_groups(op)
    nu = sum(1 for f in operators.flavor_listing(op, op.snk[0][0]) if f == 0)

    def split(v):
        U, iu = np.unique(v[:, :nu], axis=0, return_inverse=True)
        D, idd = np.unique(v[:, nu:], axis=0, return_inverse=True)
        return U, iu.reshape(-1), D, idd.reshape(-1)

    Us, ius, Ds, ids = split(vs)
    Uh, iuh, Dh, idh = split(vh)

    def dets(M, R, K):
        sub = M[R[:, None, :, None], K[None, :, None, :]]
        return np.abs(np.linalg.det(sub)) if R.shape[1] else np.ones((len(R), len(K)))

    T = Su.shape[0]
    ts = range(T) if t_slices is None else t_slices
    out = np.zeros(len(ts))
    aws, awh = np.abs(ws), np.abs(wh)
    for n, t in enumerate(ts):
        su = _site_major(Su[t])
        sd = _site_major(Sd[t])
        for x in range(su.shape[0]):
            du = dets(su[x], Us, Uh)
            dd = dets(sd[x], Ds, Dh)
            A = du[ius][:, iuh] * dd[ids][:, idh]
            out[n] += aws @ A @ awh
    return abs(op.scale) * out


def table_sum(kidx, coef, B_sets):
    """sum_n coef_n prod_a B[s].flat[kidx[a, n]] for every block set s, on all
    threads: a given flat term table (Eq. 2.6 written as a list of products of
    block entries) evaluated on the CPU. With |coef| and |B| it gives
    sum_n |term_n|, the error scale of a correlator; on the oracle's own merged
    term list (``merged_terms``) it reproduces ``sum_dp``."""
    kidx = np.ascontiguousarray(kidx, dtype=np.uint16)
    coef = np.ascontiguousarray(coef, dtype=np.complex128)
    B = np.ascontiguousarray(B_sets, dtype=np.complex128).reshape(len(B_sets), -1)
    out = np.zeros((B.shape[0], 2))
    lib().oracle_table_sum(kidx.shape[0], kidx.shape[1], _p(kidx), _p(coef), B.shape[0], B.shape[1], _p(B), _p(out))
    return out[:, 0] + 1j * out[:, 1]
