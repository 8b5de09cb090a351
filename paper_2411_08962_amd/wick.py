"""Thin Python binding of ``libwick.so`` (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; PyTorch
supplies device memory and the current stream. The entry points mirror the C
ABI in ``include/wick.h``: :func:`plan`, :func:`plan_std`, :func:`blocks`,
:func:`contract`, :func:`correlator`, :func:`autotune`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwick.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ECORRUPT, ETOOBIG = 0, -1, -2, -3, -4, -5, -6
C128, C64 = 0, 1
PRECISIONS = {"p64": 0, "p32": 1, "pb3": 2, "pb6": 3}
BLOCK_LEN = 792


class WickError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"wick status {status}: {msg}")
        self.status = status


class _Kind(ctypes.Structure):
    _fields_ = [("flavor", ctypes.c_int32 * 3), ("n_w", ctypes.c_int32),
                ("j", ctypes.POINTER(ctypes.c_int8)),
                ("w_re", ctypes.POINTER(ctypes.c_int64)), ("w_im", ctypes.POINTER(ctypes.c_int64))]


class _Desc(ctypes.Structure):
    _fields_ = [("A", ctypes.c_int32), ("n_kinds", ctypes.c_int32), ("kinds", ctypes.POINTER(_Kind)),
                ("n_snk", ctypes.c_int32), ("snk_kind", ctypes.POINTER(ctypes.c_int32)),
                ("snk_re", ctypes.POINTER(ctypes.c_int64)), ("snk_im", ctypes.POINTER(ctypes.c_int64)),
                ("n_src", ctypes.c_int32), ("src_kind", ctypes.POINTER(ctypes.c_int32)),
                ("src_re", ctypes.POINTER(ctypes.c_int64)), ("src_im", ctypes.POINTER(ctypes.c_int64)),
                ("scale", ctypes.c_double), ("hash_seed", ctypes.c_uint64),
                ("hash_trials", ctypes.c_int32), ("hash_sites", ctypes.c_int32)]


class _Item(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_int32), ("cfg", ctypes.c_int32)]


EXPORTS = ["wick_plan", "wick_plan_std", "wick_plan_info", "wick_plan_stats", "wick_plan_table",
           "wick_plan_kind", "wick_plan_save", "wick_plan_load", "wick_plan_truncate", "wick_plan_destroy", "wick_blocks",
           "wick_contract", "wick_correlator", "wick_autotune", "wick_shutdown", "wick_last_error",
           "wick_version", "wick_profile", "wick_profile_read", "wick_point_plan", "wick_point_plan_std",
           "wick_point_info", "wick_point_correlator", "wick_point_destroy", "wick_gevp_plan", "wick_gevp_info",
           "wick_gevp_table", "wick_gevp_kinds", "wick_gevp_contract", "wick_gevp_destroy", "wick_gevp_plan_std",
           "wick_plan_std_pair", "wick_point_blocks_correlator", "wick_contract_noalloc",
           "wick_autotune_batch", "wick_plan_sum_work"]

_lib = None


def lib():
    """Load the HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2411_08962_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.wick_plan.argtypes = [ctypes.POINTER(_Desc), pp]
    L.wick_plan_std.argtypes = [ctypes.c_char_p, i32, pp]
    L.wick_plan_std_pair.argtypes = [ctypes.c_char_p, i32, ctypes.c_char_p, i32, pp]
    L.wick_plan_info.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.wick_plan_stats.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(ctypes.c_double)]
    L.wick_plan_table.argtypes = [P, P, P]
    L.wick_plan_sum_work.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                     ctypes.POINTER(i64)]
    L.wick_plan_kind.argtypes = [P, i32, P, ctypes.POINTER(i32), P, P, P]
    L.wick_plan_save.argtypes = [P, ctypes.c_char_p]
    L.wick_plan_load.argtypes = [ctypes.c_char_p, pp]
    L.wick_plan_truncate.argtypes = [P, P, i32, ctypes.c_double, pp, P]
    L.wick_plan_destroy.argtypes = [P]
    L.wick_plan_destroy.restype = None
    L.wick_blocks.argtypes = [P, P, P, st, P, i32, st, P, P]
    L.wick_contract.argtypes = [P, P, i32, i32, P, P]
    L.wick_contract_noalloc.argtypes = [P, P, i32, i32, P, P]
    L.wick_correlator.argtypes = [P, i32, P, i32, P, P, st, P, i32, st, i32, P, P]
    L.wick_autotune.argtypes = [P, P, st, st, ctypes.c_char_p]
    L.wick_autotune_batch.argtypes = [P, i32, P, i32, P, P, st, P, i32, st, ctypes.c_char_p]
    L.wick_shutdown.argtypes = []
    L.wick_profile.argtypes = [i32]
    L.wick_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    L.wick_point_plan.argtypes = [ctypes.POINTER(_Desc), pp]
    L.wick_point_plan_std.argtypes = [ctypes.c_char_p, i32, pp]
    L.wick_point_info.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)] + [ctypes.POINTER(i64)] * 6
    L.wick_point_correlator.argtypes = [P, P, P, st, P, i32, P, P]
    L.wick_point_blocks_correlator.argtypes = [P, P, P, st, P, i32, P, P]
    L.wick_gevp_plan.argtypes = [ctypes.POINTER(_Desc), i32, pp]
    L.wick_gevp_plan_std.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i32), i32, pp]
    L.wick_gevp_info.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                 ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.wick_gevp_table.argtypes = [P, P, P]
    L.wick_gevp_kinds.argtypes = [P, pp]
    L.wick_gevp_contract.argtypes = [P, P, i32, i32, P, P]
    L.wick_gevp_destroy.argtypes = [P]
    L.wick_gevp_destroy.restype = None
    L.wick_point_destroy.argtypes = [P]
    L.wick_point_destroy.restype = None
    L.wick_last_error.restype = ctypes.c_char_p
    L.wick_version.restype = ctypes.c_char_p
    for name in ("wick_plan", "wick_plan_std", "wick_plan_info", "wick_plan_stats", "wick_plan_table", "wick_plan_sum_work",
                 "wick_plan_kind", "wick_plan_save", "wick_plan_load", "wick_plan_truncate", "wick_blocks",
                 "wick_contract",
                 "wick_correlator", "wick_autotune", "wick_shutdown", "wick_profile", "wick_profile_read",
                 "wick_point_plan", "wick_point_plan_std", "wick_point_info", "wick_point_correlator",
                 "wick_gevp_plan", "wick_gevp_info", "wick_gevp_table", "wick_gevp_kinds", "wick_gevp_contract",
                 "wick_gevp_plan_std", "wick_plan_std_pair", "wick_point_blocks_correlator"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != OK:
        raise WickError(status, lib().wick_last_error().decode())


class Plan:
    """A deduplicated Wick-term table (owned by the library)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.wick_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def info(self):
        A, K, N = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().wick_plan_info(self._h, ctypes.byref(A), ctypes.byref(K), ctypes.byref(N)))
        return A.value, K.value, N.value

    @property
    def A(self):
        return self.info()[0]

    @property
    def n_kinds(self):
        return self.info()[1]

    @property
    def n_terms(self):
        return self.info()[2]

    def stats(self):
        e, g, n, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().wick_plan_stats(self._h, ctypes.byref(e), ctypes.byref(g), ctypes.byref(n), ctypes.byref(b)))
        return {"n_enumerated": e.value, "n_groups": g.value, "n_terms": n.value, "false_merge_bound": b.value}

    SUM_FORMS = ("plain", "packed", "segmented-palette", "segmented", "factored")

    def sum_work(self):
        """Work of the term sum per time slice: {"form", "words2", "words1",
        "segments"} (see wick_plan_sum_work)."""
        f, w2, w1, sg = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().wick_plan_sum_work(self._h, ctypes.byref(f), ctypes.byref(w2), ctypes.byref(w1),
                                        ctypes.byref(sg)))
        return {"form": self.SUM_FORMS[f.value], "words2": w2.value, "words1": w1.value, "segments": sg.value}

    def table(self):
        """(kidx [A, N] uint16, coef [N] complex128)."""
        A, K, N = self.info()
        kidx = np.zeros((A, N), dtype=np.uint16)
        coef = np.zeros((N, 2), dtype=np.float64)
        _check(lib().wick_plan_table(self._h, kidx.ctypes.data_as(ctypes.c_void_p),
                                     coef.ctypes.data_as(ctypes.c_void_p)))
        return kidx, coef[:, 0] + 1j * coef[:, 1]

    def kind_flavors(self, k):
        f = (ctypes.c_int32 * 3)()
        nw = ctypes.c_int32()
        _check(lib().wick_plan_kind(self._h, k, f, ctypes.byref(nw), None, None, None))
        return tuple(f), nw.value

    def kind(self, k):
        """Block kind k: (flavors (3,), weights [(j1, j2, j3, w_re, w_im), ...])."""
        fl, nw = self.kind_flavors(k)
        j = np.zeros((max(nw, 1), 3), dtype=np.int8)
        re = np.zeros(max(nw, 1), dtype=np.int64)
        im = np.zeros(max(nw, 1), dtype=np.int64)
        _check(lib().wick_plan_kind(self._h, k, None, None, j.ctypes.data_as(ctypes.c_void_p),
                                    re.ctypes.data_as(ctypes.c_void_p), im.ctypes.data_as(ctypes.c_void_p)))
        return fl, [(int(j[e, 0]), int(j[e, 1]), int(j[e, 2]), int(re[e]), int(im[e])) for e in range(nw)]

    def save(self, path):
        _check(lib().wick_plan_save(self._h, str(path).encode()))

    def truncate(self, B_cal, keep_fraction):
        """Important-term truncation: a new plan with the terms that dominate on
        the calibration blocks B_cal ([..., n_kinds, 792, 2] float64 or
        [..., n_kinds, 792] complex128; numpy or torch, copied to the host),
        and the per-slice sum of |dropped terms| ([n_slices] float64)."""
        if hasattr(B_cal, "detach"):
            B_cal = B_cal.detach().cpu().numpy()
        B = np.asarray(B_cal)
        if np.iscomplexobj(B):
            B = np.stack([B.real, B.imag], axis=-1)
        B = np.ascontiguousarray(B, dtype=np.float64)
        K = self.n_kinds
        if B.ndim < 3 or B.shape[-3:] != (K, BLOCK_LEN, 2):
            raise ValueError(f"B_cal must end in ({K}, {BLOCK_LEN}, 2)")
        n_slices = int(np.prod(B.shape[:-3], dtype=np.int64))
        dropped = np.zeros(max(n_slices, 1), dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().wick_plan_truncate(self._h, B.ctypes.data_as(ctypes.c_void_p), n_slices, float(keep_fraction),
                                        ctypes.byref(h), dropped.ctypes.data_as(ctypes.c_void_p)))
        return Plan(h.value), dropped[:n_slices]

    @staticmethod
    def load(path):
        h = ctypes.c_void_p()
        _check(lib().wick_plan_load(str(path).encode(), ctypes.byref(h)))
        return Plan(h.value)


def plan_std(nucleus, J=0):
    """Built-in operator of Sec. 3.3: '1H', '2H', '3He', '3H', '4He'."""
    h = ctypes.c_void_p()
    _check(lib().wick_plan_std(nucleus.encode(), int(J), ctypes.byref(h)))
    return Plan(h.value)


def _desc(A, kinds, snk, src, scale=1.0, hash_seed=0, hash_trials=0, hash_sites=0):
    """The operator as a wick_nucleus_desc; returns (desc, arrays to keep alive)."""
    keep = []
    ks = (_Kind * len(kinds))()
    for i, (fl, w) in enumerate(kinds):
        j = np.array([[e[0], e[1], e[2]] for e in w], dtype=np.int8).reshape(-1)
        re = np.array([int(e[3]) for e in w], dtype=np.int64)
        im = np.array([int(e[4]) for e in w], dtype=np.int64)
        keep += [j, re, im]
        ks[i].flavor[:] = [int(f) for f in fl]
        ks[i].n_w = len(w)
        ks[i].j = j.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        ks[i].w_re = re.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        ks[i].w_im = im.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    keep.append(ks)

    def pats(ps):
        k = np.array([x for p in ps for x in p[0]], dtype=np.int32)
        re = np.array([int(p[1][0]) for p in ps], dtype=np.int64)
        im = np.array([int(p[1][1]) for p in ps], dtype=np.int64)
        keep.extend([k, re, im])
        return (len(ps), k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                re.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), im.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))

    d = _Desc()
    d.A, d.n_kinds, d.kinds = int(A), len(kinds), ks
    d.n_snk, d.snk_kind, d.snk_re, d.snk_im = pats(snk)
    d.n_src, d.src_kind, d.src_re, d.src_im = pats(src)
    d.scale, d.hash_seed, d.hash_trials, d.hash_sites = float(scale), int(hash_seed), int(hash_trials), int(hash_sites)
    return d, keep


def plan_std_pair(sink, source, J_sink=0, J_source=0):
    """The correlator with built-in operator `sink` at the sink and `source` at the source."""
    h = ctypes.c_void_p()
    _check(lib().wick_plan_std_pair(sink.encode(), int(J_sink), source.encode(), int(J_source), ctypes.byref(h)))
    return Plan(h.value)


def plan(A, kinds, snk, src, scale=1.0, hash_seed=0, hash_trials=0, hash_sites=0):
    """Plan a general operator.

    kinds: list of (flavors (3,), weights [(j1, j2, j3, w_re, w_im), ...]);
    snk, src: list of (tuple of A kind indices, (c_re, c_im)).
    """
    d, keep = _desc(A, kinds, snk, src, scale, hash_seed, hash_trials, hash_sites)
    h = ctypes.c_void_p()
    _check(lib().wick_plan(ctypes.byref(d), ctypes.byref(h)))
    return Plan(h.value)


class PointPlan:
    """A point-sink determinant plan (owned by the library)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.wick_point_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def info(self):
        nu, nd = ctypes.c_int32(), ctypes.c_int32()
        v = [ctypes.c_int64() for _ in range(6)]
        _check(lib().wick_point_info(self._h, ctypes.byref(nu), ctypes.byref(nd), *[ctypes.byref(x) for x in v]))
        keys = ("n_sink_groups", "n_src_groups", "n_rows_u", "n_cols_u", "n_rows_d", "n_cols_d")
        out = {"n_u": nu.value, "n_d": nd.value}
        out.update({k: x.value for k, x in zip(keys, v)})
        return out


class _BorrowedPlan(Plan):
    """A plan handle owned by another object (never destroyed here)."""

    def __init__(self, handle, owner):
        super().__init__(handle)
        self._owner = owner

    def __del__(self):
        pass


class GevpPlan:
    """An N x N correlation-matrix plan (owned by the library)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.wick_gevp_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def info(self):
        n, A, K = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        N, Ne = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().wick_gevp_info(self._h, *[ctypes.byref(x) for x in (n, A, K, N, Ne)]))
        return {"n_ops": n.value, "A": A.value, "n_kinds": K.value, "n_terms": N.value, "n_element_terms": Ne.value}

    def table(self):
        """(kidx [A, N] uint16, coef [N, n_ops, n_ops] complex128)."""
        i = self.info()
        A, N, n = i["A"], i["n_terms"], i["n_ops"]
        kidx = np.zeros((A, N), dtype=np.uint16)
        coef = np.zeros((N, n * n, 2), dtype=np.float64)
        _check(lib().wick_gevp_table(self._h, kidx.ctypes.data_as(ctypes.c_void_p), coef.ctypes.data_as(ctypes.c_void_p)))
        return kidx, (coef[..., 0] + 1j * coef[..., 1]).reshape(N, n, n)

    def blocks_plan(self):
        """The borrowed plan with the matrix's block kinds (for blocks(), autotune(), kind())."""
        h = ctypes.c_void_p()
        _check(lib().wick_gevp_kinds(self._h, ctypes.byref(h)))
        return _BorrowedPlan(h.value, self)


def gevp_plan(ops):
    """Correlation-matrix plan of operators given as dicts of plan() arguments."""
    descs = (_Desc * len(ops))()
    keep = []
    for i, o in enumerate(ops):
        d, k = _desc(**o)
        descs[i] = d
        keep.append(k)
    h = ctypes.c_void_p()
    _check(lib().wick_gevp_plan(descs, len(ops), ctypes.byref(h)))
    return GevpPlan(h.value)


def gevp_plan_std(names, J=None):
    """Correlation-matrix plan of built-in operators (e.g. ["2H", "2H-", "2H0"])."""
    n = len(names)
    arr = (ctypes.c_char_p * n)(*[x.encode() for x in names])
    js = (ctypes.c_int32 * n)(*([0] * n if J is None else [int(x) for x in J]))
    h = ctypes.c_void_p()
    _check(lib().wick_gevp_plan_std(arr, js, n, ctypes.byref(h)))
    return GevpPlan(h.value)


def gevp_contract(g: GevpPlan, B, out=None):
    """C [n_cfg, T, n_ops, n_ops, 2] float64 from blocks of g.blocks_plan()."""
    torch = _torch()
    i = g.info()
    n = i["n_ops"]
    if not B.is_cuda or not B.is_contiguous() or B.dtype != torch.float64 or B.dim() != 5:
        raise ValueError("B must be a contiguous float64 device tensor [n_cfg, T, K, 792, 2]")
    if B.shape[2:] != (i["n_kinds"], BLOCK_LEN, 2):
        raise ValueError("B does not match the matrix's block kinds")
    n_cfg, T = B.shape[:2]
    if out is None:
        out = torch.empty((n_cfg, T, n, n, 2), dtype=torch.float64, device=B.device)
    _check_out(out, (n_cfg, T, n, n, 2), B.device)
    _check(lib().wick_gevp_contract(g.handle, ctypes.c_void_p(B.data_ptr()), n_cfg, T, _stream(),
                                    ctypes.c_void_p(out.data_ptr())))
    return out


def point_plan(A, kinds, snk, src, scale=1.0):
    """Point-sink plan of a general operator (same arguments as plan())."""
    d, keep = _desc(A, kinds, snk, src, scale)
    h = ctypes.c_void_p()
    _check(lib().wick_point_plan(ctypes.byref(d), ctypes.byref(h)))
    return PointPlan(h.value)


def point_plan_std(nucleus, J=0):
    h = ctypes.c_void_p()
    _check(lib().wick_point_plan_std(nucleus.encode(), int(J), ctypes.byref(h)))
    return PointPlan(h.value)


# ----------------------------------------------------------------- GPU calls
def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prop_args(S_u, S_d):
    torch = _torch()
    for S in (S_u, S_d):
        if not S.is_cuda or not S.is_contiguous():
            raise ValueError("propagators must be contiguous device tensors")
        if S.dtype not in (torch.complex128, torch.complex64):
            raise ValueError("propagators must be complex128 or complex64")
        if S.dim() != 7 or S.shape[-2:] != (12, 12):
            raise ValueError("propagators must have shape [n_cfg, T, Z, Y, X, 12, 12]")
    if S_u.shape != S_d.shape or S_u.dtype != S_d.dtype or S_u.device != S_d.device:
        raise ValueError("S_u and S_d differ in shape or dtype")
    n_cfg, T, Z, Y, X = S_u.shape[:5]
    dims = (ctypes.c_int32 * 4)(X, Y, Z, T)
    dtype = C128 if S_u.dtype == torch.complex128 else C64
    return n_cfg, T, dims, dtype


def _check_out(out, shape, device):
    torch = _torch()
    if (not out.is_cuda or out.device != device or not out.is_contiguous() or out.dtype != torch.float64
            or tuple(out.shape) != tuple(shape)):
        raise ValueError(f"out must be a contiguous float64 tensor of shape {tuple(shape)} on {device}")


def blocks(p: Plan, S_u, S_d, precision="p64", out=None):
    """Blocks B [n_cfg, T, n_kinds, 792, 2] float64 on the device."""
    torch = _torch()
    n_cfg, T, dims, dtype = _prop_args(S_u, S_d)
    K = p.n_kinds
    if out is None:
        out = torch.empty((n_cfg, T, K, BLOCK_LEN, 2), dtype=torch.float64, device=S_u.device)
    _check_out(out, (n_cfg, T, K, BLOCK_LEN, 2), S_u.device)
    _check(lib().wick_blocks(p.handle, ctypes.c_void_p(S_u.data_ptr()), ctypes.c_void_p(S_d.data_ptr()), dtype,
                             dims, n_cfg, PRECISIONS[precision], _stream(), ctypes.c_void_p(out.data_ptr())))
    return out


def contract(p: Plan, B, out=None):
    """C [n_cfg, T, 2] float64 from blocks B [n_cfg, T, n_kinds, 792, 2]."""
    torch = _torch()
    if not B.is_cuda or not B.is_contiguous() or B.dtype != torch.float64 or B.dim() != 5:
        raise ValueError("B must be a contiguous float64 device tensor [n_cfg, T, K, 792, 2]")
    n_cfg, T = B.shape[:2]
    if B.shape[2:] != (p.n_kinds, BLOCK_LEN, 2):
        raise ValueError("B does not match the plan's kinds")
    if out is None:
        out = torch.empty((n_cfg, T, 2), dtype=torch.float64, device=B.device)
    _check_out(out, (n_cfg, T, 2), B.device)
    _check(lib().wick_contract(p.handle, ctypes.c_void_p(B.data_ptr()), n_cfg, T, _stream(),
                               ctypes.c_void_p(out.data_ptr())))
    return out


def contract_noalloc(p: Plan, B, out):
    """wick_contract_noalloc: as contract(), into a caller-provided out
    [n_cfg, T, 2] float64; the library allocates nothing (see wick.h)."""
    torch = _torch()
    if not B.is_cuda or not B.is_contiguous() or B.dtype != torch.float64 or B.dim() != 5:
        raise ValueError("B must be a contiguous float64 device tensor [n_cfg, T, K, 792, 2]")
    n_cfg, T = B.shape[:2]
    if B.shape[2:] != (p.n_kinds, BLOCK_LEN, 2):
        raise ValueError("B does not match the plan's kinds")
    _check_out(out, (n_cfg, T, 2), B.device)
    _check(lib().wick_contract_noalloc(p.handle, ctypes.c_void_p(B.data_ptr()), n_cfg, T, _stream(),
                                       ctypes.c_void_p(out.data_ptr())))
    return out


def correlator(plans, items, S_u, S_d, precision="p64", use_graph=False, out=None):
    """C [n_items, T, 2] for (plan index, configuration) items."""
    torch = _torch()
    n_cfg, T, dims, dtype = _prop_args(S_u, S_d)
    hp = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    it = (_Item * len(items))()
    for i, (pi, cfg) in enumerate(items):
        it[i].plan, it[i].cfg = int(pi), int(cfg)
    if out is None:
        out = torch.empty((len(items), T, 2), dtype=torch.float64, device=S_u.device)
    _check_out(out, (len(items), T, 2), S_u.device)
    _check(lib().wick_correlator(hp, len(plans), it, len(items), ctypes.c_void_p(S_u.data_ptr()),
                                 ctypes.c_void_p(S_d.data_ptr()), dtype, dims, n_cfg, PRECISIONS[precision],
                                 1 if use_graph else 0, _stream(), ctypes.c_void_p(out.data_ptr())))
    return out


def point_correlator(p: PointPlan, S_u, S_d, out=None):
    """Point-sink C [n_cfg, T, 2] float64 on the device (FP64 determinants)."""
    torch = _torch()
    n_cfg, T, dims, dtype = _prop_args(S_u, S_d)
    if out is None:
        out = torch.empty((n_cfg, T, 2), dtype=torch.float64, device=S_u.device)
    _check_out(out, (n_cfg, T, 2), S_u.device)
    _check(lib().wick_point_correlator(p.handle, ctypes.c_void_p(S_u.data_ptr()), ctypes.c_void_p(S_d.data_ptr()),
                                       dtype, dims, n_cfg, _stream(), ctypes.c_void_p(out.data_ptr())))
    return out


def point_blocks_correlator(p: Plan, S_u, S_d, out=None):
    """Point-sink C [n_cfg, T, 2] in the block form: per-site blocks and the plan's term table."""
    torch = _torch()
    n_cfg, T, dims, dtype = _prop_args(S_u, S_d)
    if out is None:
        out = torch.empty((n_cfg, T, 2), dtype=torch.float64, device=S_u.device)
    _check_out(out, (n_cfg, T, 2), S_u.device)
    _check(lib().wick_point_blocks_correlator(p.handle, ctypes.c_void_p(S_u.data_ptr()),
                                              ctypes.c_void_p(S_d.data_ptr()), dtype, dims, n_cfg, _stream(),
                                              ctypes.c_void_p(out.data_ptr())))
    return out


def autotune(p: Plan, dims, dtype="c128", precision="p64", cache_path=None):
    d = (ctypes.c_int32 * 4)(*dims)
    _check(lib().wick_autotune(p.handle, d, C128 if dtype == "c128" else C64, PRECISIONS[precision],
                               None if cache_path is None else str(cache_path).encode()))


def autotune_batch(plans, items, S_u, S_d, precision="p64", cache_path=None):
    """Tune the batched launch of correlator(plans, items, S_u, S_d, precision)
    as a whole (block sites and term-sum terms per workgroup)."""
    n_cfg, T, dims, dtype = _prop_args(S_u, S_d)
    hp = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    it = (_Item * len(items))()
    for i, (pi, cfg) in enumerate(items):
        it[i].plan, it[i].cfg = int(pi), int(cfg)
    _check(lib().wick_autotune_batch(hp, len(plans), it, len(items), ctypes.c_void_p(S_u.data_ptr()),
                                     ctypes.c_void_p(S_d.data_ptr()), dtype, dims, n_cfg, PRECISIONS[precision],
                                     None if cache_path is None else str(cache_path).encode()))


def profile(enable=True):
    """Start (clearing earlier records) or stop per-kernel HIP-event timing."""
    _check(lib().wick_profile(1 if enable else 0))


def profile_read(kernel):
    """(launches, total milliseconds) recorded for a kernel since profile(True)."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().wick_profile_read(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def version():
    return lib().wick_version().decode()
