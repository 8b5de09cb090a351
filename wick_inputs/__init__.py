"""Seeded synthetic quark propagators.

This module is the only code shared by the CPU oracle and the GPU path. It
draws random numbers and nothing else: it holds none of the contraction
arithmetic.

Layout of one flavor's propagator on one gauge configuration:
``S[t, z, y, x, j, i]`` with ``j`` the sink spin-color index and ``i`` the
source spin-color index, both ``chi = 3*spin + color`` in ``[0, 12)``.

Values: real and imaginary parts independent N(0, 1), times ``exp(-0.5 t)``
(the time dependence of the synthetic stand-in for a point-source
propagator). Every time slice of every (workload, configuration, flavor) has
its own Philox stream, keyed by ``SeedSequence([seed, t])`` with
``seed = 2*(1000*workload_id + cfg) + flavor`` (flavor 0 = u, 1 = d), so any
slice can be regenerated on its own. complex64 storage rounds the complex128
draw to nearest.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

U, D = 0, 1


def seed_of(workload_id: int, cfg: int, flavor: int) -> int:
    return 2 * (1000 * int(workload_id) + int(cfg)) + int(flavor)


def _slice(seed: int, t: int, vol: int, dtype) -> np.ndarray:
    g = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, t])))
    z = g.standard_normal(2 * vol * 144)
    out = np.empty(vol * 144, dtype=np.complex128)
    out.real = z[0::2]
    out.imag = z[1::2]
    out *= np.exp(-0.5 * t)
    out = out.reshape(vol, 12, 12)
    if dtype == np.complex64:
        out = out.astype(np.complex64)
    return out


def propagator(workload_id: int, cfg: int, flavor: int, dims, dtype=np.complex128,
               t_slices=None, threads: int | None = None) -> np.ndarray:
    """Return ``S[len(t_slices), Z, Y, X, 12, 12]`` for one flavor and configuration.

    ``dims`` is ``(X, Y, Z, T)``. ``t_slices`` defaults to ``range(T)``.
    """
    X, Y, Z, T = (int(v) for v in dims)
    vol = X * Y * Z
    ts = list(range(T)) if t_slices is None else [int(t) for t in t_slices]
    dtype = np.dtype(dtype).type
    out = np.empty((len(ts), Z, Y, X, 12, 12), dtype=dtype)
    seed = seed_of(workload_id, cfg, flavor)

    def fill(k):
        out[k] = _slice(seed, ts[k], vol, dtype).reshape(Z, Y, X, 12, 12)

    n = threads or min(16, os.cpu_count() or 1)
    if len(ts) > 1 and n > 1:
        with _cf.ThreadPoolExecutor(n) as ex:
            list(ex.map(fill, range(len(ts))))
    else:
        for k in range(len(ts)):
            fill(k)
    return out


def propagator_pair(workload_id: int, cfg: int, dims, dtype=np.complex128, t_slices=None):
    """(S_u, S_d) for one configuration."""
    return (propagator(workload_id, cfg, U, dims, dtype, t_slices),
            propagator(workload_id, cfg, D, dims, dtype, t_slices))
