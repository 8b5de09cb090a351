"""Spin-color conventions of the oracle (test infrastructure only).

The paper fixes C = gamma_4 gamma_2 (Sec. 2, generic baryon interpolator) but
not the gamma basis. The oracle uses a Dirac-Pauli Euclidean basis with
gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = diag(-1, -1, 1, 1) and
gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4. In it C gamma_5 = diag(i sigma_2,
i sigma_2) and the parity projectors P_pm = (1 pm gamma_4)/2 (Sec. 3.3,
nucleon operators with projectors) are real integer matrices, so every
operator weight is an exact integer. The sign of gamma_4 is the reading under
which the operator term counts of the paper's method comparison table (356
for 2H, 1026 for each 3He spin, 2716 for 4He; Sec. 3.3) are reproduced.

Combined index (Sec. 2.1, after the block equations): chi = 3*spin + color.
"""
import itertools

import numpy as np

_s1 = np.array([[0, 1], [1, 0]], dtype=complex)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
_s3 = np.array([[1, 0], [0, -1]], dtype=complex)
_z2 = np.zeros((2, 2), dtype=complex)
_i2 = np.eye(2, dtype=complex)


def _blk(a, b, c, d):
    return np.block([[a, b], [c, d]])


def gammas():
    """Return (g1, g2, g3, g4, g5) as 4x4 complex arrays."""
    g = [_blk(_z2, -1j * s, 1j * s, _z2) for s in (_s1, _s2, _s3)]
    g4 = _blk(-_i2, _z2, _z2, _i2)
    g5 = g[0] @ g[1] @ g[2] @ g4
    return g[0], g[1], g[2], g4, g5


def _to_int(m):
    assert np.allclose(m.imag, 0) and np.allclose(m.real, np.round(m.real))
    return np.round(m.real).astype(np.int64)


def charge_conjugation():
    g1, g2, g3, g4, g5 = gammas()
    return g4 @ g2


def cg5():
    """C gamma_5 as an exact integer 4x4 matrix."""
    g5 = gammas()[4]
    return _to_int(charge_conjugation() @ g5)


def projector2(sign):
    """2 * P_pm = 1 pm gamma_4 (integer); P_pm itself has entries 0 and 1 here."""
    g4 = gammas()[3]
    return _to_int(np.eye(4) + sign * g4)


def proj(sign):
    """P_pm = (1 pm gamma_4)/2 as an integer matrix (exact in this basis)."""
    p2 = projector2(sign)
    assert np.all(p2 % 2 == 0)
    return p2 // 2


def levi_civita():
    e = np.zeros((3, 3, 3), dtype=np.int64)
    for p in itertools.permutations(range(3)):
        inv = sum(1 for i in range(3) for j in range(i + 1, 3) if p[i] > p[j])
        e[p] = -1 if inv % 2 else 1
    return e


def chi(spin, color):
    return 3 * spin + color


def spin_of(j):
    return j // 3


def color_of(j):
    return j % 3
