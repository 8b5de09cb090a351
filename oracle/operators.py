"""Interpolating operators of the oracle, as exact integer weights (test infrastructure only).

A nucleon "kind" is one zero-momentum nucleon operator with a fixed sink spin
alpha. The proton of Eq. (2.2)-(2.3) (the p, n operators of Sec. 2.1) is
p_alpha = eps_abc u^a_alpha u^b_beta (C g5 Q)_{beta eta} d^c_eta, with
Q = 1, P_+ or P_- (the projected forms p_pm, n_pm of Sec. 3.3). Its three
quark slots are listed here in the order (u^a_alpha, d^c_eta, u^b_beta), so a
kind has flavors (u, d, u) and weight

    w(j1, j2, j3) = delta(spin j1 = alpha) eps[c(j1), c(j3), c(j2)] M[s(j3), s(j2)],
    M = C g5 Q.

Moving d^c in front of u^b flips the sign of every nucleon; sink and source use
the same listing, so the correlator is unchanged. The neutron swaps u and d.

A nuclear operator is a sum of patterns: a product of A kinds (in nucleon
order) times an exact Gaussian-integer coefficient. The source operator uses
the same real tensors as the sink (the paper writes the same eps and C g5 at
the source, Eq. 2.6). A real FP64 ``scale`` carries irrational normalisations.
"""
from dataclasses import dataclass, field

import numpy as np

from . import conventions as cv

U, D = 0, 1
FLAVORS = {"p": (U, D, U), "n": (D, U, D)}


@dataclass
class Kind:
    flavors: tuple
    w: list  # (j1, j2, j3, w_re, w_im)
    label: str = ""


@dataclass
class Operator:
    A: int
    kinds: list
    snk: list  # (tuple of kind indices, (c_re, c_im))
    src: list
    scale: float = 1.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_u(self):
        k = self.kinds[self.snk[0][0][0]]
        return sum(sum(1 for f in self.kinds[i].flavors if f == U) for i in self.snk[0][0])

    @property
    def n_d(self):
        return 3 * self.A - self.n_u


def diquark_matrix(proj):
    m = cv.cg5()
    if proj == 0:
        return m
    return m @ cv.proj(proj)


def nucleon_kind(ntype, proj, alpha):
    """Weights of p_alpha / n_alpha with diquark matrix C g5 (proj=0) or C g5 P_pm."""
    M = diquark_matrix(proj)
    eps = cv.levi_civita()
    w = []
    for j1 in range(12):
        if cv.spin_of(j1) != alpha:
            continue
        for j2 in range(12):
            for j3 in range(12):
                v = eps[cv.color_of(j1), cv.color_of(j3), cv.color_of(j2)] * \
                    M[cv.spin_of(j3), cv.spin_of(j2)]
                if v:
                    w.append((j1, j2, j3, int(v), 0))
    lab = f"{ntype}{'' if proj == 0 else ('+' if proj > 0 else '-')}{alpha}"
    return Kind(FLAVORS[ntype], w, lab)


class _KindTable:
    def __init__(self):
        self.kinds, self.index = [], {}

    def get(self, ntype, proj, alpha):
        key = (ntype, proj, alpha)
        if key not in self.index:
            self.index[key] = len(self.kinds)
            self.kinds.append(nucleon_kind(ntype, proj, alpha))
        return self.index[key]


def proton(alpha=0, proj=0):
    """A = 1: a single proton of sink spin alpha (the single-nucleon case, App. B)."""
    kt = _KindTable()
    k = kt.get("p", proj, alpha)
    pats = [((k,), (1, 0))]
    return Operator(1, kt.kinds, pats, list(pats), 1.0, f"p{alpha}")


def proton_pair(alpha_snk, alpha_src, proj=0):
    """A = 1 with different sink and source spins: the (alpha, alpha') entry of C_p."""
    kt = _KindTable()
    a = kt.get("p", proj, alpha_snk)
    b = kt.get("p", proj, alpha_src)
    return Operator(1, kt.kinds, [((a,), (1, 0))], [((b,), (1, 0))], 1.0,
                    f"p{alpha_snk}{alpha_src}")


def deuteron(proj=+1):
    """O_2H = n^T (C g5 P_+) p with unprojected p, n (Sec. 3.3, deuteron operator).

    proj = -1 puts P_- in place of P_+ and proj = 0 drops the projector: the
    same block kinds with other couplings, a basis for a correlation matrix.
    """
    kt = _KindTable()
    M = cv.cg5() @ cv.proj(proj) if proj else cv.cg5()
    pats = []
    for beta in range(4):
        for alpha in range(4):
            c = int(M[beta, alpha])
            if c:
                pats.append(((kt.get("n", 0, beta), kt.get("p", 0, alpha)), (c, 0)))
    return Operator(2, kt.kinds, pats, list(pats), 1.0, "2H" if proj == 1 else f"2H({proj:+d})")


def _three_body(first, mid, last, J):
    """(first_-)_a (C g5)_{ab} (mid_+)_b (last_+)_J: the 3He form (Sec. 3.3) and its mirror."""
    kt = _KindTable()
    M = cv.cg5()
    pats = []
    for a in range(4):
        for b in range(4):
            c = int(M[a, b])
            if c:
                pats.append(((kt.get(first, -1, a), kt.get(mid, +1, b), kt.get(last, +1, J)), (c, 0)))
    return kt, pats


def helium3(J=0):
    """O^J_3He = p_-^T (C g5) n_+ p_+^J (Sec. 3.3); J = 0 is spin up."""
    kt, pats = _three_body("p", "n", "p", J)
    return Operator(3, kt.kinds, pats, list(pats), 1.0, "3He")


def triton(J=0):
    """The 3H cluster of the 7Li operator: n_-^T (C g5) p_+ n_+^J (Sec. 3.3)."""
    kt, pats = _three_body("n", "p", "n", J)
    return Operator(3, kt.kinds, pats, list(pats), 1.0, "3H")


# Spin / isospin wave functions of the 4He operator (Sec. 3.3), times 2 and sqrt(12).
_CHI = {"udud": 1, "dudu": 1, "uddu": -1, "duud": -1}
_CHIBAR = {"udud": 1, "dudu": 1, "uddu": 1, "duud": 1, "uudd": -2, "dduu": -2}


def helium4():
    """O_4He = (chibar eta - chi etabar)/sqrt(2) (Sec. 3.3), up = spin 0, down = spin 1.

    The nucleons are the unprojected p, n of Eqs. 2.2-2.3 (diquark C g5): the
    paper names no projector for 4He, and with unprojected nucleons the
    operator has exactly the 2716 terms the paper quotes for it.

    Both wave functions carry 1/2 and 1/sqrt(12), so the integer pattern
    coefficients are chibar'(s) eta'(i) - chi'(s) etabar'(i) and the correlator
    scale is (1/sqrt(2) * 1/(2 sqrt(12)))^2 = 1/96.
    """
    kt = _KindTable()
    coef = {}
    for s, cs_bar in _CHIBAR.items():
        for i, ci in _CHI.items():
            coef[(s, i)] = coef.get((s, i), 0) + cs_bar * ci
    for s, cs in _CHI.items():
        for i, ci_bar in _CHIBAR.items():
            coef[(s, i)] = coef.get((s, i), 0) - cs * ci_bar
    pats = []
    for (s, i), c in sorted(coef.items()):
        if c == 0:
            continue
        ks = tuple(kt.get("p" if i[a] == "u" else "n", 0, 0 if s[a] == "u" else 1) for a in range(4))
        pats.append((ks, (int(c), 0)))
    return Operator(4, kt.kinds, pats, list(pats), 1.0 / 96.0, "4He")


def gevp_element(op_list, i, j):
    """The (i, j) element of a correlation matrix (Eqs. E1-E3) as one Operator:
    operator i at the sink, operator j at the source. The kinds are the union
    of the operators' kinds (equal flavors and weights are one kind) and the
    scale is sqrt(scale_i scale_j) (the paper gives no normalisation; each
    scale is the square of an operator normalisation)."""
    kinds, index, maps = [], {}, []
    for op in op_list:
        m = []
        for k in op.kinds:
            key = (tuple(k.flavors), tuple(sorted((a, b, c, x, y) for a, b, c, x, y in k.w if x or y)))
            if key not in index:
                index[key] = len(kinds)
                kinds.append(k)
            m.append(index[key])
        maps.append(m)
    snk = [(tuple(maps[i][k] for k in p), c) for p, c in op_list[i].snk]
    src = [(tuple(maps[j][k] for k in p), c) for p, c in op_list[j].src]
    scale = float(np.sqrt(op_list[i].scale * op_list[j].scale))
    return Operator(op_list[i].A, kinds, snk, src, scale, f"{op_list[i].name}|{op_list[j].name}")


def by_name(name):
    return {"2H": deuteron, "3He": helium3, "3H": triton, "4He": helium4}[name]()


def flavor_listing(op, pattern_kinds):
    out = []
    for k in pattern_kinds:
        out.extend(op.kinds[k].flavors)
    return out


def sparsify(op, keep, rng, keep_patterns=None):
    """A random sub-operator: every kind keeps `keep` weight entries, optionally fewer patterns.

    Any coefficient tensor is a legal operator (Sec. 3.1, the generic local
    operator), so a sparsified operator tests the same algebra with fewer terms.
    """
    kinds = []
    for k in op.kinds:
        idx = rng.choice(len(k.w), size=min(keep, len(k.w)), replace=False)
        kinds.append(Kind(k.flavors, [k.w[i] for i in sorted(idx)], k.label))
    snk = list(op.snk)
    if keep_patterns is not None and keep_patterns < len(snk):
        sel = sorted(rng.choice(len(snk), size=keep_patterns, replace=False))
        snk = [snk[i] for i in sel]
    return Operator(op.A, kinds, snk, list(snk), op.scale, op.name + "-sparse")
