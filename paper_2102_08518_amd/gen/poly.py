"""Exact multivariate polynomials over the rationals (dict: exponent tuple -> Fraction)."""
from __future__ import annotations

from fractions import Fraction
from math import comb
from typing import Dict, Iterable, Tuple

Exp = Tuple[int, ...]


class Poly:
    __slots__ = ("n", "t")

    def __init__(self, n: int, terms: Dict[Exp, Fraction] | None = None):
        self.n = n
        self.t: Dict[Exp, Fraction] = {}
        if terms:
            for e, c in terms.items():
                if c != 0:
                    self.t[e] = Fraction(c)

    # -- constructors
    @staticmethod
    def const(n: int, c) -> "Poly":
        return Poly(n, {(0,) * n: Fraction(c)})

    @staticmethod
    def affine(n: int, lin: Iterable, c0=0) -> "Poly":
        terms = {(0,) * n: Fraction(c0)}
        for i, a in enumerate(lin):
            e = [0] * n
            e[i] = 1
            terms[tuple(e)] = Fraction(a)
        return Poly(n, terms)

    # -- arithmetic
    def copy(self) -> "Poly":
        p = Poly(self.n)
        p.t = dict(self.t)
        return p

    def iadd(self, other: "Poly", scale=1) -> "Poly":
        scale = Fraction(scale)
        if scale == 0:
            return self
        for e, c in other.t.items():
            v = self.t.get(e, Fraction(0)) + scale * c
            if v == 0:
                self.t.pop(e, None)
            else:
                self.t[e] = v
        return self

    def __add__(self, other: "Poly") -> "Poly":
        return self.copy().iadd(other)

    def __sub__(self, other: "Poly") -> "Poly":
        return self.copy().iadd(other, -1)

    def scale(self, s) -> "Poly":
        s = Fraction(s)
        if s == 0:
            return Poly(self.n)
        return Poly(self.n, {e: c * s for e, c in self.t.items()})

    def __mul__(self, other: "Poly") -> "Poly":
        out: Dict[Exp, Fraction] = {}
        for e1, c1 in self.t.items():
            for e2, c2 in other.t.items():
                e = tuple(a + b for a, b in zip(e1, e2))
                out[e] = out.get(e, Fraction(0)) + c1 * c2
        return Poly(self.n, out)

    def is_zero(self) -> bool:
        return not self.t

    def degree(self) -> int:
        return max((sum(e) for e in self.t), default=-1)

    def __call__(self, pt) -> Fraction:
        acc = Fraction(0)
        for e, c in self.t.items():
            term = c
            for x, k in zip(pt, e):
                if k:
                    term *= Fraction(x) ** k
            acc += term
        return acc

    def eval_float(self, pts):
        """Evaluate at an (N, n) float array in float64 (testing convenience)."""
        import numpy as np
        pts = np.asarray(pts, dtype=np.float64)
        out = np.zeros(pts.shape[0])
        for e, c in self.t.items():
            term = np.full(pts.shape[0], float(c))
            for i, k in enumerate(e):
                if k:
                    term *= pts[:, i] ** k
            out += term
        return out

    def deriv(self, i: int) -> "Poly":
        out: Dict[Exp, Fraction] = {}
        for e, c in self.t.items():
            if e[i]:
                e2 = list(e)
                e2[i] -= 1
                out[tuple(e2)] = c * e[i]
        return Poly(self.n, out)

    def translate(self, shift) -> "Poly":
        """Return q with q(u) = p(u + shift)."""
        shift = [Fraction(s) for s in shift]
        out: Dict[Exp, Fraction] = {}
        for e, c in self.t.items():
            # expand prod_i (u_i + s_i)^{e_i}
            partial = {(): c}
            for i, k in enumerate(e):
                nxt = {}
                for pe, pc in partial.items():
                    for j in range(k + 1):
                        coef = pc * comb(k, j) * (shift[i] ** (k - j))
                        if coef == 0:
                            continue
                        ne = pe + (j,)
                        nxt[ne] = nxt.get(ne, Fraction(0)) + coef
                partial = nxt
            for pe, pc in partial.items():
                out[pe] = out.get(pe, Fraction(0)) + pc
        return Poly(self.n, out)

    def __eq__(self, other) -> bool:  # exact equality
        return isinstance(other, Poly) and self.t == other.t

    def __repr__(self) -> str:
        if not self.t:
            return "0"
        parts = []
        for e in sorted(self.t, key=lambda e: (-sum(e), e)):
            mono = "*".join("y%d^%d" % (i, k) if k > 1 else "y%d" % i
                            for i, k in enumerate(e) if k)
            parts.append("%s%s" % (self.t[e], ("*" + mono) if mono else ""))
        return " + ".join(parts)


def monomials(n: int, degree: int):
    """All exponent tuples of total degree <= degree, graded lexicographic."""
    out = []

    def rec(prefix, left, k):
        if k == n:
            out.append(tuple(prefix))
            return
        for a in range(left, -1, -1):
            rec(prefix + [a], left - a, k + 1)

    for d in range(degree + 1):
        rec([], d, 0)
        # keep only exact degree d of this pass
    return sorted({e for e in out if sum(e) <= degree}, key=lambda e: (sum(e), tuple(-x for x in e)))
