"""Derivation of the reference sub-region polynomials of a box spline.

This is the analysis the paper takes from its prequel (Sec. 3): a region of
evaluation (ROE) that tiles space under lattice shifts, its dissection into
sub-regions on which the convolution sum is a single polynomial, and the
symmetries that map every sub-region onto a few reference sub-regions.  For
the splines built here the ROE, the symmetry and the reference sub-regions are
stated per spline in ``specs.py``; this module derives, in exact rational
arithmetic, for each reference sub-region

  * its stencil: the lattice offsets o_j whose translate phi(y - o_j) is not
    identically zero on the sub-region (the sites c_0..c_{n-1} of Fig. 1);
  * the polynomial w_j(y) = phi(y - o_j) on the sub-region, so that the sum is
    f = sum_j c_j w_j(y) there;

and it checks that no knot plane of any stencil translate crosses the
sub-region (so each w_j really is one polynomial there) and that the weights
sum to exactly one.

The pieces are obtained from a polynomial-valued form of the box-spline
recurrence with the recurrence parameter t supported on a basis of the
current direction set (t_xi = 0 off the basis), worked symbolically around an
interior point of the sub-region.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from math import gcd
from typing import Dict, List, Sequence, Tuple

from .poly import Poly

F = Fraction


def _det(m: Sequence[Sequence[F]]) -> F:
    n = len(m)
    if n == 1:
        return F(m[0][0])
    if n == 2:
        return F(m[0][0]) * m[1][1] - F(m[0][1]) * m[1][0]
    return (F(m[0][0]) * (F(m[1][1]) * m[2][2] - F(m[1][2]) * m[2][1])
            - F(m[0][1]) * (F(m[1][0]) * m[2][2] - F(m[1][2]) * m[2][0])
            + F(m[0][2]) * (F(m[1][0]) * m[2][1] - F(m[1][1]) * m[2][0]))


def _inv(m: Sequence[Sequence[F]]) -> List[List[F]]:
    n = len(m)
    d = _det(m)
    if d == 0:
        raise ZeroDivisionError("singular")
    out = [[F(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            minor = [[m[r][c] for c in range(n) if c != j] for r in range(n) if r != i]
            cof = (-1) ** (i + j) * (_det(minor) if minor else F(1))
            out[j][i] = cof / d
    return out


def _rank(vecs: Sequence[Sequence[int]], s: int) -> int:
    rows = [[F(x) for x in v] for v in vecs]
    r = 0
    for col in range(s):
        piv = next((i for i in range(r, len(rows)) if rows[i][col] != 0), None)
        if piv is None:
            continue
        rows[r], rows[piv] = rows[piv], rows[r]
        for i in range(len(rows)):
            if i != r and rows[i][col] != 0:
                f = rows[i][col] / rows[r][col]
                rows[i] = [a - f * b for a, b in zip(rows[i], rows[r])]
        r += 1
    return r


class BoxSpline:
    """M_Xi for a direction multiset; phi(y) = |det L| M_Xi(y + centre)."""

    def __init__(self, s: int, directions: Sequence[Sequence[int]], det_L: int):
        self.s = s
        dist: List[Tuple[int, ...]] = []
        mult: List[int] = []
        for d in directions:
            d = tuple(int(x) for x in d)
            sg = next(((x > 0) - (x < 0) for x in d if x), 0)
            if sg == 0:
                raise ValueError("zero direction")
            d = tuple(sg * x for x in d)
            if d in dist:
                mult[dist.index(d)] += 1
            else:
                dist.append(d)
                mult.append(1)
        self.dirs = dist
        self.mult0 = tuple(mult)
        self.det_L = F(abs(det_L))
        self.centre = tuple(F(sum(m * d[i] for d, m in zip(dist, mult)), 2) for i in range(s))
        self.halfwidth = tuple(F(sum(m * abs(d[i]) for d, m in zip(dist, mult)), 2)
                               for i in range(s))
        self.degree = sum(mult) - s

    # -- geometry of the knot planes
    def plane_families(self):
        """(primitive normal, spacing g) for every hyperplane spanned by s-1
        directions; knots of the uncentred M lie on normal . z in g Z."""
        fams = {}
        if self.s == 1:
            g = 0
            for d in self.dirs:
                g = gcd(g, abs(d[0]))
            return [((1,), g)]
        for combo in itertools.combinations(self.dirs, self.s - 1):
            if self.s == 3:
                a, b = combo
                n = (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])
            else:
                (a,) = combo
                n = (-a[1], a[0])
            if all(x == 0 for x in n):
                continue
            g = 0
            for x in n:
                g = gcd(g, abs(x))
            n = tuple(x // g for x in n)
            sg = next(((x > 0) - (x < 0) for x in n if x), 1)
            n = tuple(sg * x for x in n)
            sp = 0
            for d in self.dirs:
                sp = gcd(sp, abs(sum(x * y for x, y in zip(n, d))))
            fams[n] = sp
        return sorted(fams.items())

    # -- the polynomial piece
    def _spans(self, mult) -> bool:
        return _rank([d for d, m in zip(self.dirs, mult) if m], self.s) == self.s

    def piece(self, offset: Sequence[F], y0: Sequence[F], ybox) -> Poly:
        """Polynomial P(y) = M_Xi(y + offset) valid on the cell of the knot-plane
        arrangement that contains y0.  ybox: per-axis (lo, hi) bounds of the
        region, used to drop translates whose support box misses it."""
        s = self.s
        memo: Dict[Tuple, Poly] = {}
        offset = tuple(F(x) for x in offset)

        def rec(mult: Tuple[int, ...], shift: Tuple[int, ...]) -> Poly:
            key = (mult, shift)
            if key in memo:
                return memo[key]
            # w(y) = y + offset - shift; support of M_{Xi(mult)} lies in the
            # box sum_d mult_d [min(0,d), max(0,d)]
            for i in range(s):
                lo = sum(m * min(0, d[i]) for d, m in zip(self.dirs, mult))
                hi = sum(m * max(0, d[i]) for d, m in zip(self.dirs, mult))
                wlo = ybox[i][0] + offset[i] - shift[i]
                whi = ybox[i][1] + offset[i] - shift[i]
                if whi <= lo or wlo >= hi:
                    memo[key] = Poly(s)
                    return memo[key]
            n = sum(mult)
            if n == s:
                B = [[F(d[i]) for d, m in zip(self.dirs, mult) if m] for i in range(s)]
                Binv = _inv(B)
                w0 = [F(y0[i]) + offset[i] - shift[i] for i in range(s)]
                u = [sum(Binv[r][c] * w0[c] for c in range(s)) for r in range(s)]
                if any(x == 0 or x == 1 for x in u):
                    raise ValueError("interior point lies on a knot plane")
                inside = all(0 < x < 1 for x in u)
                p = Poly.const(s, 1 / abs(_det(B))) if inside else Poly(s)
                memo[key] = p
                return p
            # basis-supported recurrence parameter: the first s independent
            # directions (in a fixed order) carry t = B^{-1} w, the rest t = 0
            basis: List[int] = []
            for k, (d, m) in enumerate(zip(self.dirs, mult)):
                if m and _rank([self.dirs[b] for b in basis] + [d], s) == len(basis) + 1:
                    basis.append(k)
                if len(basis) == s:
                    break
            B = [[F(self.dirs[b][i]) for b in basis] for i in range(s)]
            Binv = _inv(B)
            tpoly = {}
            for r, b in enumerate(basis):
                lin = [Binv[r][c] for c in range(s)]
                c0 = sum(Binv[r][c] * (offset[c] - shift[c]) for c in range(s))
                tpoly[b] = Poly.affine(s, lin, c0)
            acc = Poly(s)
            one = Poly.const(s, 1)
            for k, (d, m) in enumerate(zip(self.dirs, mult)):
                if not m:
                    continue
                sub = list(mult)
                sub[k] -= 1
                sub = tuple(sub)
                if not self._spans(sub):
                    continue
                sh2 = tuple(shift[i] + d[i] for i in range(s))
                here = rec(sub, shift)
                there = rec(sub, sh2)
                if k in tpoly:
                    t = tpoly[k]
                    acc.iadd(t * here)
                    acc.iadd((one - t) * there)
                    acc.iadd(there, m - 1)
                else:
                    acc.iadd(there, m)
            p = acc.scale(F(1, n - s))
            memo[key] = p
            return p

        return rec(self.mult0, (0,) * s)

    def phi_piece(self, o: Sequence[int], y0, ybox) -> Poly:
        """phi(y - o) = |det L| M(y - o + centre) on the cell containing y0."""
        off = [self.centre[i] - o[i] for i in range(self.s)]
        return self.piece(off, y0, ybox).scale(self.det_L)


# ---------------------------------------------------------------- regions

def polytope_vertices(halfspaces, s: int):
    """Vertices of {y : a . y + b >= 0 for (a, b) in halfspaces}, exactly."""
    verts = set()
    for combo in itertools.combinations(halfspaces, s):
        A = [[F(x) for x in a] for a, _ in combo]
        if _det(A) == 0:
            continue
        Ainv = _inv(A)
        rhs = [-F(b) for _, b in combo]
        y = tuple(sum(Ainv[i][j] * rhs[j] for j in range(s)) for i in range(s))
        if all(sum(F(a[i]) * y[i] for i in range(s)) + F(b) >= 0 for a, b in halfspaces):
            verts.add(y)
    return sorted(verts)


class Derived:
    """Stencil and tap polynomials of one reference sub-region."""

    def __init__(self, name, taps, polys, vertices, frame):
        self.name = name
        self.taps = taps          # list of integer offsets o_j (reference frame)
        self.polys = polys        # w_j(y) in the global-origin frame
        self.vertices = vertices
        self.frame = frame        # local frame origin y_c (rational)
        self.local = [p.translate(frame) for p in polys]  # w_j(u + y_c)


def lattice_points_in_box(spec, lo, hi):
    """All lattice sites n with lo_i <= n_i <= hi_i (integers)."""
    out = []
    rngs = [range(lo[i], hi[i] + 1) for i in range(spec.s)]
    for n in itertools.product(*rngs):
        if spec.in_lattice(n):
            out.append(n)
    return out


def derive_region(spec, bs: BoxSpline, region) -> Derived:
    s = spec.s
    verts = polytope_vertices(region.halfspaces, s)
    if len(verts) < s + 1:
        raise ValueError("degenerate region %s" % region.name)
    ybox = [(min(v[i] for v in verts), max(v[i] for v in verts)) for i in range(s)]
    y0 = tuple(F(x) for x in region.interior)
    for a, b in region.halfspaces:
        if sum(F(a[i]) * y0[i] for i in range(s)) + F(b) <= 0:
            raise ValueError("interior point not strictly inside %s" % region.name)
    lo = [int(_floor(ybox[i][0] - bs.halfwidth[i])) for i in range(s)]
    hi = [int(_ceil(ybox[i][1] + bs.halfwidth[i])) for i in range(s)]
    taps, polys = [], []
    for o in lattice_points_in_box(spec, lo, hi):
        p = bs.phi_piece(o, y0, ybox)
        if not p.is_zero():
            taps.append(tuple(o))
            polys.append(p)
    # partition of unity, exactly
    tot = Poly(s)
    for p in polys:
        tot.iadd(p)
    if tot != Poly.const(s, 1):
        raise AssertionError("weights of %s do not sum to one: %s" % (region.name, tot))
    # no knot plane of any stencil translate may cross the region's interior
    for nrm, g in bs.plane_families():
        vals = [sum(F(nrm[i]) * v[i] for i in range(s)) for v in verts]
        vmin, vmax = min(vals), max(vals)
        for o in taps:
            # knots of phi(y - o): nrm . (y - o + centre) in g Z
            base = sum(F(nrm[i]) * (F(o[i]) - bs.centre[i]) for i in range(s))
            # smallest knot value > vmin
            k = _floor((vmin - base) / g) + 1
            if base + k * g < vmax:
                raise AssertionError("knot plane %s . y = %s crosses region %s"
                                     % (nrm, base + k * g, region.name))
    frame = tuple(sum(v[i] for v in verts) / len(verts) for i in range(s))
    frame = tuple(_round_frac(x, 16) for x in frame)
    return Derived(region.name, taps, polys, verts, frame)


def _floor(x: F) -> int:
    return x.numerator // x.denominator


def _ceil(x: F) -> int:
    return -((-x.numerator) // x.denominator)


def _round_frac(x: F, den: int) -> F:
    return F(round(x * den), den)
