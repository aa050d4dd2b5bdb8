"""Automatic specs: the region of evaluation, the symmetry and the reference
sub-regions of a box spline found from its lattice and direction matrix alone.

This is the analysis the paper takes from its prequel (Sec. 3): choose a
region of evaluation (ROE) that tiles space under lattice shifts, reduce it
by the symmetries of the spline to a fundamental domain, and cut that domain
by the knot planes of the stencil translates into sub-regions on which the
convolution sum is one polynomial each.  Here:

  * symmetry: none for tensor products on Z^3 (separable code); else all
    signed permutations if the direction multiset is invariant under them
    (and the point-location code supports them on the lattice: Z^3 and BCC),
    else coordinate sign flips (FCC), else none (Z^3 only);
  * ROE: the Voronoi cell on BCC and FCC; on Z^3 the centred cube with
    symmetry, else whichever of the unit cube and the centred cube needs
    fewer sub-regions;
  * sub-regions: the cells of the knot-plane arrangement inside the
    fundamental domain, found by cutting it plane by plane in exact rational
    arithmetic.  The cuts form a binary tree, which is also the region
    lookup: at each node the point goes to the far side when n . y > t.

Every cell is then derived and checked by derive.derive_region (its stencil
polynomials sum to one and no knot plane crosses it).
"""
from __future__ import annotations

import itertools
from fractions import Fraction as F
from typing import List, Sequence, Tuple

from .derive import BoxSpline, _floor, polytope_vertices

HALF = F(1, 2)

LATTICES = {
    "cc": dict(L=[[1, 0, 0], [0, 1, 0], [0, 0, 1]], D=(1, 1, 1), shifts=[(0, 0, 0)]),
    "bcc": dict(L=[[-1, 1, 1], [1, -1, 1], [1, 1, -1]], D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 1)]),
    "fcc": dict(L=[[0, 1, 1], [1, 0, 1], [1, 1, 0]], D=(2, 2, 2),
                shifts=[(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]),
}


def _canon(d):
    sg = next(((x > 0) - (x < 0) for x in d if x), 1)
    return tuple(sg * x for x in d)


def _invariant(Xi, mats) -> bool:
    base = sorted(_canon(d) for d in Xi)
    for G in mats:
        img = sorted(_canon(tuple(sum(G[i][k] * d[k] for k in range(3)) for i in range(3))) for d in Xi)
        if img != base:
            return False
    return True


def _signed_perms():
    out = []
    for perm in itertools.permutations(range(3)):
        for sg in itertools.product((1, -1), repeat=3):
            out.append([[sg[i] if perm[i] == k else 0 for k in range(3)] for i in range(3)])
    return out


def _sign_flips():
    return [[[sg[i] if i == k else 0 for k in range(3)] for i in range(3)]
            for sg in itertools.product((1, -1), repeat=3)]


def _domain(lattice: str, roe: str, symmetry: str):
    """Half-spaces a . y + b >= 0 of the fundamental domain."""
    if lattice == "cc":
        if roe == "floor":
            return [((1, 0, 0), 0), ((0, 1, 0), 0), ((0, 0, 1), 0),
                    ((-1, 0, 0), 1), ((0, -1, 0), 1), ((0, 0, -1), 1)]
        if symmetry == "signed_perm":
            return [((1, -1, 0), 0), ((0, 1, -1), 0), ((0, 0, 1), 0), ((-1, 0, 0), HALF)]
        return [((1, 0, 0), HALF), ((0, 1, 0), HALF), ((0, 0, 1), HALF),
                ((-1, 0, 0), HALF), ((0, -1, 0), HALF), ((0, 0, -1), HALF)]
    if lattice == "bcc":
        return [((1, -1, 0), 0), ((0, 1, -1), 0), ((0, 0, 1), 0),
                ((-1, 0, 0), 1), ((-1, -1, -1), F(3, 2))]
    return [((1, 0, 0), 0), ((0, 1, 0), 0), ((0, 0, 1), 0),
            ((-1, -1, 0), 1), ((-1, 0, -1), 1), ((0, -1, -1), 1)]


def _dot(a, y):
    return sum(F(a[i]) * y[i] for i in range(3))


def _knot_planes(bs: BoxSpline, spec, verts) -> List[Tuple[Tuple[int, ...], F]]:
    """Every knot plane n . y = t of a stencil translate phi(y - o) that
    crosses the interior of the polytope with vertices verts."""
    lo = [min(v[i] for v in verts) for i in range(3)]
    hi = [max(v[i] for v in verts) for i in range(3)]
    olo = [_floor(lo[i] - bs.halfwidth[i]) - 1 for i in range(3)]
    ohi = [_floor(hi[i] + bs.halfwidth[i]) + 1 for i in range(3)]
    taps = [o for o in itertools.product(*[range(olo[i], ohi[i] + 1) for i in range(3)])
            if spec.in_lattice(o)]
    planes = set()
    for nrm, g in bs.plane_families():
        vals = [_dot(nrm, v) for v in verts]
        vmin, vmax = min(vals), max(vals)
        for o in taps:
            # knots of phi(y - o): nrm . (y - o + centre) in g Z
            base = sum(F(nrm[i]) * (F(o[i]) - bs.centre[i]) for i in range(3))
            k = _floor((vmin - base) / g) + 1
            while base + k * g < vmax:
                planes.add((nrm, base + k * g))
                k += 1
    return sorted(planes)


def _crosses(verts, nrm, t) -> bool:
    vals = [_dot(nrm, v) - t for v in verts]
    return min(vals) < 0 < max(vals)


def _split(halfspaces, planes, leaves):
    """Cut the polytope by the planes that cross it; returns the lookup tree
    (a leaf index, or (normal, t, near, far))."""
    verts = polytope_vertices(halfspaces, 3)
    for idx, (nrm, t) in enumerate(planes):
        if _crosses(verts, nrm, t):
            rest = planes[idx + 1:]
            near = _split(halfspaces + [(tuple(-x for x in nrm), t)], rest, leaves)
            far = _split(halfspaces + [(nrm, -t)], rest, leaves)
            return (nrm, t, near, far)
    leaves.append((halfspaces, verts))
    return len(leaves) - 1


def _cells(spec, bs: BoxSpline):
    dom = _domain(spec.lattice, spec.roe, spec.symmetry)
    planes = _knot_planes(bs, spec, polytope_vertices(dom, 3))
    leaves = []
    tree = _split(dom, planes, leaves)
    return tree, leaves


def auto_spec(name: str, lattice: str, Xi: Sequence[Tuple[int, ...]], kind: int = -1):
    """The Spec of the box spline with directions Xi on lattice ("cc", "bcc",
    "fcc"), with its sub-regions and region lookup found automatically."""
    from .specs import Region, Spec  # specs.py builds its own table with this function
    lat = LATTICES[lattice]
    Xi = [tuple(int(v) for v in d) for d in Xi]
    axis_only = all(sum(1 for v in d if v) == 1 for d in Xi)
    if lattice == "cc" and axis_only:
        # a tensor product: separable code without any symmetry transform
        symmetry = "none"
    elif _invariant(Xi, _signed_perms()) and lattice in ("cc", "bcc"):
        symmetry = "signed_perm"
    elif lattice == "fcc" and _invariant(Xi, _sign_flips()):
        symmetry = "signs"
    elif lattice == "cc":
        symmetry = "none"
    else:
        raise ValueError("%s: the %s point location needs a spline invariant under %s"
                         % (name, lattice, "sign flips" if lattice == "fcc" else "signed permutations"))
    if lattice != "cc":
        roes = ["voronoi"]
    elif symmetry == "signed_perm":
        roes = ["round"]
    else:
        roes = ["floor", "round"]
    best = None
    det = abs(_det3(lat["L"]))
    bs = BoxSpline(3, Xi, det)
    for roe in roes:
        spec = Spec(name=name, kind=kind, lattice=lattice, s=3, L=lat["L"], Xi=Xi, D=lat["D"],
                    shifts=lat["shifts"], roe=roe, symmetry=symmetry)
        tree, leaves = _cells(spec, bs)
        if best is None or len(leaves) < len(best[2]):
            best = (spec, tree, leaves)
    spec, tree, leaves = best
    spec.regions = []
    for k, (hs, verts) in enumerate(leaves):
        interior = tuple(sum(v[i] for v in verts) / len(verts) for i in range(3))
        spec.regions.append(Region("cell%d" % k, hs, interior))
    spec.tree = tree if len(leaves) > 1 else 0
    return spec


def _det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))
