"""The splines the library generates code for, with their lattices, regions of
evaluation and reference sub-regions.

Each spec states (Sec. 4.1.2, Sec. 4.1.3, Fig. 1):
  * the lattice L Z^3 as Cartesian cosets n = D * idx + shift_m (the memory
    layout is one array per coset, Sec. 4.1);
  * the direction matrix Xi of the box spline;
  * the ROE: a floor parallelepiped or the Voronoi cell of the lattice;
  * the symmetry used to reach the reference sub-regions: none, coordinate
    sign flips, or signed permutations (y = sort_desc |x - k|);
  * the reference sub-regions as half-space systems a . y + b >= 0, each with
    an interior point.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction as F
from typing import List, Sequence, Tuple


@dataclass
class Region:
    name: str
    halfspaces: List[Tuple[Tuple, object]]
    interior: Tuple


@dataclass
class Spec:
    name: str
    s: int
    L: Sequence[Sequence[int]]
    Xi: Sequence[Tuple[int, ...]]
    D: Tuple[int, ...]
    shifts: List[Tuple[int, ...]]
    roe: str                # "floor", "round" (cube [-1/2,1/2)^s) or "voronoi"
    symmetry: str           # "none", "signs", "signed_perm"
    regions: List[Region] = field(default_factory=list)
    # region selector for several reference sub-regions: (normal, threshold):
    # region 0 if normal . y <= threshold, else region 1
    selector: Tuple = None
    kind: int = -1          # index of the spline in the library's kind table
    lattice: str = "cc"     # "cc", "bcc" or "fcc"
    # region lookup for any number of reference sub-regions: a leaf index, or
    # (normal, t, near, far) -- far when normal . y > t (see auto.py); None:
    # from the selector
    tree: object = None

    def lookup_tree(self):
        if self.tree is not None:
            return self.tree
        if self.selector is not None:
            return (tuple(self.selector[0]), self.selector[1], 0, 1)
        return 0

    def in_lattice(self, n) -> bool:
        return any(all((n[i] - sh[i]) % self.D[i] == 0 for i in range(self.s)) for sh in self.shifts)

    @property
    def det_L(self) -> int:
        L = self.L
        if self.s == 2:
            return abs(L[0][0] * L[1][1] - L[0][1] * L[1][0])
        return abs(L[0][0] * (L[1][1] * L[2][2] - L[1][2] * L[2][1])
                   - L[0][1] * (L[1][0] * L[2][2] - L[1][2] * L[2][0])
                   + L[0][2] * (L[1][0] * L[2][1] - L[1][1] * L[2][0]))


E = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
DIAG = [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]

# Tensor-product cubic B-spline on Z^3 (Xi = [I I I I]); floor parallelepiped
# ROE [0,1)^3 is a single sub-region with no symmetry needed.
TRICUBIC = Spec(
    name="tricubic", kind=0, lattice="cc", s=3, L=[[1, 0, 0], [0, 1, 0], [0, 0, 1]], Xi=E * 4,
    D=(1, 1, 1), shifts=[(0, 0, 0)], roe="floor", symmetry="none",
    regions=[Region("unit_cube",
                    [((1, 0, 0), 0), ((0, 1, 0), 0), ((0, 0, 1), 0),
                     ((-1, 0, 0), 1), ((0, -1, 0), 1), ((0, 0, -1), 1)],
                    (F(1, 2), F(1, 3), F(1, 5)))])

# BCC lattice L = [[-1,1,1],[1,-1,1],[1,1,-1]] = 2Z^3 u (2Z^3 + 1); the four
# diagonals each twice.  Voronoi ROE (truncated octahedron |y_i| <= 1,
# sum |y_i| <= 3/2); the spline is invariant under all signed permutations, so
# y = sort_desc(|x - k|) lands in the wedge 0 <= y2 <= y1 <= y0, which no knot
# plane (y_i +- y_j in 2Z) crosses: one reference sub-region.
BCC8 = Spec(
    name="bcc8", kind=1, lattice="bcc", s=3, L=[[-1, 1, 1], [1, -1, 1], [1, 1, -1]], Xi=DIAG * 2,
    D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 1)], roe="voronoi", symmetry="signed_perm",
    regions=[Region("wedge",
                    [((1, -1, 0), 0), ((0, 1, -1), 0), ((0, 0, 1), 0),
                     ((-1, 0, 0), 1), ((-1, -1, -1), F(3, 2))],
                    (F(1, 2), F(3, 10), F(1, 10)))])

# FCC lattice D3 = {n : sum n even}, L = [[0,1,1],[1,0,1],[1,1,0]], stored as
# 4 cosets of 2Z^3.  Six directions (1,+-1,0), (1,0,+-1), (0,1,+-1).  Voronoi
# ROE (rhombic dodecahedron |y_i| + |y_j| <= 1); sign flips take a point to the
# positive octant, which the knot plane y0 + y1 + y2 = 1 cuts into two
# reference sub-regions (inner tetrahedron and outer piece).
FCC6 = Spec(
    name="fcc6", kind=2, lattice="fcc", s=3, L=[[0, 1, 1], [1, 0, 1], [1, 1, 0]],
    Xi=[(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)],
    D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)],
    roe="voronoi", symmetry="signs",
    regions=[Region("inner",
                    [((1, 0, 0), 0), ((0, 1, 0), 0), ((0, 0, 1), 0), ((-1, -1, -1), 1)],
                    (F(3, 10), F(1, 5), F(1, 10))),
             Region("outer",
                    [((1, 0, 0), 0), ((0, 1, 0), 0), ((0, 0, 1), 0), ((1, 1, 1), -1),
                     ((-1, -1, 0), 1), ((-1, 0, -1), 1), ((0, -1, -1), 1)],
                    (F(1, 2), F(7, 20), F(1, 4)))],
    selector=((1, 1, 1), 1))

_UNIT_CUBE = [((1, 0, 0), 0), ((0, 1, 0), 0), ((0, 0, 1), 0),
              ((-1, 0, 0), 1), ((0, -1, 0), 1), ((0, 0, -1), 1)]
_HALF = F(1, 2)
_CENTRED_CUBE = [((1, 0, 0), _HALF), ((0, 1, 0), _HALF), ((0, 0, 1), _HALF),
                 ((-1, 0, 0), _HALF), ((0, -1, 0), _HALF), ((0, 0, -1), _HALF)]

# Order-2 splines of the paper's first comparison (Sec. 5.1): the trilinear
# B-spline on Z^3 and the linear rhombic-dodecahedron box spline on BCC (the
# four diagonals once; four lookups per point).  The tensor-product
# quadratic on Z^3 (order 3) needs the centred cube as ROE, since its knot
# planes sit at half-integers.
TRILINEAR = Spec(
    name="trilinear", kind=3, lattice="cc", s=3, L=[[1, 0, 0], [0, 1, 0], [0, 0, 1]], Xi=E * 2,
    D=(1, 1, 1), shifts=[(0, 0, 0)], roe="floor", symmetry="none",
    regions=[Region("unit_cube", _UNIT_CUBE, (F(1, 2), F(1, 3), F(1, 5)))])

BCC4 = Spec(
    name="bcc4", kind=4, lattice="bcc", s=3, L=[[-1, 1, 1], [1, -1, 1], [1, 1, -1]], Xi=DIAG,
    D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 1)], roe="voronoi", symmetry="signed_perm",
    regions=[Region("wedge",
                    [((1, -1, 0), 0), ((0, 1, -1), 0), ((0, 0, 1), 0),
                     ((-1, 0, 0), 1), ((-1, -1, -1), F(3, 2))],
                    (F(1, 2), F(3, 10), F(1, 10)))])

TRIQUADRATIC = Spec(
    name="triquadratic", kind=5, lattice="cc", s=3, L=[[1, 0, 0], [0, 1, 0], [0, 0, 1]], Xi=E * 3,
    D=(1, 1, 1), shifts=[(0, 0, 0)], roe="round", symmetry="none",
    regions=[Region("centred_cube", _CENTRED_CUBE, (F(1, 5), F(1, 7), F(1, 11)))])

# Fourth-order splines of the paper's third comparison (Sec. 5.1).  The
# seven-direction box spline on Z^3 (the three axes and the four diagonals):
# centred-cube ROE; the spline is invariant under all signed permutations and
# its knot planes (y_i in Z + 1/2, y_i +- y_j in Z) miss the interior of the
# wedge 0 <= y2 <= y1 <= y0 <= 1/2, which is one reference sub-region.  The
# quartic box spline on BCC (the four diagonals and the three shortest
# axis-aligned lattice vectors 2 e_i): knot planes y_i in Z, y_i +- y_j in 2Z,
# so the wedge of the truncated octahedron is again one sub-region.
CC7 = Spec(
    name="cc7", kind=6, lattice="cc", s=3, L=[[1, 0, 0], [0, 1, 0], [0, 0, 1]], Xi=E + DIAG,
    D=(1, 1, 1), shifts=[(0, 0, 0)], roe="round", symmetry="signed_perm",
    regions=[Region("wedge",
                    [((1, -1, 0), 0), ((0, 1, -1), 0), ((0, 0, 1), 0), ((-1, 0, 0), _HALF)],
                    (F(3, 10), F(1, 5), F(1, 10)))])

BCC7 = Spec(
    name="bcc7", kind=7, lattice="bcc", s=3, L=[[-1, 1, 1], [1, -1, 1], [1, 1, -1]],
    Xi=DIAG + [(2, 0, 0), (0, 2, 0), (0, 0, 2)],
    D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 1)], roe="voronoi", symmetry="signed_perm",
    regions=[Region("wedge",
                    [((1, -1, 0), 0), ((0, 1, -1), 0), ((0, 0, 1), 0),
                     ((-1, 0, 0), 1), ((-1, -1, -1), F(3, 2))],
                    (F(1, 2), F(3, 10), F(1, 10)))])

def _auto_specs():
    # splines whose ROE, symmetry and reference sub-regions are derived from
    # (L, Xi) alone (auto.py): the six face diagonals on Z^3 (degree 3, C^1;
    # three reference sub-regions in the wedge of the centred cube)
    from .auto import auto_spec
    return [auto_spec("cc6", "cc", [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)],
                      kind=8)]


SPECS = {sp.name: sp for sp in sorted((TRICUBIC, BCC8, FCC6, TRILINEAR, BCC4, TRIQUADRATIC, CC7, BCC7)
                                      + tuple(_auto_specs()), key=lambda sp: sp.kind)}
