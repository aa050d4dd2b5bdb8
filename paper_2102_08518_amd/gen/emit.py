"""Emit HIP device code and a JSON table description for each spline.

For every reference sub-region the emitted code contains (Sec. 4.3, Sec. 4.4):

  * ``<name>_eval_r<k>(c, y0, y1, y2)``: the sub-region polynomial in
    multivariate Horner form.  The coefficients of the monomials are first
    formed from the fetched stencil values (one group holding every tap), then
    a single Horner pass runs over the local coordinates u = y - frame.
  * ``<name>_eval_grad_r<k>``: value and the three partial derivatives in the
    reference frame (derivatives of the sub-region polynomial, Sec. 3).
  * ``<name>_weights_r<k>``: the per-tap weights w_j(u), each in Horner form
    (group size one), used by the backward pass.

For a tensor-product spline (exact factorisation checked here) the code is the
separable contraction instead of the expanded polynomial.

The JSON file records the stencils, frames and exact rational polynomials so a
plain CPU interpreter can check the tables without a GPU.
"""
from __future__ import annotations

import itertools
import json
import os
import re
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .derive import BoxSpline, Derived, derive_region
from .poly import Poly
from .specs import SPECS, Spec, Region

F = Fraction
HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(os.path.dirname(HERE), "csrc", "generated")


def flit(x) -> str:
    """FP32 literal (round-to-nearest of the exact rational)."""
    v = float(np.float32(float(x)))
    if v == 0:
        return "0.0f"
    r = repr(v)
    if "e" not in r and "." not in r:
        r += ".0"
    return r + "f"


# ----------------------------------------------------------- frame choice

def _region_samples(region: Region, verts, n=4000, seed=7):
    rng = np.random.default_rng(seed)
    V = np.array([[float(x) for x in v] for v in verts])
    w = rng.dirichlet(np.ones(len(V)), size=n)
    return w @ V


def condition(polys: Sequence[Poly], frame, pts) -> float:
    """max over sample points of sum_j sum_m |W_jm| |u^m| (a-priori error scale)."""
    U = pts - np.array([float(x) for x in frame])
    tot = np.zeros(len(U))
    for p in polys:
        q = p.translate(frame)
        for e, c in q.t.items():
            tot += abs(float(c)) * np.abs(np.prod([U[:, i] ** e[i] for i in range(len(e))], axis=0))
    return float(tot.max())


def choose_frame(d: Derived, region: Region, max_cond=6.5):
    pts = _region_samples(region, d.vertices)
    cands = [tuple(F(0) for _ in d.frame), d.frame] + list(d.vertices)
    best = None
    for fr in cands:
        loc = [p.translate(fr) for p in d.polys]
        nnz = sum(len(p.t) for p in loc)
        cond = condition(d.polys, fr, pts)
        key = (cond > max_cond, nnz, cond)
        if best is None or key < best[0]:
            best = (key, fr, nnz, cond)
    return best[1], best[2], best[3]


# ----------------------------------------------------------- symmetry group

def symmetry_elements(symmetry: str):
    """(sym id, axis, sgn) for every element G of the symmetry used to reach the
    reference sub-region, in the encoding the device code uses: reference axis r
    maps to global axis axis[r] with sign sgn[r], so (G^T o)[axis[r]] =
    sgn[r] * o[r]; sym id = (axis[0] * 3 + axis[1]) * 8 + (bits of sgn < 0)."""
    out = []
    perms = [(0, 1, 2)] if symmetry in ("none", "signs") else list(itertools.permutations(range(3)))
    signs = [(1, 1, 1)] if symmetry == "none" else list(itertools.product((1, -1), repeat=3))
    for ax in perms:
        for sg in signs:
            bits = sum(1 << r for r in range(3) if sg[r] < 0)
            sid = bits if symmetry != "signed_perm" else (ax[0] * 3 + ax[1]) * 8 + bits
            out.append((sid, ax, sg))
    return out


def transposed_stencil(union, symmetry: str):
    """U: every global offset G^T o_j over the group and the union stencil
    (sorted z, y, x); J[sym][u]: the union tap j with G^T o_j = U[u], or -1."""
    els = symmetry_elements(symmetry)
    vs = set()
    img = {}
    for sid, ax, sg in els:
        for j, o in enumerate(union):
            v = [0, 0, 0]
            for r in range(3):
                v[ax[r]] = sg[r] * o[r]
            v = tuple(v)
            vs.add(v)
            img[(sid, v)] = j
    U = sorted(vs, key=lambda v: (v[2], v[1], v[0]))
    nsym = 1 if symmetry == "none" else (8 if symmetry == "signs" else 72)
    J = [[img.get((sid, v), -1) for v in U] for sid in range(nsym)]
    return U, J


# ----------------------------------------------------------- code helpers

def horner(terms: Dict[Tuple[int, ...], str], nvars: int, names: Sequence[str]) -> str:
    """Nested multivariate Horner expression for sum_e terms[e] * u^e."""
    if not terms:
        return "0.0f"

    def rec(tms: Dict[Tuple[int, ...], str], var: int) -> str:
        if var == nvars:
            assert len(tms) == 1
            return next(iter(tms.values()))
        groups: Dict[int, Dict] = {}
        for e, t in tms.items():
            groups.setdefault(e[var], {})[e] = t
        kmax = max(groups)
        acc = rec(groups[kmax], var + 1)
        for k in range(kmax - 1, -1, -1):
            if k in groups:
                acc = "fmaf(%s, %s, %s)" % (acc, names[var], rec(groups[k], var + 1))
            else:
                acc = "(%s) * %s" % (acc, names[var])
        return acc

    return rec(terms, 0)


def lin_comb(pairs: List[Tuple[str, F]]) -> str:
    """sum of var * const as a chain of fmaf."""
    pairs = [(v, c) for v, c in pairs if c != 0]
    if not pairs:
        return "0.0f"
    v0, c0 = pairs[0]
    expr = "%s * %s" % (v0, flit(c0))
    for v, c in pairs[1:]:
        expr = "fmaf(%s, %s, %s)" % (v, flit(c), expr)
    return expr


def cse_pairs(rows: List[Dict[str, F]]):
    """Greedy common-subexpression elimination for a linear map.

    rows[m] maps input names to exact coefficients (row m = sum_v w_v v).  A
    temporary t = v_i + r v_j replaces the pair (v_i, v_j) in every row where
    both occur with coefficient ratio w_j / w_i = r; the pair occurring in the
    most rows is taken first, until no pair occurs twice.  Returns the
    temporaries [(name, v_i, v_j, r)] in evaluation order and the rewritten
    rows (over inputs and temporaries).  The rewriting is exact: expanding
    the temporaries gives back the original rows (checked here)."""
    rows = [dict(r) for r in rows]
    temps = []
    while True:
        cnt: Dict[Tuple[str, str, F], int] = {}
        for r in rows:
            items = sorted(r.items())
            for a in range(len(items)):
                for b in range(a + 1, len(items)):
                    (vi, wi), (vj, wj) = items[a], items[b]
                    key = (vi, vj, wj / wi)
                    cnt[key] = cnt.get(key, 0) + 1
        if not cnt:
            break
        best = max(cnt.items(), key=lambda kv: (kv[1], -abs(kv[0][2].numerator) - kv[0][2].denominator))
        (vi, vj, ratio), n = best
        if n < 2:
            break
        t = "t%d" % len(temps)
        temps.append((t, vi, vj, ratio))
        for r in rows:
            if vi in r and vj in r and r[vj] / r[vi] == ratio:
                w = r.pop(vi)
                r.pop(vj)
                r[t] = w
    return temps, rows


def cse_expand(temps, rows):
    """Inverse of cse_pairs: rows over the original inputs only."""
    defs: Dict[str, Dict[str, F]] = {}
    for t, vi, vj, ratio in temps:
        d: Dict[str, F] = {}
        for v, w in ((vi, F(1)), (vj, ratio)):
            for u, x in (defs[v].items() if v in defs else ((v, F(1)),)):
                d[u] = d.get(u, F(0)) + w * x
        defs[t] = d
    out = []
    for r in rows:
        e: Dict[str, F] = {}
        for v, w in r.items():
            for u, x in (defs[v].items() if v in defs else ((v, F(1)),)):
                e[u] = e.get(u, F(0)) + w * x
        out.append({u: x for u, x in e.items() if x != 0})
    return out


# ----------------------------------------------------------- emission

class SplineCode:
    def __init__(self, spec: Spec):
        self.spec = spec
        self.bs = BoxSpline(spec.s, spec.Xi, spec.det_L)
        self.regions: List[Derived] = [derive_region(spec, self.bs, r) for r in spec.regions]
        self.frames, self.nnz, self.cond = [], [], []
        for d, r in zip(self.regions, spec.regions):
            fr, nnz, cond = choose_frame(d, r)
            self.frames.append(fr)
            self.nnz.append(nnz)
            self.cond.append(cond)
        # union stencil (order: first region's taps, then new ones)
        union: List[Tuple[int, ...]] = []
        for d in self.regions:
            for o in d.taps:
                if o not in union:
                    union.append(o)
        # order taps for locality: z-major, then y, then x (x fastest)
        union.sort(key=lambda o: (o[2], o[1], o[0]))
        self.union = union
        self.tensor = self._tensor_factors() if spec.symmetry == "none" else None

    # tensor-product detection: w_(i,j,k)(y) == b_i(y0) b_j(y1) b_k(y2)
    def _tensor_factors(self):
        spec = self.spec
        if len(self.regions) != 1:
            return None
        d = self.regions[0]
        axis_dirs = [tuple(x[i] for x in spec.Xi) for i in range(spec.s)]
        mult = []
        for i in range(spec.s):
            cnt = sum(1 for x in spec.Xi if sum(abs(v) for v in x) == abs(x[i]) and x[i] != 0)
            mult.append(cnt)
        if sum(mult) != len(spec.Xi):
            return None
        # 1D pieces from the same derivation in one dimension
        from .specs import Region as R
        from . import derive as dv

        class Spec1:
            s = 1
            D = (1,)
            shifts = [(0,)]

            def in_lattice(self, n):
                return True

        fac = []
        for i in range(spec.s):
            bs1 = dv.BoxSpline(1, [(1,)] * mult[i], 1)
            if spec.roe == "round":
                reg = R("centred", [((1,), F(1, 2)), ((-1,), F(1, 2))], (F(1, 5),))
            else:
                reg = R("unit", [((1,), 0), ((-1,), 1)], (F(1, 3),))
            d1 = dv.derive_region(Spec1(), bs1, reg)
            fac.append(dict(zip([o[0] for o in d1.taps], d1.polys)))
        for o, p in zip(d.taps, d.polys):
            prod = Poly.const(spec.s, 1)
            for i in range(spec.s):
                q = fac[i][o[i]]
                lifted = Poly(spec.s, {tuple(e[0] if a == i else 0 for a in range(spec.s)): c
                                       for e, c in q.t.items()})
                prod = prod * lifted
            if prod != p:
                return None
        return fac

    # -- JSON description
    def tables(self) -> dict:
        spec = self.spec
        regs = []
        for d, fr, nnz, cond in zip(self.regions, self.frames, self.nnz, self.cond):
            loc = [p.translate(fr) for p in d.polys]
            regs.append({
                "name": d.name,
                "taps": [list(o) for o in d.taps],
                "union_index": [self.union.index(o) for o in d.taps],
                "frame": [str(x) for x in fr],
                "vertices": [[str(x) for x in v] for v in d.vertices],
                "nnz": nnz,
                "cond": cond,
                "weights": [{",".join(map(str, e)): str(c) for e, c in q.t.items()} for q in loc],
            })
        return {
            "name": spec.name, "kind": spec.kind, "lattice": spec.lattice, "s": spec.s,
            "L": [list(r) for r in spec.L],
            "Xi": [list(x) for x in spec.Xi], "D": list(spec.D), "shifts": [list(x) for x in spec.shifts],
            "roe": spec.roe, "symmetry": spec.symmetry,
            "selector": None if spec.selector is None else [list(spec.selector[0]), spec.selector[1]],
            "tree": _tree_json(spec.lookup_tree()),
            "degree": self.bs.degree, "union": [list(o) for o in self.union],
            "radius": max(abs(v) for o in self.union for v in o),
            "tensor": self.tensor is not None,
            "regions": regs,
            "transposed": dict(zip(("U", "J"), transposed_stencil(self.union, spec.symmetry))),
            "mfma": self._mfma_json(),
        }

    def _mfma_json(self):
        form = self.mfma_form()
        if form is None:
            return None
        _, _, mons, _ = self._region_terms(0)
        return {"Q": form["Q"], "rows": form["rows"], "Wq": form["Wq"],
                "monomials": [list(e) for e in mons]}

    # -- counts
    def fma_counts(self) -> dict:
        if self.tensor is not None:
            n = [len(f) for f in self.tensor]
            nt = int(np.prod(n))
            w = sum(sum(len(p.t) for p in f.values()) for f in self.tensor)
            contract = nt + n[1] * n[2] + n[2]
            return {"eval": w + contract, "weights": w + nt}
        out = {}
        ev = 0
        for k in range(len(self.regions)):
            temps, rows = self._coef_cse(k)
            ev += len(temps) + sum(len(r) for r in rows) + len(rows)
        out["eval"] = ev
        out["weights"] = sum(min(self._weights_cost(k)) for k in range(len(self.regions)))
        return out

    # -- code
    def emit(self) -> str:
        spec = self.spec
        nm = spec.name
        L = []
        L.append("// Generated by paper_2102_08518_amd.gen.emit from the exact sub-region analysis")
        L.append("// of the %s box spline.  Do not edit; regenerate with" % nm)
        L.append("//   python -m paper_2102_08518_amd.gen")
        L.append("#pragma once")
        L.append("")
        L.append("namespace lsp {")
        L.append("namespace gen {")
        L.append("")
        L.append("struct %s_tables {" % nm)
        L.append("  static constexpr int kKind = %d;" % spec.kind)
        L.append("  static constexpr int kLattice = %d;    // 0 Z^3, 1 BCC, 2 FCC" % {"cc": 0, "bcc": 1, "fcc": 2}[spec.lattice])
        L.append("  static constexpr int kRoe = %d;        // 0 floor cube, 1 centred cube, 2 Voronoi cell" % {"floor": 0, "round": 1, "voronoi": 2}[spec.roe])
        L.append("  static constexpr int kSymmetry = %d;   // 0 none, 1 reflections, 2 signed permutations" % {"none": 0, "signs": 1, "signed_perm": 2}[spec.symmetry])
        L.append("  static constexpr int kD = %d;          // coset scale" % spec.D[0])
        L.append("  static constexpr int kNumCosets = %d;" % len(spec.shifts))
        L.append("  static constexpr int kShift[4][3] = {%s};" % ", ".join(
            "{%d, %d, %d}" % tuple(spec.shifts[m]) if m < len(spec.shifts) else "{0, 0, 0}" for m in range(4)))
        L.append("  // lattice generators (columns) and box-spline directions (rows)")
        L.append("  static constexpr int kL[3][3] = {%s};" % ", ".join("{%d, %d, %d}" % tuple(r) for r in spec.L))
        L.append("  static constexpr int kNumDirs = %d;" % len(spec.Xi))
        L.append("  static constexpr int kXi[kNumDirs][3] = {%s};" % ", ".join("{%d, %d, %d}" % tuple(x) for x in spec.Xi))
        L.append("  static constexpr int kTaps = %d;       // union stencil size" % len(self.union))
        L.append("  static constexpr int kRegions = %d;    // reference sub-regions" % len(self.regions))
        L.append("  static constexpr int kRadius = %d;     // max |offset component|" % max(abs(v) for o in self.union for v in o))
        L.append("  static constexpr int kDegree = %d;" % self.bs.degree)
        L.append("  static constexpr bool kTensor = %s;" % ("true" if self.tensor is not None else "false"))
        fc = self.fma_counts()
        L.append("  static constexpr int kFmaEval = %d;    // FMAs of the value polynomial(s)" % fc["eval"])
        L.append("  static constexpr int kFmaWeights = %d; // FMAs of all per-tap weights" % fc["weights"])
        offs = ", ".join("{%d, %d, %d}" % o for o in self.union)
        L.append("  // reference-frame stencil offsets o_j (lattice vectors), x fastest")
        L.append("  static constexpr signed char kOff[kTaps][3] = {%s};" % offs)
        par = ", ".join(str((o[0] & 1) | ((o[1] & 1) << 1) | ((o[2] & 1) << 2)) for o in self.union)
        L.append("  // parity pattern of each offset: bit0 x, bit1 y, bit2 z")
        L.append("  static constexpr unsigned char kParity[kTaps] = {%s};" % par)
        L.append("  // order in which the gather issues the tap loads: the order in which the")
        L.append("  // code of the first sub-region's polynomial first reads them (loads complete")
        L.append("  // in issue order, so the polynomial can start on the first ones)")
        L.append("  static constexpr unsigned char kIssue[kTaps] = {%s};" % ", ".join(str(j) for j in self.issue_order()))
        for k, d in enumerate(self.regions):
            mask = sum(1 << self.union.index(o) for o in d.taps)
            L.append("  static constexpr unsigned long long kRegionMask%d = 0x%xull;" % (k, mask))
        U, J = transposed_stencil(self.union, spec.symmetry)
        L.append("  // transposed stencil: every offset G^T o_j over the symmetry group, and the")
        L.append("  // union tap j that lands there for each symmetry element (-1: none)")
        L.append("  static constexpr int kNumU = %d;" % len(U))
        L.append("  static constexpr int kNumSym = %d;" % len(J))
        L.append("  static constexpr signed char kU[kNumU][3] = {%s};" % ", ".join("{%d, %d, %d}" % v for v in U))
        L.append("  static constexpr signed char kJ[kNumSym][kNumU] = {%s};" % ", ".join(
            "{%s}" % ", ".join(str(j) for j in row) for row in J))
        L.append("};")
        L.append("")
        if self.tensor is not None:
            L += self._emit_tensor()
        else:
            for k in range(len(self.regions)):
                L += self._emit_region(k)
        L += self._emit_poly_struct()
        L += self._emit_mfma()
        L.append("}  // namespace gen")
        L.append("}  // namespace lsp")
        L.append("")
        return "\n".join(L)

    def _region_terms(self, k: int):
        """Local tap polynomials of sub-region k, their union-tap indices, and the
        monomials in the order of the coefficient array A."""
        d = self.regions[k]
        loc = [p.translate(self.frames[k]) for p in d.polys]
        uidx = [self.union.index(o) for o in d.taps]
        mons = sorted(set().union(*[set(q.t) for q in loc]), key=lambda e: (-sum(e), e))
        return loc, uidx, mons, {e: i for i, e in enumerate(mons)}

    def issue_order(self) -> List[int]:
        """Union tap indices in the order the emitted coefficient code of
        sub-region 0 first reads them, then any taps it does not read; table
        order for the separable splines (their code reads the taps slab by
        slab in table order)."""
        n = len(self.union)
        if self.tensor is not None:
            return list(range(n))
        temps, rows = self._coef_cse(0)
        text = [lin_comb([(vi, F(1)), (vj, ratio)]) for _, vi, vj, ratio in temps]
        text += [lin_comb(sorted(row.items())) for row in rows]
        order = []
        for expr in text:
            for tok in re.findall(r"\bc\[(\d+)\]", expr):
                if int(tok) not in order:
                    order.append(int(tok))
        order += [j for j in range(n) if j not in order]
        return order

    def _coef_cse(self, k: int):
        """Monomial coefficients of sub-region k (row m = A[m], over the
        fetched values c[j] of the union stencil) after pair elimination."""
        memo = self.__dict__.setdefault("_cse_memo", {})
        if k in memo:
            return memo[k]
        memo[k] = self._coef_cse_uncached(k)
        return memo[k]

    def _coef_cse_uncached(self, k: int):
        loc, uidx, mons, midx = self._region_terms(k)
        rows = [{"c[%d]" % uidx[j]: q.t[e] for j, q in enumerate(loc) if e in q.t} for e in mons]
        temps, new = cse_pairs(rows)
        assert cse_expand(temps, new) == [{v: w for v, w in r.items() if w != 0} for r in rows]
        return temps, new

    def _weights_cost(self, k: int):
        """(Horner per tap, monomials + shared pairs) operation counts."""
        mono, temps, rows = self._weights_cse(k)
        return self.nnz[k], len(mono) - 1 + len(temps) + sum(len(r) for r in rows)

    def _weights_use_cse(self, k: int) -> bool:
        horner_ops, cse_ops = self._weights_cost(k)
        return cse_ops < horner_ops

    def _weights_cse(self, k: int):
        """Per-tap weights of sub-region k as combinations of monomials:
        the monomials (each a lower one times one coordinate, in order of
        degree), the pair temporaries and one row per tap."""
        loc, uidx, mons, midx = self._region_terms(k)
        name = lambda e: "m%d%d%d" % e
        need = set(mons)
        for e in list(need):
            f = list(e)
            while sum(f) > 0:   # parents along the first nonzero exponent
                i = next(a for a in range(3) if f[a] > 0)
                f[i] -= 1
                need.add(tuple(f))
        mono = []
        for e in sorted(need, key=lambda e: (sum(e), e)):
            if sum(e) == 0:
                mono.append((name(e), None, None))
            else:
                i = next(a for a in range(3) if e[a] > 0)
                f = list(e)
                f[i] -= 1
                mono.append((name(e), name(tuple(f)), i))
        rows = [{name(e): c for e, c in q.t.items()} for q in loc]
        temps, new = cse_pairs(rows)
        assert cse_expand(temps, new) == [{v: w for v, w in r.items() if w != 0} for r in rows]
        return mono, temps, new

    def mfma_form(self):
        """Integer form of the weight matrix for the matrix-core path.

        With one reference sub-region the monomial coefficients are A = W c,
        W (monomials x union taps) constant.  Q is the least common denominator
        of W; Wq = Q W is an integer matrix.  The form applies when Wq fits a
        64 x 32 tile and every entry is exact in bfloat16 (at most 8 significant
        bits), so the matrix cores form every product W_mj c_j without rounding.
        Returns None otherwise."""
        if self.tensor is not None or len(self.regions) != 1 or len(self.union) > 32:
            return None
        loc, uidx, mons, midx = self._region_terms(0)
        if len(mons) > 64:
            return None
        Q = 1
        for q in loc:
            for c in q.t.values():
                Q = Q * c.denominator // np.gcd(Q, c.denominator)
        Wq = [[0] * 32 for _ in range(64)]
        for j, q in enumerate(loc):
            for e, c in q.t.items():
                v = c * Q
                assert v.denominator == 1
                Wq[midx[e]][uidx[j]] = int(v)

        def sig_bits(n):
            n = abs(n)
            while n and n % 2 == 0:
                n //= 2
            return n.bit_length()

        if any(sig_bits(v) > 8 or abs(v) >= 2 ** 15 for row in Wq for v in row):
            return None
        return {"Q": int(Q), "rows": len(mons), "Wq": Wq}

    def _emit_mfma(self) -> List[str]:
        nm = self.spec.name
        form = self.mfma_form()
        L = ["// matrix-core form of the sub-region polynomial: the monomial coefficients",
             "// are A = (Wq c) / kQ, Wq an integer matrix exact in bfloat16 (rows: the",
             "// monomials in the order of A, padded to 64; columns: union taps, padded",
             "// to 32); value/value_grad take Q A and return unscaled results",
             "struct %s_mfma {" % nm]
        if form is None:
            L += ["  static constexpr bool kOk = false;", "};", ""]
            return L
        loc, uidx, mons, midx = self._region_terms(0)
        fr = self.frames[0]
        L.append("  static constexpr bool kOk = true;")
        L.append("  static constexpr int kRows = %d;" % form["rows"])
        L.append("  static constexpr int kQ = %d;" % form["Q"])
        L.append("  static constexpr short kWq[64][32] = {%s};" % ", ".join(
            "{%s}" % ", ".join(str(v) for v in row) for row in form["Wq"]))
        frame_lines = ["    const float u%d = y%d - %s;" % (i, i, flit(fr[i])) if fr[i] != 0
                       else "    const float u%d = y%d;" % (i, i) for i in range(3)]
        L.append("  static __device__ __forceinline__ float value(const float* __restrict__ A, float y0, float y1, float y2) {")
        L += frame_lines
        L.append("    return %s;" % horner({e: "A[%d]" % midx[e] for e in mons}, 3, ["u0", "u1", "u2"]))
        L.append("  }")
        L.append("  static __device__ __forceinline__ float value_grad(const float* __restrict__ A, float y0, float y1, float y2,")
        L.append("                                                    float& g0, float& g1, float& g2) {")
        L += frame_lines
        for r in range(3):
            dt = {}
            for e in mons:
                if e[r]:
                    e2 = list(e)
                    e2[r] -= 1
                    dt[tuple(e2)] = "A[%d]" % midx[e] if e[r] == 1 else "(A[%d] * %d.0f)" % (midx[e], e[r])
            L.append("    g%d = %s;" % (r, horner(dt, 3, ["u0", "u1", "u2"])))
        L.append("    return %s;" % horner({e: "A[%d]" % midx[e] for e in mons}, 3, ["u0", "u1", "u2"]))
        L.append("  }")
        L += ["};", ""]
        return L

    def _emit_region(self, k: int) -> List[str]:
        nm = self.spec.name
        d = self.regions[k]
        fr = self.frames[k]
        loc, uidx, mons, midx = self._region_terms(k)
        L = []
        frame_lines = ["  const float u%d = y%d - %s;" % (i, i, flit(fr[i])) if fr[i] != 0
                       else "  const float u%d = y%d;" % (i, i) for i in range(3)]
        # value (monomial coefficients first, then one Horner pass)
        L.append("// sub-region %d (%s): %d taps, frame (%s), %d weight terms, cond %.2f"
                 % (k, d.name, len(d.taps), ", ".join(str(x) for x in fr), self.nnz[k], self.cond[k]))
        L.append("__device__ __forceinline__ void %s_coef_r%d(const float* __restrict__ c, float* __restrict__ A) {" % (nm, k))
        temps, rows = self._coef_cse(k)
        for t, vi, vj, ratio in temps:
            L.append("  const float %s = %s;" % (t, lin_comb([(vi, F(1)), (vj, ratio)])))
        for m, row in enumerate(rows):
            L.append("  A[%d] = %s;" % (m, lin_comb(sorted(row.items()))))
        L.append("}")
        L.append("")
        L.append("__device__ __forceinline__ float %s_eval_r%d(const float* __restrict__ c, float y0, float y1, float y2) {" % (nm, k))
        L += frame_lines
        L.append("  float A[%d];" % len(mons))
        L.append("  %s_coef_r%d(c, A);" % (nm, k))
        L.append("  return %s;" % horner({e: "A[%d]" % midx[e] for e in mons}, 3, ["u0", "u1", "u2"]))
        L.append("}")
        L.append("")
        # value + gradient
        L.append("__device__ __forceinline__ float %s_eval_grad_r%d(const float* __restrict__ c, float y0, float y1, float y2," % (nm, k))
        L.append("                                                float& g0, float& g1, float& g2) {")
        L += frame_lines
        L.append("  float A[%d];" % len(mons))
        L.append("  %s_coef_r%d(c, A);" % (nm, k))
        for r in range(3):
            dt = {}
            for e in mons:
                if e[r]:
                    e2 = list(e)
                    e2[r] -= 1
                    term = "A[%d]" % midx[e] if e[r] == 1 else "(A[%d] * %d.0f)" % (midx[e], e[r])
                    dt[tuple(e2)] = term
            L.append("  g%d = %s;" % (r, horner(dt, 3, ["u0", "u1", "u2"])))
        L.append("  return %s;" % horner({e: "A[%d]" % midx[e] for e in mons}, 3, ["u0", "u1", "u2"]))
        L.append("}")
        L.append("")
        # value, gradient and Hessian (h: d2/du0du0, du0du1, du0du2, du1du1,
        # du1du2, du2du2)
        L.append("__device__ __forceinline__ float %s_eval_hess_r%d(const float* __restrict__ c, float y0, float y1, float y2," % (nm, k))
        L.append("                                                float& g0, float& g1, float& g2, float* __restrict__ h) {")
        L += frame_lines
        L.append("  float A[%d];" % len(mons))
        L.append("  %s_coef_r%d(c, A);" % (nm, k))
        for r in range(3):
            dt = {}
            for e in mons:
                if e[r]:
                    e2 = list(e)
                    e2[r] -= 1
                    dt[tuple(e2)] = "A[%d]" % midx[e] if e[r] == 1 else "(A[%d] * %d.0f)" % (midx[e], e[r])
            L.append("  g%d = %s;" % (r, horner(dt, 3, ["u0", "u1", "u2"])))
        for hi_, (r, q) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
            dt = {}
            for e in mons:
                e2 = list(e)
                k1 = e2[r]
                e2[r] -= 1
                k2 = e2[q]
                e2[q] -= 1
                if k1 > 0 and k2 > 0:
                    mult = k1 * k2
                    dt[tuple(e2)] = "A[%d]" % midx[e] if mult == 1 else "(A[%d] * %d.0f)" % (midx[e], mult)
            L.append("  h[%d] = %s;" % (hi_, horner(dt, 3, ["u0", "u1", "u2"])))
        L.append("  return %s;" % horner({e: "A[%d]" % midx[e] for e in mons}, 3, ["u0", "u1", "u2"]))
        L.append("}")
        L.append("")
        # per-tap weights (union-indexed; taps outside this sub-region get 0):
        # the monomials once, then every weight as a combination of them with
        # shared pair terms
        L.append("__device__ __forceinline__ void %s_weights_r%d(float y0, float y1, float y2, float* __restrict__ w) {" % (nm, k))
        L += frame_lines
        for j in range(len(self.union)):
            if j not in uidx:
                L.append("  w[%d] = 0.0f;" % j)
        if self._weights_use_cse(k):
            mono, temps, rows = self._weights_cse(k)
            for name, parent, var in mono:
                L.append("  const float %s = %s;" % (name, "1.0f" if parent is None else "%s * u%d" % (parent, var)))
            for t, vi, vj, ratio in temps:
                L.append("  const float %s = %s;" % (t, lin_comb([(vi, F(1)), (vj, ratio)])))
            for j, row in enumerate(rows):
                L.append("  w[%d] = %s;" % (uidx[j], lin_comb(sorted(row.items()))))
        else:
            for j, q in enumerate(loc):
                L.append("  w[%d] = %s;" % (uidx[j], horner({e: flit(c) for e, c in q.t.items()}, 3, ["u0", "u1", "u2"])))
        L.append("}")
        L.append("")
        return L

    def _emit_tensor(self) -> List[str]:
        nm = self.spec.name
        fac = self.tensor
        L = []
        taps1 = [sorted(f) for f in fac]
        for i in range(3):
            L.append("// axis %d: 1D weights at offsets %s on [0,1)" % (i, taps1[i]))
            L.append("__device__ __forceinline__ void %s_w1d_%d(float t, float* w, float* dw, float* ddw = nullptr) {" % (nm, i))
            for a, o in enumerate(taps1[i]):
                q = fac[i][o]
                L.append("  w[%d] = %s;" % (a, horner({e: flit(c) for e, c in q.t.items()}, 1, ["t"])))
                dq = q.deriv(0)
                L.append("  if (dw) dw[%d] = %s;" % (a, horner({e: flit(c) for e, c in dq.t.items()}, 1, ["t"])))
                ddq = dq.deriv(0)
                L.append("  if (ddw) ddw[%d] = %s;" % (a, horner({e: flit(c) for e, c in ddq.t.items()}, 1, ["t"])))
            L.append("}")
            L.append("")
        n0, n1, n2 = (len(t) for t in taps1)
        N = max(n0, n1, n2)
        idx = {o: j for j, o in enumerate(self.union)}

        def cidx(a, b, cc):
            return idx[(taps1[0][a], taps1[1][b], taps1[2][cc])]

        def W(o, axis, a):
            # the 1D weight of derivative order o along axis at its a-th offset
            return "w[%d]" % ((o * 3 + axis) * N + a)

        # the y-dependent part, separable from the coefficients: the 1D
        # weights of derivative orders 0..DER, w[(order * 3 + axis) * N + a]
        L.append("// 1D weights of derivative orders 0..DER along the three axes,")
        L.append("// w[(order * 3 + axis) * %d + a]: all that depends on y alone" % N)
        L.append("template <int DER>")
        L.append("__device__ __forceinline__ void %s_pre(float y0, float y1, float y2, float* __restrict__ w) {" % nm)
        for i, y in enumerate(("y0", "y1", "y2")):
            L.append("  %s_w1d_%d(%s, w + %d, DER >= 1 ? w + %d : nullptr, DER >= 2 ? w + %d : nullptr);"
                     % (nm, i, y, i * N, (3 + i) * N, (6 + i) * N))
        L.append("}")
        L.append("")
        # value
        L.append("__device__ __forceinline__ float %s_eval_r0_pre(const float* __restrict__ c, const float* __restrict__ w) {" % nm)
        L.append("  float f = 0.0f;")
        for cc in range(n2):
            L.append("  {")
            L.append("    float r = 0.0f;")
            for b in range(n1):
                e = "c[%d] * %s" % (cidx(0, b, cc), W(0, 0, 0))
                for a in range(1, n0):
                    e = "fmaf(c[%d], %s, %s)" % (cidx(a, b, cc), W(0, 0, a), e)
                L.append("    r = fmaf(%s, %s, r);" % (e, W(0, 1, b)))
            L.append("    f = fmaf(r, %s, f);" % W(0, 2, cc))
            L.append("  }")
        L.append("  return f;")
        L.append("}")
        L.append("")
        # value + gradient
        L.append("__device__ __forceinline__ float %s_eval_grad_r0_pre(const float* __restrict__ c, const float* __restrict__ w," % nm)
        L.append("                                                    float& g0, float& g1, float& g2) {")
        L.append("  float f = 0.0f; g0 = 0.0f; g1 = 0.0f; g2 = 0.0f;")
        for cc in range(n2):
            L.append("  {")
            L.append("    float r = 0.0f, rx = 0.0f, ry = 0.0f;")
            for b in range(n1):
                e = "c[%d] * %s" % (cidx(0, b, cc), W(0, 0, 0))
                ed = "c[%d] * %s" % (cidx(0, b, cc), W(1, 0, 0))
                for a in range(1, n0):
                    e = "fmaf(c[%d], %s, %s)" % (cidx(a, b, cc), W(0, 0, a), e)
                    ed = "fmaf(c[%d], %s, %s)" % (cidx(a, b, cc), W(1, 0, a), ed)
                L.append("    { const float s = %s, sd = %s;" % (e, ed))
                L.append("      r = fmaf(s, %s, r); ry = fmaf(s, %s, ry); rx = fmaf(sd, %s, rx); }"
                         % (W(0, 1, b), W(1, 1, b), W(0, 1, b)))
            L.append("    f = fmaf(r, %s, f); g2 = fmaf(r, %s, g2);" % (W(0, 2, cc), W(1, 2, cc)))
            L.append("    g1 = fmaf(ry, %s, g1); g0 = fmaf(rx, %s, g0);" % (W(0, 2, cc), W(0, 2, cc)))
            L.append("  }")
        L.append("  return f;")
        L.append("}")
        L.append("")
        # value, gradient and Hessian: contractions with the 1D weights of
        # derivative orders (ox, oy, oz), ox + oy + oz <= 2
        L.append("__device__ __forceinline__ float %s_eval_hess_r0_pre(const float* __restrict__ c, const float* __restrict__ w," % nm)
        L.append("                                                    float& g0, float& g1, float& g2, float* __restrict__ h) {")
        orders = [(ox, oy, oz) for ox in range(3) for oy in range(3) for oz in range(3) if ox + oy + oz <= 2]
        pairs = sorted(set((ox, oy) for ox, oy, _ in orders))
        L.append("  float F[%d] = {};" % len(orders))
        for cc in range(n2):
            L.append("  {")
            L.append("    float r[%d] = {};" % len(pairs))
            for b in range(n1):
                sums = []
                for ox in range(3):
                    e = "c[%d] * %s" % (cidx(0, b, cc), W(ox, 0, 0))
                    for a in range(1, n0):
                        e = "fmaf(c[%d], %s, %s)" % (cidx(a, b, cc), W(ox, 0, a), e)
                    sums.append(e)
                L.append("    { const float s0 = %s, s1 = %s, s2 = %s;" % tuple(sums))
                for pi, (ox, oy) in enumerate(pairs):
                    L.append("      r[%d] = fmaf(s%d, %s, r[%d]);" % (pi, ox, W(oy, 1, b), pi))
                L.append("    }")
            for oi, (ox, oy, oz) in enumerate(orders):
                L.append("    F[%d] = fmaf(r[%d], %s, F[%d]);" % (oi, pairs.index((ox, oy)), W(oz, 2, cc), oi))
            L.append("  }")
        oid = {o: i for i, o in enumerate(orders)}
        L.append("  g0 = F[%d]; g1 = F[%d]; g2 = F[%d];" % (oid[(1, 0, 0)], oid[(0, 1, 0)], oid[(0, 0, 1)]))
        L.append("  h[0] = F[%d]; h[1] = F[%d]; h[2] = F[%d]; h[3] = F[%d]; h[4] = F[%d]; h[5] = F[%d];" % (
            oid[(2, 0, 0)], oid[(1, 1, 0)], oid[(1, 0, 1)], oid[(0, 2, 0)], oid[(0, 1, 1)], oid[(0, 0, 2)]))
        L.append("  return F[%d];" % oid[(0, 0, 0)])
        L.append("}")
        L.append("")
        # the same from y
        L.append("__device__ __forceinline__ float %s_eval_r0(const float* __restrict__ c, float y0, float y1, float y2) {" % nm)
        L.append("  float w[%d];" % (3 * N))
        L.append("  %s_pre<0>(y0, y1, y2, w);" % nm)
        L.append("  return %s_eval_r0_pre(c, w);" % nm)
        L.append("}")
        L.append("")
        L.append("__device__ __forceinline__ float %s_eval_grad_r0(const float* __restrict__ c, float y0, float y1, float y2," % nm)
        L.append("                                                float& g0, float& g1, float& g2) {")
        L.append("  float w[%d];" % (6 * N))
        L.append("  %s_pre<1>(y0, y1, y2, w);" % nm)
        L.append("  return %s_eval_grad_r0_pre(c, w, g0, g1, g2);" % nm)
        L.append("}")
        L.append("")
        L.append("__device__ __forceinline__ float %s_eval_hess_r0(const float* __restrict__ c, float y0, float y1, float y2," % nm)
        L.append("                                                float& g0, float& g1, float& g2, float* __restrict__ h) {")
        L.append("  float w[%d];" % (9 * N))
        L.append("  %s_pre<2>(y0, y1, y2, w);" % nm)
        L.append("  return %s_eval_hess_r0_pre(c, w, g0, g1, g2, h);" % nm)
        L.append("}")
        L.append("")
        # weights
        L.append("__device__ __forceinline__ void %s_weights_r0(float y0, float y1, float y2, float* __restrict__ w) {" % nm)
        L.append("  float wx[%d], wy[%d], wz[%d];" % (n0, n1, n2))
        L.append("  %s_w1d_0(y0, wx, nullptr); %s_w1d_1(y1, wy, nullptr); %s_w1d_2(y2, wz, nullptr);" % (nm, nm, nm))
        for cc in range(n2):
            for b in range(n1):
                L.append("  { const float t = wy[%d] * wz[%d];" % (b, cc))
                for a in range(n0):
                    L.append("    w[%d] = wx[%d] * t;" % (cidx(a, b, cc), a))
                L.append("  }")
        L.append("}")
        L.append("")
        return L


def _tree_json(t):
    if isinstance(t, int):
        return t
    n, thr, near, far = t
    return {"n": list(n), "t": str(F(thr)), "near": _tree_json(near), "far": _tree_json(far)}


def _tree_expr(t) -> str:
    """The region lookup as nested selects: far when n . y > t."""
    if isinstance(t, int):
        return str(t)
    n, thr, near, far = t
    terms = [("%s * y%d" % (flit(v), i)) for i, v in enumerate(n) if v]
    return "((%s > %s) ? %s : %s)" % (" + ".join(terms), flit(F(thr)), _tree_expr(far), _tree_expr(near))


def _emit_poly_struct_general(nm: str, nreg: int) -> List[str]:
    """Uniform entry points for three or more reference sub-regions: a branch
    per point (switch), or every polynomial and a select (PRED)."""
    def pick(expr_k, decl, ret):
        L = ["    if (PRED) {"]
        L += ["      " + decl(k) for k in range(nreg)]
        L += ["      " + ret, "    }", "    switch (region) {"]
        L += ["      case %d: %s" % (k, expr_k(k)) for k in range(1, nreg)]
        L += ["      default: %s" % expr_k(0), "    }"]
        return L
    L = ["// uniform entry points: the reference sub-region loop (Sec. 4.3)",
         "struct %s_poly {" % nm,
         "  template <bool PRED>",
         "  static __device__ __forceinline__ float value(const float* __restrict__ c, float y0, float y1, float y2, int region) {"]
    L += pick(lambda k: "return %s_eval_r%d(c, y0, y1, y2);" % (nm, k),
              lambda k: "const float v%d = %s_eval_r%d(c, y0, y1, y2);" % (k, nm, k),
              "float v = v0;" + "".join(" v = region == %d ? v%d : v;" % (k, k) for k in range(1, nreg)) + " return v;")
    L += ["  }", "  template <bool PRED>",
          "  static __device__ __forceinline__ float value_grad(const float* __restrict__ c, float y0, float y1, float y2, int region,",
          "                                                    float& g0, float& g1, float& g2) {"]
    L += pick(lambda k: "return %s_eval_grad_r%d(c, y0, y1, y2, g0, g1, g2);" % (nm, k),
              lambda k: "float a%d[3]; const float v%d = %s_eval_grad_r%d(c, y0, y1, y2, a%d[0], a%d[1], a%d[2]);" % (k, k, nm, k, k, k, k),
              "float v = v0; g0 = a0[0]; g1 = a0[1]; g2 = a0[2];" + "".join(
                  " if (region == %d) { v = v%d; g0 = a%d[0]; g1 = a%d[1]; g2 = a%d[2]; }" % (k, k, k, k, k)
                  for k in range(1, nreg)) + " return v;")
    L += ["  }", "  template <bool PRED>",
          "  static __device__ __forceinline__ float value_grad_hess(const float* __restrict__ c, float y0, float y1, float y2, int region,",
          "                                                         float& g0, float& g1, float& g2, float* __restrict__ h) {"]
    L += pick(lambda k: "return %s_eval_hess_r%d(c, y0, y1, y2, g0, g1, g2, h);" % (nm, k),
              lambda k: "float a%d[3], h%d[6]; const float v%d = %s_eval_hess_r%d(c, y0, y1, y2, a%d[0], a%d[1], a%d[2], h%d);"
              % (k, k, k, nm, k, k, k, k, k),
              "float v = v0; g0 = a0[0]; g1 = a0[1]; g2 = a0[2]; for (int i = 0; i < 6; ++i) h[i] = h0[i];" + "".join(
                  " if (region == %d) { v = v%d; g0 = a%d[0]; g1 = a%d[1]; g2 = a%d[2]; for (int i = 0; i < 6; ++i) h[i] = h%d[i]; }"
                  % (k, k, k, k, k, k) for k in range(1, nreg)) + " return v;")
    L += ["  }",
          "  static __device__ __forceinline__ void weights(float y0, float y1, float y2, int region, float* __restrict__ w) {",
          "    switch (region) {"]
    L += ["      case %d: %s_weights_r%d(y0, y1, y2, w); return;" % (k, nm, k) for k in range(1, nreg)]
    L += ["      default: %s_weights_r0(y0, y1, y2, w); return;" % nm, "    }", "  }", "};", ""]
    return L


def _emit_poly_struct_impl(nm: str, nreg: int) -> List[str]:
    """Uniform entry points over the reference sub-regions: the unrolled
    reference sub-region loop of Sec. 4.3, branchy or predicated."""
    L = ["// uniform entry points: the reference sub-region loop (Sec. 4.3)",
         "struct %s_poly {" % nm,
         "  template <bool PRED>",
         "  static __device__ __forceinline__ float value(const float* __restrict__ c, float y0, float y1, float y2, int region) {"]
    if nreg == 1:
        L += ["    (void)region;", "    return %s_eval_r0(c, y0, y1, y2);" % nm, "  }"]
    else:
        L += ["    if (PRED) {",
              "      const float v0 = %s_eval_r0(c, y0, y1, y2);" % nm,
              "      const float v1 = %s_eval_r1(c, y0, y1, y2);" % nm,
              "      return region ? v1 : v0;",
              "    }",
              "    if (region) return %s_eval_r1(c, y0, y1, y2);" % nm,
              "    return %s_eval_r0(c, y0, y1, y2);" % nm, "  }"]
    L += ["  template <bool PRED>",
          "  static __device__ __forceinline__ float value_grad(const float* __restrict__ c, float y0, float y1, float y2, int region,",
          "                                                    float& g0, float& g1, float& g2) {"]
    if nreg == 1:
        L += ["    (void)region;", "    return %s_eval_grad_r0(c, y0, y1, y2, g0, g1, g2);" % nm, "  }"]
    else:
        L += ["    if (PRED) {",
              "      float a0, a1, a2, b0, b1, b2;",
              "      const float v0 = %s_eval_grad_r0(c, y0, y1, y2, a0, a1, a2);" % nm,
              "      const float v1 = %s_eval_grad_r1(c, y0, y1, y2, b0, b1, b2);" % nm,
              "      g0 = region ? b0 : a0; g1 = region ? b1 : a1; g2 = region ? b2 : a2;",
              "      return region ? v1 : v0;",
              "    }",
              "    if (region) return %s_eval_grad_r1(c, y0, y1, y2, g0, g1, g2);" % nm,
              "    return %s_eval_grad_r0(c, y0, y1, y2, g0, g1, g2);" % nm, "  }"]
    L += ["  template <bool PRED>",
          "  static __device__ __forceinline__ float value_grad_hess(const float* __restrict__ c, float y0, float y1, float y2, int region,",
          "                                                         float& g0, float& g1, float& g2, float* __restrict__ h) {"]
    if nreg == 1:
        L += ["    (void)region;", "    return %s_eval_hess_r0(c, y0, y1, y2, g0, g1, g2, h);" % nm, "  }"]
    else:
        L += ["    if (PRED) {",
              "      float a0, a1, a2, b0, b1, b2, ha[6], hb[6];",
              "      const float v0 = %s_eval_hess_r0(c, y0, y1, y2, a0, a1, a2, ha);" % nm,
              "      const float v1 = %s_eval_hess_r1(c, y0, y1, y2, b0, b1, b2, hb);" % nm,
              "      g0 = region ? b0 : a0; g1 = region ? b1 : a1; g2 = region ? b2 : a2;",
              "      for (int i = 0; i < 6; ++i) h[i] = region ? hb[i] : ha[i];",
              "      return region ? v1 : v0;",
              "    }",
              "    if (region) return %s_eval_hess_r1(c, y0, y1, y2, g0, g1, g2, h);" % nm,
              "    return %s_eval_hess_r0(c, y0, y1, y2, g0, g1, g2, h);" % nm, "  }"]
    L += ["  static __device__ __forceinline__ void weights(float y0, float y1, float y2, int region, float* __restrict__ w) {"]
    if nreg == 1:
        L += ["    (void)region;", "    %s_weights_r0(y0, y1, y2, w);" % nm, "  }"]
    else:
        L += ["    if (region) %s_weights_r1(y0, y1, y2, w);" % nm,
              "    else %s_weights_r0(y0, y1, y2, w);" % nm, "  }"]
    L += ["};", ""]
    return L


def _emit_poly_struct_full(self) -> List[str]:
    nreg = len(self.regions)
    nm = self.spec.name
    L = (_emit_poly_struct_impl if nreg <= 2 else _emit_poly_struct_general)(nm, nreg)
    # the region lookup: which reference sub-region a transformed point is in
    L[L.index("};"):L.index("};")] = [
        "  static __host__ __device__ __forceinline__ int region(float y0, float y1, float y2) {",
        "    (void)y0; (void)y1; (void)y2;",
        "    return %s;" % _tree_expr(self.spec.lookup_tree()), "  }"]
    if self.tensor is None:
        pre = ["  static constexpr int kPre = 0;  // no y-only phase"]
    else:
        N = max(len(f) for f in self.tensor)
        pre = ["  // tensor product: the 1D weights (y alone) can be formed before the",
               "  // coefficients arrive; kPre floats hold derivative orders 0..2",
               "  static constexpr int kPre = %d;" % (9 * N),
               "  template <int DER>",
               "  static __device__ __forceinline__ void pre(float y0, float y1, float y2, float* __restrict__ w) {",
               "    %s_pre<DER>(y0, y1, y2, w);" % nm, "  }",
               "  static __device__ __forceinline__ float value_pre(const float* __restrict__ c, const float* __restrict__ w) {",
               "    return %s_eval_r0_pre(c, w);" % nm, "  }",
               "  static __device__ __forceinline__ float value_grad_pre(const float* __restrict__ c, const float* __restrict__ w,",
               "                                                        float& g0, float& g1, float& g2) {",
               "    return %s_eval_grad_r0_pre(c, w, g0, g1, g2);" % nm, "  }",
               "  static __device__ __forceinline__ float value_grad_hess_pre(const float* __restrict__ c, const float* __restrict__ w,",
               "                                                             float& g0, float& g1, float& g2, float* __restrict__ h) {",
               "    return %s_eval_hess_r0_pre(c, w, g0, g1, g2, h);" % nm, "  }"]
    end = L.index("};")
    return L[:end] + pre + L[end:]


SplineCode._emit_poly_struct = _emit_poly_struct_full


def emit_kind_map(names) -> str:
    L = ["// Generated by paper_2102_08518_amd.gen.emit: the spline kinds the library",
         "// was generated for, indexed by kind.  Do not edit.",
         "#pragma once", ""]
    for nm in names:
        L.append('#include "%s.h"' % nm)
    L += ["", "namespace lsp {", "namespace gen {", "",
          "constexpr int kNumKinds = %d;" % len(names), "",
          "template <int KIND> struct SplineOf;"]
    for nm in names:
        sp = SPECS[nm]
        L.append("template <> struct SplineOf<%d> { using T = %s_tables; using P = %s_poly; using M = %s_mfma; "
                 "static constexpr const char* kName = \"%s\"; };" % (sp.kind, nm, nm, nm, nm))
    L += ["", "}  // namespace gen", "}  // namespace lsp", ""]
    return "\n".join(L)


def generate(names=None, out_dir=OUT_DIR, verbose=True):
    os.makedirs(out_dir, exist_ok=True)
    names = names or list(SPECS)
    result = {}
    for nm in names:
        sc = SplineCode(SPECS[nm])
        code = sc.emit()
        tab = sc.tables()
        tab["fma"] = sc.fma_counts()
        with open(os.path.join(out_dir, "%s.h" % nm), "w") as fh:
            fh.write(code)
        with open(os.path.join(out_dir, "%s.json" % nm), "w") as fh:
            json.dump(tab, fh, indent=1, sort_keys=True)
        result[nm] = tab
        if verbose:
            print("%-12s taps %3d regions %d fma %s frames %s cond %s" % (
                nm, len(sc.union), len(sc.regions), tab["fma"],
                [[str(x) for x in f] for f in sc.frames], ["%.2f" % c for c in sc.cond]))
    if sorted(names) == sorted(SPECS):
        with open(os.path.join(out_dir, "all.h"), "w") as fh:
            fh.write(emit_kind_map(list(SPECS)))
    return result
