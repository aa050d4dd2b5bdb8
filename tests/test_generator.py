"""The sub-region generator: structural counts, the paper's worked example
reproduced exactly, and the emitted tables checked against the oracle through
a CPU interpreter of the device algorithm."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2102_08518_amd.gen import interp
from paper_2102_08518_amd.gen.derive import BoxSpline, derive_region
from paper_2102_08518_amd.gen.emit import SplineCode
from paper_2102_08518_amd.gen.specs import SPECS, Region, Spec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(77)
ORACLE_SPLINE = {"tricubic": oracle.TRICUBIC, "bcc8": oracle.BCC8, "fcc6": oracle.FCC6,
                 "trilinear": oracle.TRILINEAR, "bcc4": oracle.BCC4,
                 "triquadratic": oracle.TRIQUADRATIC, "cc7": oracle.CC7, "bcc7": oracle.BCC7,
                 "cc6": oracle.CC6}
ALL = list(ORACLE_SPLINE)


def test_generator_reproduces_fig1_zp_polynomial_exactly():
    """Fig. 1: one reference sub-region {x0 >= |x1|} of the ROE [-1/2,1/2]^2 with
    seven taps; its polynomial equals the printed one coefficient by coefficient."""
    zp = Spec(name="zp", s=2, L=[[1, 0], [0, 1]], Xi=[(1, 0), (0, 1), (1, 1), (1, -1)],
              D=(1, 1), shifts=[(0, 0)], roe="voronoi", symmetry="rot90",
              regions=[Region("sub1", [((1, -1), 0), ((1, 1), 0), ((-1, 0), Fraction(1, 2))],
                              (Fraction(3, 10), Fraction(1, 20)))])
    bs = BoxSpline(2, zp.Xi, 1)
    d = derive_region(zp, bs, zp.regions[0])
    with open(os.path.join(GOLDEN, "zp_fig1.json")) as fh:
        g = json.load(fh)
    assert len(d.taps) == 7
    assert sorted(d.taps) == sorted(tuple(o) for o in g["offsets"])
    for o, row in zip(g["offsets"], g["weights"]):
        p = d.polys[d.taps.index(tuple(o))]
        expect = {tuple(e): Fraction(c) for e, c in zip(g["monomials"], row) if Fraction(c) != 0}
        assert p.t == expect, (o, p)


@pytest.mark.parametrize("name,taps,regions", [("tricubic", 64, 1), ("bcc8", 32, 1), ("fcc6", 16, 2),
                                               ("trilinear", 8, 1), ("bcc4", 4, 1),
                                               ("triquadratic", 27, 1), ("cc7", 53, 1), ("bcc7", 30, 1),
                                               ("cc6", 32, 3)])
def test_stencil_sizes(name, taps, regions):
    """Tricubic: 64 fetches (Sec. 5.1); the FCC cubic spline has two reference
    sub-regions (Sec. 5.1); every stencil has vol(supp)/|det L| sites."""
    tab = interp.load_tables(name)
    assert len(tab["regions"]) == regions
    for reg in tab["regions"]:
        assert len(reg["taps"]) == taps


@pytest.mark.parametrize("name", ALL)
def test_weights_sum_to_one_exactly(name):
    tab = interp.load_tables(name)
    for reg in tab["regions"]:
        tot = {}
        for w in reg["weights"]:
            for k, v in w.items():
                tot[k] = tot.get(k, Fraction(0)) + Fraction(v)
        tot = {k: v for k, v in tot.items() if v != 0}
        assert tot == {"0,0,0": Fraction(1)}


@pytest.mark.parametrize("name", ALL)
def test_interpreter_matches_oracle(name):
    sp = ORACLE_SPLINE[name]
    tab = interp.load_tables(name)
    E = 9
    dims = (E, E, E)
    coeffs = [rng.uniform(-1, 1, (E, E, E)) for _ in range(sp.n_cosets)]
    hi = (E - 1) * sp.D[0]
    x = rng.uniform(-1.5, hi + 1.5, (2500, 3))  # interior, boundary and outside
    a = interp.evaluate(tab, dims, coeffs, x)
    b = oracle.evaluate(sp, dims, coeffs, x)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


def test_interpreter_on_region_boundaries():
    """Points on the sub-region boundaries (ties of the location step)."""
    sp = oracle.BCC8
    tab = interp.load_tables("bcc8")
    E = 8
    coeffs = [rng.uniform(-1, 1, (E, E, E)) for _ in range(2)]
    base = rng.uniform(5, 9, (300, 3))
    base[:100, 1] = base[:100, 0]            # |d_x| == |d_y| ties
    base[100:200] = np.round(base[100:200])  # lattice and half-lattice points
    base[200:, 2] = np.round(base[200:, 2] * 2) / 2
    a = interp.evaluate(tab, (E,) * 3, coeffs, base)
    b = oracle.evaluate(sp, (E,) * 3, coeffs, base)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


@pytest.mark.slow
def test_committed_headers_are_current(tmp_path):
    from paper_2102_08518_amd.gen.emit import OUT_DIR, generate
    generate(out_dir=str(tmp_path), verbose=False)
    for nm in SPECS:
        for ext in (".h", ".json"):
            with open(os.path.join(OUT_DIR, nm + ext)) as a, open(os.path.join(tmp_path, nm + ext)) as b:
                assert a.read() == b.read(), nm + ext


@pytest.mark.parametrize("name", ALL)
def test_transposed_stencil_tables(name):
    """Every tap j of a located point reaches the site K + G^T o_j, and the
    transposed table maps (G, K + G^T o_j - K) back to exactly that j."""
    tab = interp.load_tables(name)
    U = [tuple(v) for v in tab["transposed"]["U"]]
    J = tab["transposed"]["J"]
    union = np.array(tab["union"])
    uidx = {v: i for i, v in enumerate(U)}
    x = rng.uniform(5, 12, (400, 3))
    K, y, G, region = interp.locate(tab, x)
    for i in range(x.shape[0]):
        Gi = G[i]
        if tab["symmetry"] == "none":
            sid = 0
        else:
            # reference axis r -> global axis a with G[r, a] = +-1
            ax = [int(np.nonzero(Gi[r])[0][0]) for r in range(3)]
            bits = sum(1 << r for r in range(3) if Gi[r, ax[r]] < 0)
            sid = bits if tab["symmetry"] == "signs" else (ax[0] * 3 + ax[1]) * 8 + bits
        for j, o in enumerate(union):
            v = tuple(int(round(t)) for t in Gi.T @ o)
            assert J[sid][uidx[v]] == j
    # a symmetry element maps distinct taps to distinct offsets (ids that
    # encode no group element have empty rows)
    n_el = 0
    for row in J:
        hit = [j for j in row if j >= 0]
        if hit:
            n_el += 1
            assert sorted(hit) == list(range(len(union)))
    assert n_el == {"none": 1, "signs": 8, "signed_perm": 48}[tab["symmetry"]]


@pytest.mark.parametrize("name", [n for n in ALL if interp.load_tables(n)["mfma"] is not None])
def test_matrix_core_form_is_exact(name):
    """The integer weight matrix of the matrix-core path: Wq[m][j] / Q equals
    the exact rational coefficient of monomial m in tap j's weight polynomial
    (zero where the tap is not in the sub-region), and every entry has at
    most 8 significant bits, so it is exact in bf16 and fp16."""
    tab = interp.load_tables(name)
    mf = tab["mfma"]
    Q, Wq, mons = mf["Q"], mf["Wq"], [tuple(e) for e in mf["monomials"]]
    assert len(mons) == mf["rows"] <= 64 and len(tab["union"]) <= 32
    reg = tab["regions"][0]
    expect = [[Fraction(0)] * 32 for _ in range(64)]
    for w, j in zip(reg["weights"], reg["union_index"]):
        for key, c in w.items():
            e = tuple(int(v) for v in key.split(","))
            expect[mons.index(e)][j] = Fraction(c)
    for m in range(64):
        for j in range(32):
            assert Fraction(Wq[m][j], Q) == expect[m][j], (m, j)
            v = abs(Wq[m][j])
            while v and v % 2 == 0:
                v //= 2
            assert v.bit_length() <= 8
            assert float(np.float32(Wq[m][j]).view(np.uint32) & 0xFFFF0000) == float(
                np.float32(Wq[m][j]).view(np.uint32)), "not exact in bf16"



@pytest.mark.parametrize("name", [n for n in ALL if n != "cc6"])
def test_automatic_regions_reproduce_the_written_specs(name):
    """The ROE, symmetry and reference sub-regions found from (L, Xi) alone
    (gen/auto.py) give the same sub-region polynomials as the specs written
    out from the analysis, and the same region lookup."""
    from paper_2102_08518_amd.gen.auto import auto_spec
    from paper_2102_08518_amd.gen.derive import BoxSpline, derive_region
    hand = SPECS[name]
    auto = auto_spec(name, hand.lattice, hand.Xi)
    assert (auto.roe, auto.symmetry, len(auto.regions)) == (hand.roe, hand.symmetry, len(hand.regions))

    def pieces(spec):
        bs = BoxSpline(3, spec.Xi, spec.det_L)
        out = set()
        for reg in spec.regions:
            d = derive_region(spec, bs, reg)
            out.add(frozenset((o, tuple(sorted(p.t.items()))) for o, p in zip(d.taps, d.polys)))
        return out
    assert pieces(auto) == pieces(hand)
    # the lookup puts the written regions' interior points where they belong
    if len(hand.regions) > 1:
        from paper_2102_08518_amd.gen.emit import _tree_json
        tab = {"tree": _tree_json(auto.lookup_tree())}
        ys = np.array([[float(v) for v in r.interior] for r in hand.regions])
        got = interp._lookup(tab["tree"], ys)
        a_pieces = []
        bs = BoxSpline(3, auto.Xi, auto.det_L)
        for reg in auto.regions:
            d = derive_region(auto, bs, reg)
            a_pieces.append(frozenset((o, tuple(sorted(p.t.items()))) for o, p in zip(d.taps, d.polys)))
        bsh = BoxSpline(3, hand.Xi, hand.det_L)
        for k, reg in enumerate(hand.regions):
            d = derive_region(hand, bsh, reg)
            assert a_pieces[got[k]] == frozenset((o, tuple(sorted(p.t.items()))) for o, p in zip(d.taps, d.polys))


def test_automatic_three_region_spline_lookup_is_consistent():
    """cc6 (the face diagonals on Z^3) has three reference sub-regions from
    the automatic analysis: every derived region's interior point is looked
    up into that region, and random points of the wedge land in a region
    whose half-spaces contain them."""
    tab = interp.load_tables("cc6")
    spec = SPECS["cc6"]
    assert len(tab["regions"]) == 3
    ys = np.array([[float(v) for v in r.interior] for r in spec.regions])
    assert list(interp._lookup(tab["tree"], ys)) == [0, 1, 2]
    y = rng.uniform(0, 0.5, (4000, 3))
    y = -np.sort(-y, axis=1)          # the wedge 0 <= y2 <= y1 <= y0 <= 1/2
    reg = interp._lookup(tab["tree"], y)
    for k, r in enumerate(spec.regions):
        sel = y[reg == k]
        for a, b in r.halfspaces:
            assert np.all(sel @ np.array(a, dtype=np.float64) + float(Fraction(b)) >= -1e-12)
