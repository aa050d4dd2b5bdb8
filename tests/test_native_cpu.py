"""Host-side checks of the C ABI (no GPU): the library loads and exports every
declared symbol, recognises (L, Xi) pairs up to a change of lattice basis and
direction order/sign, rejects bad arguments with status codes, and -- through
the host diagnostics -- every coefficient fetch of the location step lands on
the lattice site the stencil prescribes and inside the internal buffer."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2102_08518_amd import _native as N
from paper_2102_08518_amd import api
from paper_2102_08518_amd.gen import interp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "lsp.h")) as fh:
        hdr = fh.read()
    declared = set(re.findall(r"^[a-z_ *]*?\b(lsp_[a-z_]+)\(", hdr, flags=re.M))
    assert declared == set(N.EXPORTS)
    lib = N.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.lsp_version().decode().startswith("lsp")
    for st in range(8):
        assert lib.lsp_status_string(st)


# continuity: cubic B-spline C^2, quintic BCC 8-direction box spline C^2,
# FCC 6-direction box spline C^1, quadratic B-spline C^1, linear ones C^0,
# the 7-direction ones C^2 (no plane holds more than 3 of their directions)
@pytest.mark.parametrize("name,kind,cosets,taps,union,cont", [
    ("tricubic", 0, 1, 64, 64, 2), ("bcc8", 1, 2, 32, 32, 2), ("fcc6", 2, 4, 16, 19, 1),
    ("trilinear", 3, 1, 8, 8, 0), ("bcc4", 4, 2, 4, 4, 0), ("triquadratic", 5, 1, 27, 27, 1),
    ("cc7", 6, 1, 53, 53, 2), ("bcc7", 7, 2, 30, 30, 2), ("cc6", 8, 1, 32, 38, 1)])
def test_spline_recognition(name, kind, cosets, taps, union, cont):
    sp = getattr(api.Spline, name)()
    assert sp.info.kind == kind and sp.info.n_cosets == cosets
    assert sp.info.taps == taps and sp.info.union_taps == union
    assert sp.continuity == cont
    # another basis of the same lattice, directions shuffled and negated
    L = api.LATTICES[api.LATTICE_OF[name]]
    U = np.array([[1, 1, 0], [0, 1, 0], [0, 0, 1]], dtype=np.int32)  # unimodular
    Xi = api.DIRECTIONS[name].copy()
    rng = np.random.default_rng(3)
    Xi = Xi[:, rng.permutation(Xi.shape[1])] * rng.choice([-1, 1], Xi.shape[1])
    sp2 = api.Spline(L @ U, Xi)
    assert sp2.info.kind == kind


def test_unsupported_and_invalid_arguments():
    with pytest.raises(N.LspError) as e:
        api.Spline(np.eye(3) * 2, api.DIRECTIONS["tricubic"])   # 2Z^3 is another lattice
    assert e.value.status == 2
    with pytest.raises(N.LspError) as e:
        api.Spline(api.LATTICES["fcc"], api.DIRECTIONS["bcc4"])  # no code for this pair
    assert e.value.status == 2
    with pytest.raises(N.LspError) as e:
        api.Spline(np.zeros((3, 3)), api.DIRECTIONS["tricubic"])
    assert e.value.status == 1
    lib = N.lib()
    h = ctypes.c_void_p()
    L = np.eye(3, dtype=np.int32)
    assert lib.lsp_spline_create(2, L.ctypes.data_as(N.i32p), L.ctypes.data_as(N.i32p), 3,
                                 ctypes.byref(h)) == 2
    assert lib.lsp_spline_create(3, None, None, 3, ctypes.byref(h)) == 1
    assert lib.lsp_eval(None, None, 0, 0, None, None) == 1
    sp = api.Spline.bcc8()
    with pytest.raises(N.LspError) as e:
        sp.debug_geometry((0, 4, 4))
    assert e.value.status == 4
    with pytest.raises(N.LspError) as e:
        sp.debug_geometry((2000, 2000, 2000))
    assert e.value.status == 4
    assert lib.lsp_set_option(N.LSP_OPT_MFMA, 3) == 1
    assert lib.lsp_set_option(999, 0) == 1
    assert lib.lsp_set_option(N.LSP_OPT_MFMA, 2) == 0
    assert lib.lsp_set_option(N.LSP_OPT_PREDICATED, 2) == 1
    assert lib.lsp_set_option(N.LSP_OPT_PREDICATED, 1) == 0
    # back to the defaults for whatever runs next in this process
    assert lib.lsp_set_option(N.LSP_OPT_MFMA, 0) == 0
    assert lib.lsp_set_option(N.LSP_OPT_PREDICATED, 0) == 0
    assert lib.lsp_set_option(N.LSP_OPT_SPLIT_MAXN, -2) == 1
    assert lib.lsp_set_option(N.LSP_OPT_SPLIT_MAXN, -1) == 0


def _site_offset(tab, geo, n):
    """Byte offset of lattice site n in the internal layout (interleaved
    cosets, bricks of 2^lb sites per axis, zero halo)."""
    D = np.array(tab["D"])
    for m, sh in enumerate(tab["shifts"]):
        if np.all((n - np.array(sh)) % D == 0):
            i = [int(v) for v in (n - np.array(sh)) // D + geo["pad"]]
            off = m * geo["es"]
            for a in range(3):
                lb = geo["lb"][a]
                off += (i[a] >> lb) * geo["bs"][a] + (i[a] & ((1 << lb) - 1)) * geo["is_"][a]
            return off
    raise AssertionError("not a lattice site")


@pytest.mark.parametrize("name", ["tricubic", "bcc8", "fcc6", "trilinear", "bcc4", "triquadratic",
                                  "cc7", "bcc7", "cc6"])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_tap_offsets_hit_the_prescribed_sites_inside_the_buffer(name, storage):
    sp = api.Spline.named(name)
    tab = interp.load_tables(name)
    rng = np.random.default_rng(11)
    dims = (7, 5, 6)
    geo = sp.debug_geometry(dims, storage)
    D = tab["D"][0]
    hi = np.array([D * (d - 1) + 1 for d in dims], dtype=np.float64)
    x = rng.uniform(-7, hi.max() + 7, (6000, 3))
    # points at and around the edges of the active range, and far away
    lo_k = np.array(geo["kmin"])
    hi_k = np.array(geo["kmax"])
    edge = np.concatenate([lo_k + rng.uniform(-1.6, 1.6, (1500, 3)),
                           hi_k + rng.uniform(-1.6, 1.6, (1500, 3))])
    x = np.concatenate([x, edge, [[1e30, 0, 0], [-1e30, 3, 3], [np.inf, 1, 1], [np.nan, 2, 2]]])
    x = x.astype(np.float32).astype(np.float64)
    offs, flags = sp.debug_tap_offsets(dims, x, storage)
    es = geo["es"]
    assert offs.min() >= 0 and offs.max() <= geo["nbytes"] - es  # every fetch in bounds
    active = (flags & 1) == 1
    assert flags[-1] & 2 and not active[-4:].any()
    K, y, G, region = interp.locate(tab, x[active])
    union = np.array(tab["union"])
    sites = K[:, None, :] + np.einsum("nji,tj->nti", G, union)  # K + G^T o
    got = offs[active]
    for i in range(0, sites.shape[0], 7):
        for t in range(union.shape[0]):
            assert got[i, t] == _site_offset(tab, geo, sites[i, t]), (x[active][i], t)
    np.testing.assert_array_equal((flags[active] >> 2), region)
    # a point is active iff some tap of its stencil lies in the stored range
    fin = np.all(np.isfinite(x), axis=1) & (np.abs(x).max(axis=1) < 1e6)
    Kall, _, Gall, _ = interp.locate(tab, x[fin])
    shifts = np.array(tab["shifts"])
    for i in range(0, Kall.shape[0], 5):
        st = Kall[i][None, :] + union @ Gall[i]          # (taps, 3): K + G^T o
        reach = False
        for n in st:
            for sh in shifts:
                if np.all((n - sh) % D == 0):
                    idx = (n - sh) // D
                    reach |= bool(np.all((idx >= 0) & (idx < np.array(dims))))
        assert not reach or active[fin][i], x[fin][i]
