"""Run-time specialisation on the host: a spline given only by (lattice, Xi)
is analysed, generated and compiled into a plugin (paper_2102_08518_amd.jit),
and the library loads it.  The example plugin (the piecewise-linear spline on
the Freudenthal triangulation, Xi = [I, (1,1,1)]) is the one build() makes."""
import numpy as np
import pytest

import oracle
from paper_2102_08518_amd import _native as N
from paper_2102_08518_amd import api, jit
from paper_2102_08518_amd.gen import interp
from paper_2102_08518_amd.gen.auto import auto_spec
from paper_2102_08518_amd.gen.emit import SplineCode

FREUDENTHAL = oracle.Spline("freudenthal", np.eye(3), oracle._cols((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)),
                            D=(1, 1, 1), shifts=[(0, 0, 0)])


def test_generated_tables_of_an_unlisted_spline_match_the_oracle():
    """The automatic analysis cuts the unit cube into the six tetrahedra of
    the Freudenthal triangulation; the generated tables, walked by the CPU
    interpreter of the device algorithm, equal the FP64 convolution sum."""
    spec = auto_spec("freudenthal", *jit.EXAMPLE)
    assert (spec.roe, spec.symmetry, len(spec.regions)) == ("floor", "none", 6)
    tab = SplineCode(spec).tables()
    E = 7
    rng = np.random.default_rng(3)
    c = rng.uniform(-1, 1, (1, E, E, E))
    x = rng.uniform(-1, E, (3000, 3))
    f = interp.evaluate(tab, (E, E, E), list(c), x)
    ref = oracle.evaluate(FREUDENTHAL, (E, E, E), list(c), x)
    np.testing.assert_allclose(f, ref, atol=1e-12)
    # linear interpolation: exact on the lattice, linear on each tetrahedron
    sites = rng.integers(0, E, (50, 3)).astype(np.float64)
    np.testing.assert_allclose(interp.evaluate(tab, (E, E, E), list(c), sites),
                               c[0][sites[:, 2].astype(int), sites[:, 1].astype(int), sites[:, 0].astype(int)],
                               atol=1e-12)


def test_library_loads_the_compiled_plugin():
    path = jit.build_example(force=False)
    sp = api.Spline.from_plugin(path)
    i = sp.info
    assert (i.kind, i.taps, i.union_taps, i.n_reference, i.degree) == (jit.PLUGIN_KIND, 4, 8, 6, 1)
    assert sp.continuity == 0 and i.n_cosets == 1
    assert api.Spline.from_plugin(path).info.n_reference == 6      # loading twice is fine
    assert jit.spline_name(*jit.EXAMPLE) == jit.spline_name("cc", [(0, 0, -1), (1, 1, 1), (0, 1, 0), (-1, 0, 0)])


def test_plugin_refusals():
    with pytest.raises(N.LspError) as e:
        api.Spline.from_plugin("/nonexistent/plugin.so")
    assert e.value.status == 2
    with pytest.raises(N.LspError) as e:       # a library without the plugin entry points
        api.Spline.from_plugin(N.LIB_PATH)
    assert e.value.status == 2
    with pytest.raises(ValueError):            # BCC point location needs the full symmetry
        auto_spec("odd", "bcc", [(1, 1, 1), (1, -1, -1), (2, 0, 0)])


def test_bcc_plugin_describes_the_builtin_spline():
    """The BCC quartic compiled as a plugin describes the same spline as the
    built-in one (kind aside)."""
    a = api.Spline.from_plugin(jit.build_example(force=False, name="jit_bcc7")).info
    b = api.Spline.bcc7().info
    fields = ("n_cosets", "taps", "union_taps", "n_reference", "degree", "radius", "fma_eval", "pad", "continuity")
    assert [getattr(a, f) for f in fields] == [getattr(b, f) for f in fields]
    assert list(a.D) == list(b.D) and a.kind == jit.PLUGIN_KIND
