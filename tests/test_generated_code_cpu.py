"""The generated device code itself, compiled for the host with g++ (the
device qualifiers defined away): value, gradient, Hessian and per-tap weights of every
spline's reference polynomials, in FP32 as on the GPU, against the exact
rational tables the generator derived (the tables are pinned to the oracle
by tests/test_generator.py).  This covers the emitted straight-line code,
including the shared-term form of the linear map from fetched values to
monomial coefficients, without a GPU.

Tolerance: the code evaluates in FP32 a polynomial whose coefficient-weighted
condition number the generator keeps below 6.5, so |f_fp32 - f_exact| stays
within a few units of 2^-24 * sum_j |c_j| |w_j|-scale terms; 2e-6 * max|c| for
values and weights, 2e-5 * max|c| for gradients (as the GPU tests) and
2e-4 * max|c| for second derivatives (one more differentiation of the same
monomial coefficients, with factors up to degree * (degree - 1))."""
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from paper_2102_08518_amd.gen import interp
from paper_2102_08518_amd.gen.emit import OUT_DIR

NAMES = ["tricubic", "bcc8", "fcc6", "trilinear", "bcc4", "triquadratic", "cc7", "bcc7", "cc6"]

HARNESS = r"""
#include <cmath>
#include <cstdio>
#define __device__
#define __host__
#define __forceinline__ inline
#define __restrict__
#include "%(name)s.h"
using namespace lsp::gen;
int main() {
  int n, taps;
  if (scanf("%%d %%d", &n, &taps) != 2) return 1;
  for (int i = 0; i < n; ++i) {
    float y[3]; int region; float c[64];
    scanf("%%f %%f %%f %%d", &y[0], &y[1], &y[2], &region);
    for (int j = 0; j < taps; ++j) scanf("%%f", &c[j]);
    float g[3], w[64], gh[3], h[6];
    const float f = %(name)s_poly::value<false>(c, y[0], y[1], y[2], region);
    const float fh = %(name)s_poly::value_grad_hess<false>(c, y[0], y[1], y[2], region, gh[0], gh[1], gh[2], h);
    const float f2 = %(name)s_poly::value_grad<false>(c, y[0], y[1], y[2], region, g[0], g[1], g[2]);
    const float fp = %(name)s_poly::value<true>(c, y[0], y[1], y[2], region);
    %(name)s_poly::weights(y[0], y[1], y[2], region, w);
    printf("%%.9g %%.9g %%.9g %%.9g %%.9g %%.9g", f, f2, fp, g[0], g[1], g[2]);
    printf(" %%.9g %%.9g %%.9g %%.9g", fh, gh[0], gh[1], gh[2]);
    for (int k = 0; k < 6; ++k) printf(" %%.9g", h[k]);
    for (int j = 0; j < taps; ++j) printf(" %%.9g", w[j]);
    printf("\n");
  }
  return 0;
}
"""


def _poly_terms(w):
    return [(tuple(int(v) for v in k.split(",")), Fraction(c)) for k, c in w.items()]


def _eval(terms, u):
    """value, gradient and Hessian (00, 01, 02, 11, 12, 22) of sum c u^e."""
    f = 0.0
    g = np.zeros(3)
    h = np.zeros(6)
    pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for e, c in terms:
        c = float(c)
        f += c * u[0] ** e[0] * u[1] ** e[1] * u[2] ** e[2]
        for r in range(3):
            if e[r]:
                ee = list(e)
                ee[r] -= 1
                g[r] += c * e[r] * u[0] ** ee[0] * u[1] ** ee[1] * u[2] ** ee[2]
        for k, (r, q) in enumerate(pairs):
            ee = list(e)
            k1 = ee[r]
            ee[r] -= 1
            k2 = ee[q]
            ee[q] -= 1
            if k1 > 0 and k2 > 0:
                h[k] += c * k1 * k2 * u[0] ** ee[0] * u[1] ** ee[1] * u[2] ** ee[2]
    return f, g, h


@pytest.fixture(scope="module")
def gxx():
    exe = shutil.which("g++")
    if exe is None:
        pytest.skip("no g++")
    return exe


@pytest.mark.parametrize("name", NAMES)
def test_generated_code_matches_exact_tables(gxx, tmp_path, name):
    tab = interp.load_tables(name)
    src = tmp_path / "h.cpp"
    src.write_text(HARNESS % {"name": name})
    exe = tmp_path / "h"
    subprocess.run([gxx, "-std=c++17", "-O1", "-ffp-contract=off", "-I", OUT_DIR, str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    rng = np.random.default_rng(len(name))
    ntap = len(tab["union"])
    x = rng.uniform(3, 9, (300, 3))
    K, y, G, region = interp.locate(tab, x)
    c = rng.uniform(-1, 1, (x.shape[0], ntap)).astype(np.float32)
    y32 = y.astype(np.float32)
    lines = ["%d %d" % (x.shape[0], ntap)]
    for i in range(x.shape[0]):
        lines.append("%.9g %.9g %.9g %d " % (y32[i, 0], y32[i, 1], y32[i, 2], region[i]) +
                     " ".join("%.9g" % v for v in c[i]))
    out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    regs = [([_poly_terms(w) for w in r["weights"]], r["union_index"],
             np.array([float(Fraction(v)) for v in r["frame"]])) for r in tab["regions"]]
    for i in range(x.shape[0]):
        vals = np.array([float(v) for v in out[i].split()])
        f, f2, fp, gx = vals[0], vals[1], vals[2], vals[3:6]
        fh, gh, hh, wts = vals[6], vals[7:10], vals[10:16], vals[16:]
        polys, uidx, frame = regs[region[i]]
        u = y32[i].astype(np.float64) - frame
        fe, ge, he = 0.0, np.zeros(3), np.zeros(6)
        we = np.zeros(ntap)
        for terms, j in zip(polys, uidx):
            wj, gj, hj = _eval(terms, u)
            we[j] = wj
            fe += float(c[i, j]) * wj
            ge += float(c[i, j]) * gj
            he += float(c[i, j]) * hj
        assert abs(f - fe) <= 2e-6, (name, i, f, fe)
        assert abs(f2 - fe) <= 2e-6 and abs(fp - fe) <= 2e-6
        assert np.abs(gx - ge).max() <= 2e-5, (name, i, gx, ge)
        assert np.abs(wts - we).max() <= 2e-6, (name, i)
        assert abs(fh - fe) <= 2e-6 and np.abs(gh - ge).max() <= 2e-5
        assert np.abs(hh - he).max() <= 2e-4, (name, i, hh, he)
