"""FP64 CPU oracle for the lattice convolution sum -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product path (the HIP
library and its Python binding) never imports it and shares no code with it.

The arithmetic lives in ``box_oracle.c`` (plain C, FP64, OpenMP): the naive
convolution sum of Sec. 1 (Eq. 1) with phi evaluated by the box-spline
recurrence on the direction matrix.  This module only marshals arguments and
holds the oracle's own description of the splines and lattices used in the
paper's box-spline experiments (Sec. 5.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "box_oracle.c")
_LIB = os.path.join(_HERE, "libbox_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i32p = ctypes.POINTER(ctypes.c_int32)
            i64p = ctypes.POINTER(ctypes.c_int64)
            f64p = ctypes.POINTER(ctypes.c_double)
            lib.orc_phi.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int64,
                                    f64p, f64p, f64p]
            lib.orc_eval.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int, i32p,
                                     i32p, i64p, f64p, ctypes.c_int64, f64p, f64p, f64p,
                                     ctypes.c_int]
            lib.orc_backward_coef.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p,
                                              ctypes.c_int, i32p, i32p, i64p, ctypes.c_int64,
                                              f64p, f64p, f64p]
            lib.orc_num_threads.argtypes = []
            lib.orc_eval_hess.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int, i32p,
                                          i32p, i64p, f64p, ctypes.c_int64, f64p, f64p, f64p, f64p]
            for f in (lib.orc_phi, lib.orc_eval, lib.orc_eval_hess, lib.orc_backward_coef,
                      lib.orc_num_threads):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ---------------------------------------------------------------- splines
# Direction matrices: rows are coordinates, columns are directions.

class Spline:
    """A box spline on a lattice, with the lattice stored as Cartesian cosets.

    Coset m holds the sites n = D * idx + shift[m]; idx in C order [z][y][x].
    """

    def __init__(self, name, L, Xi, D, shifts):
        self.name = name
        self.L = np.ascontiguousarray(np.asarray(L, dtype=np.int32))
        self.Xi = np.ascontiguousarray(np.asarray(Xi, dtype=np.int32))
        self.s = self.L.shape[0]
        self.D = np.asarray(D, dtype=np.int32)
        self.shifts = np.ascontiguousarray(np.asarray(shifts, dtype=np.int32).reshape(-1, self.s))
        self.n_cosets = self.shifts.shape[0]

    @property
    def halfwidth(self):
        return 0.5 * np.abs(self.Xi).sum(axis=1)

    @property
    def det_L(self):
        return abs(round(np.linalg.det(self.L.astype(np.float64))))


def _cols(*vecs):
    return np.array(vecs, dtype=np.int32).T


# Tensor-product cubic B-spline on Z^3: each axis direction four times.
TRICUBIC = Spline("tricubic", np.eye(3), _cols(*([(1, 0, 0)] * 4 + [(0, 1, 0)] * 4 + [(0, 0, 1)] * 4)),
                  D=(1, 1, 1), shifts=[(0, 0, 0)])
# BCC lattice from the generating matrix rows [-1,1,1],[1,-1,1],[1,1,-1]; the
# four diagonals each taken twice.
_BCC_L = [[-1, 1, 1], [1, -1, 1], [1, 1, -1]]
_DIAG = [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]
BCC8 = Spline("bcc8", _BCC_L, _cols(*(_DIAG + _DIAG)), D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 1)])
# Linear rhombic-dodecahedron box spline (four diagonals once).
BCC4 = Spline("bcc4", _BCC_L, _cols(*_DIAG), D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 1)])
# FCC lattice D3 = {n : sum(n) even} with the six (1,+-1,0)-type directions.
FCC6 = Spline("fcc6", [[0, 1, 1], [1, 0, 1], [1, 1, 0]],
              _cols((1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)),
              D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)])
# The ZP element on Z^2 (the worked example of Fig. 1).
ZP = Spline("zp", np.eye(2), _cols((1, 0), (0, 1), (1, 1), (1, -1)), D=(1, 1), shifts=[(0, 0)])
# Tensor-product linear (trilinear) B-spline on Z^3.
TRILINEAR = Spline("trilinear", np.eye(3), _cols(*([(1, 0, 0)] * 2 + [(0, 1, 0)] * 2 + [(0, 0, 1)] * 2)),
                   D=(1, 1, 1), shifts=[(0, 0, 0)])

# Tensor-product quadratic B-spline on Z^3: each axis direction three times.
TRIQUADRATIC = Spline("triquadratic", np.eye(3),
                      _cols(*([(1, 0, 0)] * 3 + [(0, 1, 0)] * 3 + [(0, 0, 1)] * 3)),
                      D=(1, 1, 1), shifts=[(0, 0, 0)])

# Fourth-order splines of the paper's third comparison (Sec. 5.1): the
# seven-direction box spline on Z^3 (the axes and the four diagonals) and the
# quartic box spline on BCC (the four diagonals and the three shortest
# axis-aligned lattice vectors 2 e_i).
CC7 = Spline("cc7", np.eye(3), _cols((1, 0, 0), (0, 1, 0), (0, 0, 1), *_DIAG),
             D=(1, 1, 1), shifts=[(0, 0, 0)])
BCC7 = Spline("bcc7", _BCC_L, _cols(*_DIAG, (2, 0, 0), (0, 2, 0), (0, 0, 2)),
              D=(2, 2, 2), shifts=[(0, 0, 0), (1, 1, 1)])

# The six face diagonals on Z^3.
CC6 = Spline("cc6", np.eye(3), _cols((1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)),
             D=(1, 1, 1), shifts=[(0, 0, 0)])

SPLINES = {sp.name: sp for sp in (TRICUBIC, BCC8, BCC4, FCC6, ZP, TRILINEAR, TRIQUADRATIC, CC7, BCC7, CC6)}


# ---------------------------------------------------------------- calls

def phi(spline: Spline, y, grad: bool = False):
    """phi(y) = |det L| M_Xi(y + Xi 1/2) at points y (..., s)."""
    lib = _load()
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(-1, spline.s))
    out = np.empty(y.shape[0])
    g = np.empty_like(y) if grad else None
    rc = lib.orc_phi(spline.s, spline.Xi.shape[1], _p(spline.Xi, ctypes.c_int32),
                     _p(spline.L, ctypes.c_int32), y.shape[0], _p(y, ctypes.c_double),
                     _p(out, ctypes.c_double), _p(g, ctypes.c_double) if grad else None)
    if rc:
        raise RuntimeError("orc_phi failed: %d" % rc)
    return (out, g) if grad else out


def _layout_args(spline: Spline, dims):
    dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int64).reshape(spline.s))
    D = np.ascontiguousarray(spline.D.astype(np.int32))
    return D, dims


def _coef_flat(spline: Spline, coeffs, dims):
    """coeffs: list of per-coset arrays of shape dims[::-1] (C order z,y,x)."""
    if isinstance(coeffs, np.ndarray) and coeffs.ndim == spline.s + 1:
        coeffs = list(coeffs)
    if len(coeffs) != spline.n_cosets:
        raise ValueError("need one array per coset")
    flat = np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1) for c in coeffs])
    n = int(np.prod(dims))
    if flat.size != n * spline.n_cosets:
        raise ValueError("coefficient array size mismatch")
    return np.ascontiguousarray(flat)


def evaluate(spline: Spline, dims, coeffs, x, grad: bool = False, brute: bool = False):
    """f(x) (and grad f) for per-coset coefficient arrays of extent dims=(X,Y[,Z])."""
    lib = _load()
    D, dims = _layout_args(spline, dims)
    flat = _coef_flat(spline, coeffs, dims)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, spline.s))
    f = np.empty(x.shape[0])
    g = np.empty_like(x) if grad else None
    rc = lib.orc_eval(spline.s, spline.Xi.shape[1], _p(spline.Xi, ctypes.c_int32),
                      _p(spline.L, ctypes.c_int32), spline.n_cosets, _p(D, ctypes.c_int32),
                      _p(spline.shifts, ctypes.c_int32), _p(dims, ctypes.c_int64),
                      _p(flat, ctypes.c_double), x.shape[0], _p(x, ctypes.c_double),
                      _p(f, ctypes.c_double), _p(g, ctypes.c_double) if grad else None,
                      1 if brute else 0)
    if rc:
        raise RuntimeError("orc_eval failed: %d" % rc)
    return (f, g) if grad else f


def evaluate_hessian(spline: Spline, dims, coeffs, x):
    """f(x), grad f and the Hessian of f ((N, s, s)) for per-coset coefficient
    arrays; only for box splines that stay C^1 after removing any direction
    (the derivative identity applied twice)."""
    lib = _load()
    D, dims = _layout_args(spline, dims)
    flat = _coef_flat(spline, coeffs, dims)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, spline.s))
    f = np.empty(x.shape[0])
    g = np.empty_like(x)
    h = np.empty((x.shape[0], spline.s, spline.s))
    rc = lib.orc_eval_hess(spline.s, spline.Xi.shape[1], _p(spline.Xi, ctypes.c_int32),
                           _p(spline.L, ctypes.c_int32), spline.n_cosets, _p(D, ctypes.c_int32),
                           _p(spline.shifts, ctypes.c_int32), _p(dims, ctypes.c_int64),
                           _p(flat, ctypes.c_double), x.shape[0], _p(x, ctypes.c_double),
                           _p(f, ctypes.c_double), _p(g, ctypes.c_double), _p(h, ctypes.c_double))
    if rc:
        raise RuntimeError("orc_eval_hess failed: %d" % rc)
    return f, g, h


def backward(spline: Spline, dims, x, g_out):
    """dL/dc (list of per-coset arrays, C order) for dL/df = g_out."""
    lib = _load()
    D, dims = _layout_args(spline, dims)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, spline.s))
    g_out = np.ascontiguousarray(np.asarray(g_out, dtype=np.float64).reshape(-1))
    n = int(np.prod(dims))
    out = np.empty(n * spline.n_cosets)
    rc = lib.orc_backward_coef(spline.s, spline.Xi.shape[1], _p(spline.Xi, ctypes.c_int32),
                               _p(spline.L, ctypes.c_int32), spline.n_cosets,
                               _p(D, ctypes.c_int32), _p(spline.shifts, ctypes.c_int32),
                               _p(dims, ctypes.c_int64), x.shape[0], _p(x, ctypes.c_double),
                               _p(g_out, ctypes.c_double), _p(out, ctypes.c_double))
    if rc:
        raise RuntimeError("orc_backward_coef failed: %d" % rc)
    shape = tuple(int(d) for d in dims[::-1])
    return [out[m * n:(m + 1) * n].reshape(shape) for m in range(spline.n_cosets)]


def backward_x(spline: Spline, dims, coeffs, x, g_out):
    """dL/dx_i = g_i grad f(x_i)."""
    _, gr = evaluate(spline, dims, coeffs, x, grad=True)
    return np.asarray(g_out, dtype=np.float64).reshape(-1, 1) * gr


def site_positions(spline: Spline, dims):
    """Positions of all stored sites, in the flat coefficient order."""
    dims = [int(d) for d in dims]
    out = []
    for m in range(spline.n_cosets):
        grids = np.meshgrid(*[np.arange(d) for d in dims[::-1]], indexing="ij")
        idx = np.stack([g.reshape(-1) for g in grids[::-1]], axis=1)  # x fastest
        out.append(idx * spline.D.reshape(1, -1) + spline.shifts[m].reshape(1, -1))
    return np.concatenate(out, axis=0)


def num_threads() -> int:
    return int(_load().orc_num_threads())
