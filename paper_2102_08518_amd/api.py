"""Python binding of the lattice-spline library: torch tensors hold device
memory and the current stream; every step of the computation runs in the HIP
library (liblsp.so).  Names follow the C ABI in include/lsp.h.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N

_DT = {"f32": N.LSP_F32, "f64": N.LSP_F64, "bf16": N.LSP_BF16, "f16": N.LSP_F16}
_TORCH_DT = {torch.float32: N.LSP_F32, torch.float64: N.LSP_F64, torch.bfloat16: N.LSP_BF16,
             torch.float16: N.LSP_F16}

# Direction matrices (columns are directions) and lattice generators
# (columns are generators) of the supported splines.
_E3 = np.eye(3, dtype=np.int32)
_DIAG = np.array([(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)], dtype=np.int32)
_FCC_DIRS = np.array([(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)],
                     dtype=np.int32)
LATTICES = {
    "cc": _E3,
    "bcc": np.array([[-1, 1, 1], [1, -1, 1], [1, 1, -1]], dtype=np.int32),
    "fcc": np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=np.int32),
}
DIRECTIONS = {
    "tricubic": np.concatenate([_E3] * 4, axis=1),
    "bcc8": np.concatenate([_DIAG.T, _DIAG.T], axis=1),
    "fcc6": _FCC_DIRS.T.copy(),
    "trilinear": np.concatenate([_E3] * 2, axis=1),
    "bcc4": _DIAG.T.copy(),
    "triquadratic": np.concatenate([_E3] * 3, axis=1),
    "cc7": np.concatenate([_E3, _DIAG.T], axis=1),
    "bcc7": np.concatenate([_DIAG.T, 2 * _E3], axis=1),
    "cc6": np.array([(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)], dtype=np.int32).T.copy(),
}
LATTICE_OF = {"tricubic": "cc", "bcc8": "bcc", "fcc6": "fcc", "trilinear": "cc", "bcc4": "bcc",
              "triquadratic": "cc", "cc7": "cc", "bcc7": "bcc", "cc6": "cc"}


def set_option(option: int, value: int) -> None:
    """lsp_set_option: process-wide evaluation options (N.LSP_OPT_MFMA,
    N.LSP_OPT_PREDICATED)."""
    N.check(N.lib().lsp_set_option(option, value))


def use_predication(on: bool) -> None:
    """Branch-free (both polynomials, select) or branchy evaluation of the
    two-polynomial FCC spline in the direct entry points."""
    set_option(N.LSP_OPT_PREDICATED, 1 if on else 0)


def set_split_maxn(n: int) -> None:
    """Largest point count the separable splines evaluate with four lanes
    per point (0: never; -1: each spline's measured default)."""
    set_option(N.LSP_OPT_SPLIT_MAXN, int(n))


def use_mfma(on) -> None:
    """How the monomial coefficients of the splines with a matrix-core form
    are evaluated: False (per-lane FMAs, the default), True (matrix cores) or
    "auto" (matrix cores for 16-bit coefficient storage)."""
    set_option(N.LSP_OPT_MFMA, 2 if on == "auto" else (1 if on else 0))


def _stream(device: Optional[torch.device] = None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else None)


class Spline:
    """A (lattice, direction matrix) pair the library has generated code for."""

    def __init__(self, L, Xi):
        L = np.ascontiguousarray(np.asarray(L, dtype=np.int32))
        Xi = np.ascontiguousarray(np.asarray(Xi, dtype=np.int32))
        if L.shape != (3, 3) or Xi.ndim != 2 or Xi.shape[0] != 3:
            raise ValueError("L must be 3x3 and Xi 3xn")
        h = ctypes.c_void_p()
        N.check(N.lib().lsp_spline_create(3, L.ctypes.data_as(N.i32p), Xi.ctypes.data_as(N.i32p),
                                          Xi.shape[1], ctypes.byref(h)))
        self._h = h
        info = N.SplineInfo()
        N.check(N.lib().lsp_spline_get_info(h, ctypes.byref(info)))
        self.info = info

    @property
    def continuity(self) -> int:
        """phi is C^continuity (second derivatives need at least 1)."""
        return self.info.continuity

    @classmethod
    def tricubic(cls):
        return cls(LATTICES["cc"], DIRECTIONS["tricubic"])

    @classmethod
    def bcc8(cls):
        return cls(LATTICES["bcc"], DIRECTIONS["bcc8"])

    @classmethod
    def fcc6(cls):
        return cls(LATTICES["fcc"], DIRECTIONS["fcc6"])

    @classmethod
    def trilinear(cls):
        return cls(LATTICES["cc"], DIRECTIONS["trilinear"])

    @classmethod
    def bcc4(cls):
        return cls(LATTICES["bcc"], DIRECTIONS["bcc4"])

    @classmethod
    def triquadratic(cls):
        return cls(LATTICES["cc"], DIRECTIONS["triquadratic"])

    @classmethod
    def cc7(cls):
        """Seven-direction box spline on Z^3 (axes and diagonals), fourth order."""
        return cls(LATTICES["cc"], DIRECTIONS["cc7"])

    @classmethod
    def bcc7(cls):
        """Quartic box spline on BCC (diagonals and 2 e_i), fourth order."""
        return cls(LATTICES["bcc"], DIRECTIONS["bcc7"])

    @classmethod
    def cc6(cls):
        """Six-direction box spline on Z^3 (the face diagonals), third order;
        its reference sub-regions are derived automatically."""
        return cls(LATTICES["cc"], DIRECTIONS["cc6"])

    @classmethod
    def named(cls, name: str):
        return cls(LATTICES[LATTICE_OF[name]], DIRECTIONS[name])

    @classmethod
    def from_plugin(cls, path: str):
        """A spline compiled at run time (lsp_spline_load_plugin); see jit.py."""
        obj = cls.__new__(cls)
        h = ctypes.c_void_p()
        N.check(N.lib().lsp_spline_load_plugin(os.fsencode(path), ctypes.byref(h)))
        obj._h = h
        info = N.SplineInfo()
        N.check(N.lib().lsp_spline_get_info(h, ctypes.byref(info)))
        obj.info = info
        return obj

    @classmethod
    def compile(cls, lattice: str, Xi, name: Optional[str] = None):
        """Analyse, generate and compile the box spline with directions Xi (the
        rows) on lattice "cc", "bcc" or "fcc" at run time, then load it."""
        from . import jit
        return cls.from_plugin(jit.compile_spline(lattice, [tuple(int(v) for v in d) for d in Xi], name))

    @property
    def n_cosets(self) -> int:
        return self.info.n_cosets

    # -- host diagnostics of the location step (no device work)
    def debug_tap_offsets(self, dims, pts, storage: str = "f32"):
        pts = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        n = pts.shape[0]
        d = (ctypes.c_int64 * 3)(*[int(v) for v in dims])
        offs = np.empty((n, self.info.union_taps), dtype=np.int32)
        flags = np.empty(n, dtype=np.int32)
        N.check(N.lib().lsp_debug_tap_offsets(self._h, d, _DT[storage],
                                              pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              n, offs.ctypes.data_as(N.i32p),
                                              flags.ctypes.data_as(N.i32p)))
        return offs, flags

    def debug_geometry(self, dims, storage: str = "f32"):
        d = (ctypes.c_int64 * 3)(*[int(v) for v in dims])
        g = np.empty(20, dtype=np.int32)
        nb = ctypes.c_size_t()
        N.check(N.lib().lsp_debug_geometry(self._h, d, _DT[storage], g.ctypes.data_as(N.i32p),
                                           ctypes.byref(nb)))
        v = [int(x) for x in g]
        return dict(es=v[0], pad=v[1], kmin=v[2:5], kmax=v[5:8], lb=v[8:11], bs=v[11:14],
                    is_=v[14:17], ctype=v[17], n_cosets=v[18], nbytes=nb.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and N is not None and N._lib is not None:
            N._lib.lsp_spline_destroy(h)
            self._h = None


class Volume:
    """A spline with coefficients bound in the library's internal layout."""

    def __init__(self, spline: Spline, dims: Sequence[int], storage: str = "f32"):
        self.spline = spline
        self.dims = tuple(int(d) for d in dims)
        self.storage = storage
        d = (ctypes.c_int64 * 3)(*self.dims)
        h = ctypes.c_void_p()
        N.check(N.lib().lsp_volume_create(spline._h, d, _DT[storage], ctypes.byref(h)))
        self._h = h
        self.n_cosets = spline.n_cosets

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and N is not None and N._lib is not None:
            N._lib.lsp_volume_destroy(h)
            self._h = None

    @property
    def n_coeffs(self) -> int:
        return self.n_cosets * self.dims[0] * self.dims[1] * self.dims[2]

    def set(self, cosets) -> None:
        """cosets: a (n_cosets, Z, Y, X) tensor or a list of (Z, Y, X) tensors
        on the device; converted to the storage dtype in the library."""
        if isinstance(cosets, torch.Tensor):
            cosets = list(cosets.reshape(self.n_cosets, *self.dims[::-1]))
        if len(cosets) != self.n_cosets:
            raise ValueError("need %d coset arrays" % self.n_cosets)
        cosets = [c.contiguous() for c in cosets]
        for c in cosets:
            if c.shape != self.dims[::-1] or not c.is_cuda:
                raise ValueError("each coset must be a device tensor of shape %s" % (self.dims[::-1],))
        dt = {c.dtype for c in cosets}
        if len(dt) != 1:
            raise ValueError("coset arrays must share a dtype")
        arr = (ctypes.c_void_p * self.n_cosets)(*[c.data_ptr() for c in cosets])
        N.check(N.lib().lsp_volume_set_coeffs(self._h, arr, _TORCH_DT[cosets[0].dtype],
                                              _stream(cosets[0].device)))
        self._keep = cosets  # keep the sources alive until the stream has consumed them

    @staticmethod
    def _pts(pts: torch.Tensor) -> torch.Tensor:
        if pts.dim() != 2 or pts.shape[1] != 3:
            raise ValueError("points must be (N, 3)")
        if pts.dtype not in (torch.float32, torch.float64):
            raise ValueError("points must be float32 or float64")
        if not pts.is_cuda:
            raise ValueError("points must be on the device")
        return pts.contiguous()

    def _binned_ws(self, pts: torch.Tensor, workspace: Optional[torch.Tensor]):
        b = ctypes.c_size_t()
        N.check(N.lib().lsp_eval_binned_workspace_size(self._h, _TORCH_DT[pts.dtype], pts.shape[0],
                                                       ctypes.byref(b)))
        if workspace is None or workspace.numel() < b.value + 256:
            workspace = torch.empty(b.value + 256, dtype=torch.uint8, device=pts.device)
        base = workspace.data_ptr()
        ptr = (base + 255) // 256 * 256
        return workspace, ptr, workspace.numel() - (ptr - base)

    def eval(self, pts: torch.Tensor, out: Optional[torch.Tensor] = None, binned: bool = False,
             workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
        """f at the points; binned=True evaluates in spatially binned order
        (same results, faster for many points in random order)."""
        pts = self._pts(pts)
        if out is None:
            out = torch.empty(pts.shape[0], dtype=torch.float32, device=pts.device)
        if binned and pts.shape[0] > 0:
            workspace, ptr, n = self._binned_ws(pts, workspace)
            N.check(N.lib().lsp_eval_binned(self._h, _ptr(pts), _TORCH_DT[pts.dtype], pts.shape[0],
                                            _ptr(out), None, ctypes.c_void_p(ptr), n,
                                            _stream(pts.device)))
            return out
        N.check(N.lib().lsp_eval(self._h, _ptr(pts), _TORCH_DT[pts.dtype], pts.shape[0], _ptr(out),
                                 _stream(pts.device)))
        return out

    def eval_grad(self, pts: torch.Tensor, want_value: bool = True, binned: bool = False,
                  workspace: Optional[torch.Tensor] = None):
        pts = self._pts(pts)
        n = pts.shape[0]
        val = torch.empty(n, dtype=torch.float32, device=pts.device) if (want_value or binned) else None
        grad = torch.empty(n, 3, dtype=torch.float32, device=pts.device)
        if binned and n > 0:
            workspace, ptr, nb = self._binned_ws(pts, workspace)
            N.check(N.lib().lsp_eval_binned(self._h, _ptr(pts), _TORCH_DT[pts.dtype], n, _ptr(val),
                                            _ptr(grad), ctypes.c_void_p(ptr), nb,
                                            _stream(pts.device)))
            return (val if want_value else None), grad
        N.check(N.lib().lsp_eval_grad(self._h, _ptr(pts), _TORCH_DT[pts.dtype], n, _ptr(val),
                                      _ptr(grad), _stream(pts.device)))
        return val, grad

    def eval_hessian(self, pts: torch.Tensor, want_value: bool = True, want_grad: bool = True):
        """(f or None, grad (N, 3) or None, Hessian (N, 3, 3)) at the points.
        Only for splines that are at least C^1 (Spline.continuity >= 1)."""
        pts = self._pts(pts)
        n = pts.shape[0]
        dev = pts.device
        val = torch.empty(n, dtype=torch.float32, device=dev) if want_value else None
        grad = torch.empty(n, 3, dtype=torch.float32, device=dev) if want_grad else None
        h6 = torch.empty(n, 6, dtype=torch.float32, device=dev)
        N.check(N.lib().lsp_eval_hessian(self._h, _ptr(pts), _TORCH_DT[pts.dtype], n, _ptr(val),
                                         _ptr(grad), _ptr(h6), _stream(dev)))
        idx = torch.tensor([0, 1, 2, 1, 3, 4, 2, 4, 5], device=dev)
        return val, grad, h6[:, idx].reshape(n, 3, 3)

    def workspace_bytes(self, n: int) -> int:
        b = ctypes.c_size_t()
        N.check(N.lib().lsp_backward_workspace_size(self._h, n, ctypes.byref(b)))
        return b.value

    def backward(self, pts: torch.Tensor, dL_df: torch.Tensor, want_dc: bool = True,
                 want_dx: bool = True, workspace: Optional[torch.Tensor] = None,
                 grad_f: Optional[torch.Tensor] = None):
        """(dL/dc as (n_cosets, Z, Y, X) float32 or None, dL/dx as (N, 3) or None).
        With grad_f (the (N, 3) gradient from eval_grad of the same points),
        dL/dx is formed from it (lsp_backward_dx_from_grad) instead of
        evaluating the spline's gradient again."""
        pts = self._pts(pts)
        n = pts.shape[0]
        g = dL_df.contiguous().to(torch.float32)
        dc = (torch.empty((self.n_cosets,) + self.dims[::-1], dtype=torch.float32,
                          device=pts.device) if want_dc else None)
        dx = torch.empty(n, 3, dtype=torch.float32, device=pts.device) if want_dx else None
        if want_dx and grad_f is not None:
            gf = grad_f.contiguous()
            if gf.shape != (n, 3) or gf.dtype != torch.float32:
                raise ValueError("grad_f must be a (N, 3) float32 tensor")
            N.check(N.lib().lsp_backward_dx_from_grad(n, _ptr(g), _ptr(gf), _ptr(dx),
                                                      _stream(pts.device)))
            if not want_dc:
                return dc, dx
            dx_arg = None
        else:
            dx_arg = dx
        wsb = self.workspace_bytes(n) if want_dc else 0
        if wsb and (workspace is None or workspace.numel() < wsb):
            workspace = torch.empty(wsb + 256, dtype=torch.uint8, device=pts.device)
        ws_ptr, ws_len = None, 0
        if wsb:
            base = workspace.data_ptr()
            ws_ptr = (base + 255) // 256 * 256
            ws_len = workspace.numel() - (ws_ptr - base)
        N.check(N.lib().lsp_backward(self._h, _ptr(pts), _TORCH_DT[pts.dtype], n, _ptr(g), _ptr(dc),
                                     _ptr(dx_arg), ctypes.c_void_p(ws_ptr), ws_len,
                                     _stream(pts.device)))
        return dc, dx


class BatchPlan:
    """Many volumes of uneven size evaluated by one persistent launch that
    is captured in a HIP graph; run() replays it on the current stream."""

    def __init__(self, vols: Sequence[Volume], pts: Sequence[torch.Tensor],
                 want_grad: Sequence[bool] = None, autotune: bool = True):
        n = len(vols)
        if len(pts) != n:
            raise ValueError("one point tensor per volume")
        want_grad = list(want_grad) if want_grad is not None else [False] * n
        self.vols = list(vols)
        self.pts = [Volume._pts(p) for p in pts]
        for p in self.pts:
            if p.dtype != torch.float32:
                raise ValueError("batched points must be float32")
        dev = self.pts[0].device
        self.val = [torch.empty(p.shape[0], dtype=torch.float32, device=dev) for p in self.pts]
        self.grad = [torch.empty(p.shape[0], 3, dtype=torch.float32, device=dev) if g else None
                     for p, g in zip(self.pts, want_grad)]
        arr = lambda xs: (ctypes.c_void_p * n)(*[x if x is not None else None for x in xs])
        h = ctypes.c_void_p()
        N.check(N.lib().lsp_batch_plan_create(
            n, arr([v._h.value for v in self.vols]), arr([p.data_ptr() for p in self.pts]),
            (ctypes.c_int64 * n)(*[p.shape[0] for p in self.pts]),
            arr([v.data_ptr() for v in self.val]),
            arr([g.data_ptr() if g is not None else None for g in self.grad]),
            N.LSP_BATCH_AUTOTUNE if autotune else 0, _stream(dev), ctypes.byref(h)))
        self._h = h
        t, b, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        N.check(N.lib().lsp_batch_plan_info(h, ctypes.byref(t), ctypes.byref(b), ctypes.byref(k)))
        self.tile, self.blocks, self.n_items = t.value, b.value, k.value

    def run(self):
        N.check(N.lib().lsp_batch_run(self._h, _stream(self.pts[0].device)))
        return self.val, self.grad

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and N is not None and N._lib is not None:
            N._lib.lsp_batch_plan_destroy(h)
            self._h = None


class LatticeSplineFn(torch.autograd.Function):
    """f = sum_n c_n phi(x - n) with gradients for the points and the
    coefficients.  coeffs is the (n_cosets, Z, Y, X) float32 tensor whose
    values are (re)loaded into `vol` on every forward."""

    @staticmethod
    def forward(ctx, pts: torch.Tensor, coeffs: torch.Tensor, vol: Volume):
        vol.set(coeffs.detach())
        ctx.vol = vol
        if pts.requires_grad:
            # the gradient with respect to the points comes with the value
            val, grad = vol.eval_grad(pts.detach())
            ctx.save_for_backward(pts, grad)
            return val
        ctx.save_for_backward(pts)
        return vol.eval(pts.detach())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        saved = ctx.saved_tensors
        pts = saved[0]
        grad_f = saved[1] if len(saved) > 1 else None
        want_dx = ctx.needs_input_grad[0]
        want_dc = ctx.needs_input_grad[1]
        dc, dx = ctx.vol.backward(pts.detach(), g, want_dc=want_dc, want_dx=want_dx, grad_f=grad_f)
        if dx is not None:
            dx = dx.to(pts.dtype)
        return dx, dc, None
