"""CPU interpreter of the emitted tables (FP64, numpy).

It walks the same steps as the device code -- point location in the region
of evaluation, the symmetry transform to a reference sub-region, the stencil
lookup through the transformed offsets, and the sub-region polynomial -- so the
generated tables can be checked against the oracle without a GPU.  It belongs
to the product side (it reads only the generator's own tables), and is used by
tests only.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np

from .emit import OUT_DIR


def load_tables(name: str, directory: str = OUT_DIR) -> dict:
    with open(os.path.join(directory, "%s.json" % name)) as fh:
        return json.load(fh)


def locate(tab: dict, x: np.ndarray):
    """Return K (lattice site, int64), y (reference coords), G (N x 3 x 3 with
    y = G (x - K)), region index."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    if tab["roe"] == "floor":
        K = np.floor(x)
    elif tab["roe"] == "round":
        K = np.floor(x + 0.5)
    elif tab["lattice"] == "bcc":
        k0 = 2 * np.round(x / 2)
        k1 = 2 * np.round((x - 1) / 2) + 1
        d0 = ((x - k0) ** 2).sum(1)
        d1 = ((x - k1) ** 2).sum(1)
        K = np.where((d1 < d0)[:, None], k1, k0)
    elif tab["lattice"] == "fcc":
        r = np.round(x)
        odd = (r.sum(1) % 2) != 0
        res = x - r
        j = np.argmax(np.abs(res), axis=1)
        step = np.where(res[np.arange(N), j] >= 0, 1.0, -1.0)
        r[np.arange(N)[odd], j[odd]] += step[odd]
        K = r
    else:
        raise ValueError(tab["name"])
    d = x - K
    G = np.zeros((N, 3, 3))
    if tab["symmetry"] == "none":
        G[:] = np.eye(3)
    elif tab["symmetry"] == "signs":
        s = np.where(d < 0, -1.0, 1.0)
        for i in range(3):
            G[:, i, i] = s[:, i]
    elif tab["symmetry"] == "signed_perm":
        s = np.where(d < 0, -1.0, 1.0)
        a = np.abs(d)
        perm = np.argsort(-a, axis=1, kind="stable")
        for r in range(3):
            G[np.arange(N), r, perm[:, r]] = s[np.arange(N), perm[:, r]]
    y = np.einsum("nij,nj->ni", G, d)
    region = _lookup(tab["tree"], y)
    return K.astype(np.int64), y, G, region


def _lookup(node, y: np.ndarray) -> np.ndarray:
    """Reference sub-region of each row of y from the lookup tree (far side
    when n . y > t)."""
    if isinstance(node, int):
        return np.full(y.shape[0], node, dtype=np.int64)
    far = y @ np.array(node["n"], dtype=np.float64) > float(Fraction(node["t"]))
    return np.where(far, _lookup(node["far"], y), _lookup(node["near"], y))


def _poly_eval(terms: dict, u: np.ndarray) -> np.ndarray:
    out = np.zeros(u.shape[0])
    for key, c in terms.items():
        e = [int(v) for v in key.split(",")]
        out += float(Fraction(c)) * u[:, 0] ** e[0] * u[:, 1] ** e[1] * u[:, 2] ** e[2]
    return out


def evaluate(tab: dict, dims, coeffs, x):
    """f(x) with per-coset coefficient arrays (C order z,y,x); zero padding."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    K, y, G, region = locate(tab, x)
    D = np.array(tab["D"])
    shifts = [tuple(s) for s in tab["shifts"]]
    dims = np.array(dims)
    f = np.zeros(len(x))
    for ri, reg in enumerate(tab["regions"]):
        sel = region == ri
        if not sel.any():
            continue
        u = y[sel] - np.array([float(Fraction(v)) for v in reg["frame"]])
        for o, w in zip(reg["taps"], reg["weights"]):
            g = np.einsum("nji,j->ni", G[sel], np.array(o, dtype=np.float64))  # G^T o
            n = K[sel] + np.round(g).astype(np.int64)
            par = tuple(0 for _ in range(3))
            vals = np.zeros(sel.sum())
            for m, sh in enumerate(shifts):
                inc = np.all((n - np.array(sh)) % D == 0, axis=1)
                idx = (n - np.array(sh)) // D
                ok = inc & np.all((idx >= 0) & (idx < dims), axis=1)
                if ok.any():
                    ii = idx[ok]
                    vals[ok] = coeffs[m][ii[:, 2], ii[:, 1], ii[:, 0]]
            f[sel] += vals * _poly_eval(w, u)
    return f
