"""Seeded synthetic inputs shaped like the paper's workloads (Sec. 5: random
query points in a volume on the Cartesian, BCC and FCC lattices).

This module only draws numbers: coefficient arrays, query points and a
smooth test field.  It holds none of the spline arithmetic and serves both the
HIP path and the CPU checker, which never import each other.

Seeds: numpy PCG64 with seed = 210208518 + 100 * workload + stream, where
stream 0 draws coefficients, 1 points, 2 noise, 3 field parameters.

Workloads (lattice extents are per Cartesian coset):
  1  Z^3 32^3, tricubic; coefficients U[-1,1] (FP64); 100000 points uniform
     in the interior.
  2  BCC 2 x 64^3, 8-direction box spline; coefficients = smooth field on the
     lattice plus N(0, 0.01^2) noise; 2^22 points uniform in the interior.
  3  FCC 4 x 128^3, 6-direction box spline; coefficients U[-1,1]; 2^24
     points on 512 x 512 orthographic rays x 64 samples, ordered
     [tile_y][tile_x][sample][8 x 8 pixels].
  4  BCC 2 x 96^3; 2^23 points uniform in the interior, targets = the smooth
     field at the points.
  5  64 volumes (even: tricubic on Z^3, odd: BCC 8-direction), extent
     E ~ U{16..128} per coset, coefficients U[-1,1], N_v = floor(exp(U(ln 1e3,
     ln 2^21))) points each.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

BASE_SEED = 210208518

# lattice description needed to place points: coset scale D, shifts, and the
# per-axis support half-width r of the spline (half the sum of |Xi| per row)
LATTICE = {
    "tricubic": dict(D=1, shifts=[(0, 0, 0)], r=2),
    "bcc8": dict(D=2, shifts=[(0, 0, 0), (1, 1, 1)], r=4),
    "fcc6": dict(D=2, shifts=[(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)], r=2),
    "trilinear": dict(D=1, shifts=[(0, 0, 0)], r=1),
    "bcc4": dict(D=2, shifts=[(0, 0, 0), (1, 1, 1)], r=2),
    "triquadratic": dict(D=1, shifts=[(0, 0, 0)], r=1.5),
    "cc7": dict(D=1, shifts=[(0, 0, 0)], r=2.5),
    "bcc7": dict(D=2, shifts=[(0, 0, 0), (1, 1, 1)], r=3),
    "cc6": dict(D=1, shifts=[(0, 0, 0)], r=2),
}


def rng(workload: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + 100 * workload + stream))


def interior(spline: str, E: int) -> Tuple[float, float]:
    """[r + 1, E_max - r - 1], E_max = the smallest per-coset maximum site
    coordinate: every stencil tap of a point in this box is a stored site."""
    lat = LATTICE[spline]
    emax = lat["D"] * (E - 1) + min(max(s) for s in lat["shifts"])
    return float(lat["r"] + 1), float(emax - lat["r"] - 1)


def site_positions(spline: str, E: int) -> np.ndarray:
    """(n_cosets, E, E, E, 3) lattice positions of the stored sites, C order."""
    lat = LATTICE[spline]
    i = np.arange(E)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    base = np.stack([x, y, z], axis=-1) * lat["D"]
    return np.stack([base + np.array(s) for s in lat["shifts"]])


@dataclass
class Field:
    """g(p) = sum_k a_k cos(2 pi w_k . (p - p0) / E + th_k) / scale."""
    a: np.ndarray
    w: np.ndarray
    th: np.ndarray
    p0: float
    E: float
    scale: float = 1.0

    def __call__(self, p: np.ndarray) -> np.ndarray:
        p = np.asarray(p, dtype=np.float64)
        ph = 2 * np.pi * ((p - self.p0) @ self.w.T) / self.E + self.th
        return (np.cos(ph) * self.a).sum(axis=-1) / self.scale


def smooth_field(workload: int, lo: float, hi: float) -> Field:
    r = rng(workload, 3)
    k = np.arange(1, 9)
    a = r.uniform(0.5, 1.0, 8) / k
    w = np.zeros((8, 3), dtype=np.int64)
    for j in range(8):
        while not w[j].any():
            w[j] = r.integers(-3, 4, 3)
    th = r.uniform(0, 2 * np.pi, 8)
    f = Field(a, w.astype(np.float64), th, lo, hi - lo)
    # normalise so that max |g| over a dense sample of the box is one
    s = rng(workload, 3).uniform(lo, hi, (200000, 3))
    f.scale = float(np.abs(f(s)).max())
    return f


def uniform_points(workload: int, spline: str, E: int, n: int) -> np.ndarray:
    lo, hi = interior(spline, E)
    return rng(workload, 1).uniform(lo, hi, (n, 3)).astype(np.float32)


def workload1(n: int = 100000):
    E = 32
    c = rng(1, 0).uniform(-1, 1, (1, E, E, E))
    return dict(spline="tricubic", E=E, coeffs=c, points=uniform_points(1, "tricubic", E, n))


def workload2(n: int = 1 << 22, E: int = 64):
    lo, hi = interior("bcc8", E)
    g = smooth_field(2, lo, hi)
    pos = site_positions("bcc8", E)
    c = g(pos) + rng(2, 2).normal(0.0, 0.01, pos.shape[:-1])
    return dict(spline="bcc8", E=E, coeffs=c, points=uniform_points(2, "bcc8", E, n))


# Per-coset extents of the equal-memory comparison of Sec. 5: CC 128^3, BCC
# inside 202^3 (2 cosets of 101^3) and FCC inside 161^3 (4 cosets of 81^3),
# about 2.1 M sites each.
ORDERS_E = {"cc": 128, "bcc": 101, "fcc": 81}
ORDERS = {2: ["trilinear", "bcc4"], 3: ["triquadratic", "fcc6", "cc6"],
          4: ["tricubic", "cc7", "bcc8", "bcc7"]}
LATTICE_NAME = {"tricubic": "cc", "trilinear": "cc", "triquadratic": "cc", "cc7": "cc", "cc6": "cc",
                "bcc8": "bcc", "bcc4": "bcc", "bcc7": "bcc", "fcc6": "fcc"}


def orders_workload(spline: str, n: int = 10 ** 6):
    """One spline of the order-2/3/4 comparisons: uniform coefficients in
    [-1, 1] on the equal-memory lattice, n uniform random points inside it."""
    E = ORDERS_E[LATTICE_NAME[spline]]
    nc = len(LATTICE[spline]["shifts"])
    wl = 10 + sorted(LATTICE_NAME).index(spline)
    c = rng(wl, 0).uniform(-1, 1, (nc, E, E, E)).astype(np.float32)
    return dict(spline=spline, E=E, coeffs=c, points=uniform_points(wl, spline, E, n))


def ray_points(workload: int, spline: str, E: int, width: int = 512, height: int = 512,
               samples: int = 64, tile: int = 8) -> np.ndarray:
    """Orthographic rays through the interior box along normalize(0.2, 0.1, 1);
    the image plane covers the central 80% of the box's cross-section."""
    lo, hi = interior(spline, E)
    c = 0.5 * (lo + hi)
    d = np.array([0.2, 0.1, 1.0])
    d /= np.linalg.norm(d)
    u = np.cross(d, [0.0, 1.0, 0.0])
    u /= np.linalg.norm(u)
    v = np.cross(u, d)
    half = 0.4 * (hi - lo)
    px = (np.arange(width) + 0.5) / width * 2 - 1
    py = (np.arange(height) + 0.5) / height * 2 - 1
    origin = (c + half * px[None, :, None] * u + half * py[:, None, None] * v)  # (H, W, 3)
    # entry/exit of each ray through the box
    with np.errstate(divide="ignore"):
        t0 = (lo - origin) / d
        t1 = (hi - origin) / d
    tin = np.minimum(t0, t1).max(axis=-1)
    tout = np.maximum(t0, t1).min(axis=-1)
    k = (np.arange(samples) + 0.5) / samples
    t = tin[..., None] + k * (tout - tin)[..., None]          # (H, W, S)
    p = origin[:, :, None, :] + t[..., None] * d             # (H, W, S, 3)
    p = np.clip(p, lo, hi)
    th, tw = height // tile, width // tile
    p = p.reshape(th, tile, tw, tile, samples, 3).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(p.reshape(-1, 3)).astype(np.float32)


def workload3(E: int = 128, width: int = 512, height: int = 512, samples: int = 64):
    c = rng(3, 0).uniform(-1, 1, (4, E, E, E))
    return dict(spline="fcc6", E=E, coeffs=c, points=ray_points(3, "fcc6", E, width, height, samples))


def workload4(n: int = 1 << 23, E: int = 96):
    lo, hi = interior("bcc8", E)
    g = smooth_field(4, lo, hi)
    x = uniform_points(4, "bcc8", E, n)
    return dict(spline="bcc8", E=E, points=x, targets=g(x.astype(np.float64)).astype(np.float32),
                field=g)


def workload5(n_vol: int = 64, emin: int = 16, emax: int = 128, nmin: float = 1e3,
              nmax: float = float(1 << 21)) -> List[dict]:
    r = rng(5, 0)
    rp = rng(5, 1)
    out = []
    for v in range(n_vol):
        spline = "tricubic" if v % 2 == 0 else "bcc8"
        E = int(r.integers(emin, emax + 1))
        nc = 1 if spline == "tricubic" else 2
        n = int(np.floor(np.exp(rp.uniform(np.log(nmin), np.log(nmax)))))
        lo, hi = interior(spline, E)
        out.append(dict(spline=spline, E=E, coeffs_seed=(v,), n=n,
                        coeffs=None, lo=lo, hi=hi, nc=nc))
    for v, d in enumerate(out):
        d["coeffs"] = rng(5, 10 + v).uniform(-1, 1, (d["nc"], d["E"], d["E"], d["E"])).astype(np.float32)
        d["points"] = rng(5, 1000 + v).uniform(d["lo"], d["hi"], (d["n"], 3)).astype(np.float32)
    return out
