"""Pins for the FP64 oracle: values and identities fixed by the paper or by
mathematics, chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the recurrence, the centring, the normalisation or the
site enumeration fails at least one of them."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import BCC4, BCC7, BCC8, CC6, CC7, FCC6, TRICUBIC, TRILINEAR, TRIQUADRATIC, ZP

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(20210208)


def beta3(t):
    """Centred cubic B-spline, textbook closed form."""
    a = np.abs(t)
    return np.where(a <= 1, 2 / 3 - a ** 2 + a ** 3 / 2, np.where(a <= 2, (2 - a) ** 3 / 6, 0.0))


def hat(t):
    return np.maximum(0.0, 1 - np.abs(t))


def beta2(t):
    """Centred quadratic B-spline, textbook closed form."""
    a = np.abs(t)
    return np.where(a <= 0.5, 0.75 - a ** 2, np.where(a <= 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


# ------------------------------------------------------------ closed forms

def test_tricubic_is_tensor_product_of_cubic_bsplines():
    y = rng.uniform(-2.2, 2.2, (400, 3))
    ref = beta3(y[:, 0]) * beta3(y[:, 1]) * beta3(y[:, 2])
    np.testing.assert_allclose(oracle.phi(TRICUBIC, y), ref, rtol=0, atol=1e-14)


def test_tricubic_knot_values():
    vals = {0: 2 / 3, 0.5: 23 / 48, 1: 1 / 6, 1.5: 1 / 48, 2: 0.0}
    for t, v in vals.items():
        for s in (1, -1):
            got = oracle.phi(TRICUBIC, [[s * t, 0, 0], [0, s * t, 0], [0, 0, s * t]])
            np.testing.assert_allclose(got, v * (2 / 3) ** 2, atol=1e-15)
    np.testing.assert_allclose(oracle.phi(TRICUBIC, [[0, 0, 0]]), 8 / 27, atol=1e-15)


def test_trilinear_is_tensor_product_of_hats():
    y = rng.uniform(-1.2, 1.2, (400, 3))
    ref = hat(y[:, 0]) * hat(y[:, 1]) * hat(y[:, 2])
    np.testing.assert_allclose(oracle.phi(TRILINEAR, y), ref, atol=1e-14)


def test_triquadratic_is_tensor_product_of_quadratic_bsplines():
    y = rng.uniform(-1.7, 1.7, (400, 3))
    ref = beta2(y[:, 0]) * beta2(y[:, 1]) * beta2(y[:, 2])
    np.testing.assert_allclose(oracle.phi(TRIQUADRATIC, y), ref, rtol=0, atol=1e-14)
    # knot values 3/4, 1/2, 1/8, 0 at 0, 1/2, 1, 3/2
    for t, v in {0: 0.75, 0.5: 0.5, 1: 0.125, 1.5: 0.0}.items():
        got = oracle.phi(TRIQUADRATIC, [[t, 0, 0], [0, -t, 0]])
        np.testing.assert_allclose(got, v * 0.75 ** 2, atol=1e-15)


def test_tricubic_gradient_closed_form():
    y = rng.uniform(-2.2, 2.2, (200, 3))

    def dbeta3(t):
        a = np.abs(t)
        s = np.sign(t)
        return s * np.where(a <= 1, -2 * a + 1.5 * a ** 2, np.where(a <= 2, -0.5 * (2 - a) ** 2, 0))

    b = [beta3(y[:, i]) for i in range(3)]
    db = [dbeta3(y[:, i]) for i in range(3)]
    ref = np.stack([db[0] * b[1] * b[2], b[0] * db[1] * b[2], b[0] * b[1] * db[2]], axis=1)
    _, g = oracle.phi(TRICUBIC, y, grad=True)
    np.testing.assert_allclose(g, ref, atol=1e-13)


# ------------------------------------------------------ the worked example

def _fig1():
    with open(os.path.join(GOLDEN, "zp_fig1.json")) as fh:
        d = json.load(fh)
    W = np.array([[float(Fraction(v)) for v in row] for row in d["weights"]])
    return np.array(d["monomials"]), np.array(d["offsets"]), W


def test_zp_matches_fig1_polynomial():
    """Fig. 1: the weight of c_j in sub-region 1 is phi(x - o_j)."""
    mono, offs, W = _fig1()
    x = rng.uniform(-0.5, 0.5, (4000, 2))
    x = x[x[:, 0] >= np.abs(x[:, 1])]
    M = np.stack([x[:, 0] ** a * x[:, 1] ** b for a, b in mono], axis=1)
    expect = M @ W.T
    got = np.stack([oracle.phi(ZP, x - o) for o in offs], axis=1)
    np.testing.assert_allclose(got, expect, atol=1e-14)
    # the seven taps are all there is: partition of unity inside sub-region 1
    np.testing.assert_allclose(expect.sum(axis=1), 1.0, atol=1e-14)


def test_zp_subregions_are_rotations_of_subregion1():
    """Fig. 1 table: sub-regions 2-4 are sub-region 1 rotated by 90, 180, 270 degrees."""
    y = rng.uniform(-1.6, 1.6, (500, 2))
    base = oracle.phi(ZP, y)
    for k in range(1, 4):
        c, s = np.round(np.cos(k * np.pi / 2)), np.round(np.sin(k * np.pi / 2))
        R = np.array([[c, -s], [s, c]])
        np.testing.assert_allclose(oracle.phi(ZP, y @ R.T), base, atol=1e-14)


def test_zp_exact_values():
    pts = {(0, 0): 1 / 2, (1, 0): 1 / 8, (0, 1): 1 / 8, (-1, 0): 1 / 8, (0, -1): 1 / 8,
           (1, 1): 0, (1.5, 0): 0, (0.5, 0): 3 / 8, (0.5, 1): 1 / 16, (0.25, 0.25): 7 / 16,
           (1.25, 0.25): 1 / 32, (0.25, 1.25): 1 / 32, (0.25, -0.75): 7 / 32,
           (-0.75, 0.25): 7 / 32, (-0.75, -0.75): 1 / 16, (-0.75, 1.25): 0}
    got = oracle.phi(ZP, list(pts.keys()))
    np.testing.assert_allclose(got, list(pts.values()), atol=1e-15)


# ------------------------------------------------- paper's structural counts

def _support_count(sp, x, radius):
    """Number of lattice sites with phi(x - n) > 0 around a generic point."""
    r = int(np.ceil(radius)) + 2
    rngs = [range(int(np.floor(x[i])) - r, int(np.floor(x[i])) + r + 1) for i in range(sp.s)]
    sites = []
    for n in itertools.product(*rngs):
        n = np.array(n)
        if any(np.all((n - sh) % sp.D == 0) for sh in sp.shifts):
            sites.append(n)
    sites = np.array(sites)
    v = np.abs(oracle.phi(sp, x - sites))
    if np.any((v > 0) & (v < 1e-9)):
        return None  # too close to the support boundary to count reliably
    return int((v > 1e-9).sum())


@pytest.mark.parametrize("sp,count", [(BCC4, 4), (ZP, 7), (TRICUBIC, 64), (TRILINEAR, 8),
                                      (BCC8, 32), (FCC6, 16), (TRIQUADRATIC, 27), (CC7, 53),
                                      (BCC7, 30), (CC6, 32)])
def test_taps_at_generic_points(sp, count):
    """BCC linear: four lookups (Sec. 5.1); ZP: seven sites c0..c6 (Fig. 1);
    tricubic: 64 fetches (Sec. 5.1); in general vol(supp)/|det L|, the
    support being the zonotope of Xi, whose volume is the sum of |det| over
    all triples of directions (CC7: 1 + 12 + 24 + 16 = 53; BCC7:
    (8 + 48 + 48 + 16) / 4 = 30)."""
    done = 0
    while done < 5:
        x = rng.uniform(-3, 3, sp.s)
        got = _support_count(sp, x, sp.halfwidth.max())
        if got is None:
            continue
        assert got == count
        done += 1


def test_bcc_linear_interpolates():
    lat = np.array([(0, 0, 0), (2, 0, 0), (1, 1, 1), (-1, 1, -1), (2, 2, 0), (0, 0, 2)])
    np.testing.assert_allclose(oracle.phi(BCC4, lat), [1, 0, 0, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(oracle.phi(BCC4, [[0.5, 0.5, 0.5]]), 0.5, atol=1e-15)


# ---------------------------------------------------------- invariants

SPL3 = [TRICUBIC, BCC8, FCC6, CC7, BCC7, CC6]


def _lattice_box(sp, E):
    dims = (E,) * sp.s
    return dims


def _ext(sp, E):
    """E, or the smallest extent whose interior box (below) is at least one
    lattice unit wide."""
    need = int(np.ceil((2 * sp.halfwidth.max() + 3) / sp.D.min())) + 1
    return max(E, need)


def _interior(sp, E, n):
    hw = sp.halfwidth.max()
    hi = (E - 1) * sp.D.min() + sp.shifts.min()
    assert hi - hw - 1 >= hw + 2, "extent too small for an interior box"
    return rng.uniform(hw + 1, hi - hw - 1, (n, sp.s))


@pytest.mark.parametrize("sp", SPL3 + [ZP, BCC4, TRILINEAR, TRIQUADRATIC])
def test_partition_of_unity_and_linear_reproduction(sp):
    E = _ext(sp, 12 if sp.D.max() == 1 else 8)
    dims = _lattice_box(sp, E)
    x = _interior(sp, E, 60)
    pos = oracle.site_positions(sp, dims).astype(np.float64)
    a = rng.normal(size=sp.s)
    b = 0.7
    for coef_of, expect in [(np.ones(len(pos)), np.ones(len(x))),
                            (pos @ a + b, x @ a + b)]:
        coeffs = coef_of.reshape(sp.n_cosets, -1)
        coeffs = [c.reshape(tuple(dims[::-1])) for c in coeffs]
        f = oracle.evaluate(sp, dims, coeffs, x)
        np.testing.assert_allclose(f, expect, atol=1e-12)


@pytest.mark.parametrize("sp,M", [(TRICUBIC, np.eye(3) / 3), (BCC8, 2 * np.eye(3) / 3),
                                  (FCC6, np.eye(3) / 3), (ZP, np.eye(2) / 4),
                                  (TRIQUADRATIC, np.eye(3) / 4), (CC7, 5 * np.eye(3) / 12),
                                  (BCC7, 2 * np.eye(3) / 3), (CC6, np.eye(3) / 3)])
def test_second_moment_is_XiXiT_over_12(sp, M):
    """Sum_n (n-x)(n-x)^T phi(x-n) = Xi Xi^T / 12 for approximation order >= 3."""
    np.testing.assert_allclose(sp.Xi @ sp.Xi.T / 12.0, M)
    E = _ext(sp, 12 if sp.D.max() == 1 else 8)
    dims = _lattice_box(sp, E)
    x = _interior(sp, E, 40)
    pos = oracle.site_positions(sp, dims).astype(np.float64)
    for a in range(sp.s):
        for b in range(a, sp.s):
            # c_n = (n_a - x0_a)(n_b - x0_b) reproduces u_a u_b + M_ab
            x0 = np.full(sp.s, 3.0)
            c = (pos[:, a] - x0[a]) * (pos[:, b] - x0[b])
            coeffs = [cc.reshape(tuple(dims[::-1])) for cc in c.reshape(sp.n_cosets, -1)]
            f = oracle.evaluate(sp, dims, coeffs, x)
            u = x - x0
            np.testing.assert_allclose(f, u[:, a] * u[:, b] + M[a, b], atol=1e-11)


@pytest.mark.parametrize("sp", [TRICUBIC, BCC8, CC7, BCC7])
def test_cubic_reproduction_order4(sp):
    """Approximation order 4: cubic data give u_a u_b u_c + u_a M_bc + u_b M_ac + u_c M_ab."""
    M = sp.Xi @ sp.Xi.T / 12.0
    E = _ext(sp, 10 if sp.D.max() == 1 else 7)
    dims = _lattice_box(sp, E)
    x = _interior(sp, E, 30)
    pos = oracle.site_positions(sp, dims).astype(np.float64)
    x0 = np.array([3.0, 2.5, 4.0])
    a, b, cc = 0, 1, 2
    p = pos - x0
    c = p[:, a] * p[:, b] * p[:, cc] + p[:, 0] ** 3
    coeffs = [v.reshape(tuple(dims[::-1])) for v in c.reshape(sp.n_cosets, -1)]
    f = oracle.evaluate(sp, dims, coeffs, x)
    u = x - x0
    expect = (u[:, a] * u[:, b] * u[:, cc] + u[:, a] * M[b, cc] + u[:, b] * M[a, cc] + u[:, cc] * M[a, b]
              + u[:, 0] ** 3 + 3 * u[:, 0] * M[0, 0])
    np.testing.assert_allclose(f, expect, atol=1e-10)


def _oh_group():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            G = np.zeros((3, 3))
            for i, p in enumerate(perm):
                G[i, p] = signs[i]
            mats.append(G)
    return mats


@pytest.mark.parametrize("sp", SPL3)
def test_octahedral_symmetry(sp):
    y = rng.uniform(-2.5, 2.5, (80, 3))
    base = oracle.phi(sp, y)
    assert base.max() > 0.01
    for G in _oh_group():
        np.testing.assert_allclose(oracle.phi(sp, y @ G.T), base, atol=1e-14)


def test_direction_signs_do_not_matter():
    flipped = oracle.Spline("bcc8f", BCC8.L, BCC8.Xi * np.array([1, -1, 1, -1, 1, 1, -1, 1]),
                            BCC8.D, BCC8.shifts)
    y = rng.uniform(-3, 3, (100, 3))
    np.testing.assert_allclose(oracle.phi(flipped, y), oracle.phi(BCC8, y), atol=1e-15)


@pytest.mark.parametrize("sp", SPL3)
def test_integral_is_det_L(sp):
    """int phi = |det L|.  The Riemann sum on the grid (1/2)Z^3 + offset is exact:
    the Fourier transform of each of these box splines vanishes on 4 pi Z^3 \\ {0}
    (some direction xi has xi . omega a nonzero multiple of 2 pi there)."""
    h = 0.5
    hw = sp.halfwidth
    for _ in range(2):
        off = rng.uniform(0, h, 3)
        axes = [np.arange(-hw[i] - h, hw[i] + h, h) + off[i] for i in range(3)]
        g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
        integral = oracle.phi(sp, g).sum() * h ** 3
        assert abs(integral - sp.det_L) < 1e-12


@pytest.mark.parametrize("sp,order", [(TRICUBIC, 2), (BCC8, 2), (FCC6, 1), (ZP, 1), (CC7, 2),
                                      (BCC7, 2), (CC6, 1)])
def test_smoothness_across_knot_planes(sp, order):
    """phi is C^{m-2}: values (and gradients for C^1, Hessians for C^2)
    continue across knot planes."""
    eps = 1e-7
    pts = rng.uniform(-1.5, 1.5, (200, sp.s))
    if sp is CC7:
        pts[:, 1] = 1 - pts[:, 0]  # x + y = 1 plane
        nrm = np.array([1.0, 1.0, 0]) / np.sqrt(2)
    elif sp is CC6:
        pts[:, 2] = pts[:, 0] - pts[:, 1]  # x - y - z = 0 plane
        nrm = np.array([1.0, -1.0, -1.0]) / np.sqrt(3)
    elif sp is BCC7:
        pts[:, 2] = np.round(pts[:, 2])  # z in Z
        nrm = np.array([0, 0, 1.0])
    elif sp is TRICUBIC:
        pts[:, 0] = np.round(pts[:, 0])
        nrm = np.array([1.0, 0, 0])
    elif sp is BCC8:
        pts[:, 1] = pts[:, 0]  # x - y = 0 plane
        nrm = np.array([1.0, -1.0, 0]) / np.sqrt(2)
    elif sp is FCC6:
        pts[:, 2] = 1 - pts[:, 0] - pts[:, 1]  # x + y + z = 1 plane
        nrm = np.ones(3) / np.sqrt(3)
    else:
        pts[:, 1] = pts[:, 0] + 0.0  # x0 - x1 = 0 plane... a ZP knot line
        nrm = np.array([1.0, -1.0]) / np.sqrt(2)
    a, ga = oracle.phi(sp, pts + eps * nrm, grad=True)
    b, gb = oracle.phi(sp, pts - eps * nrm, grad=True)
    assert np.abs(a - b).max() < 1e-6
    if order >= 1:
        assert np.abs(ga - gb).max() < 1e-5
    if order >= 2:
        # f = phi(x - n0) from a single unit coefficient, away from the edges
        E = _ext(sp, 9)
        n0 = np.full(3, 4 * sp.D[0])
        coeffs = [np.zeros((E, E, E)) for _ in range(sp.n_cosets)]
        coeffs[0][4, 4, 4] = 1.0
        _, _, Ha = oracle.evaluate_hessian(sp, (E,) * 3, coeffs, n0 + pts + 1e-6 * nrm)
        _, _, Hb = oracle.evaluate_hessian(sp, (E,) * 3, coeffs, n0 + pts - 1e-6 * nrm)
        assert np.abs(Ha - Hb).max() < 1e-4


@pytest.mark.parametrize("sp", SPL3 + [BCC4, TRILINEAR, TRIQUADRATIC])
def test_continuous_where_knot_planes_meet(sp):
    """Every spline here is at least C^0, so phi on edges and vertices of the
    knot-plane arrangement (two or three coordinates on half-integers, where
    faces of the recurrence's parallelepipeds coincide) equals phi a
    distance 1e-9 away."""
    y = rng.uniform(-2.5, 2.5, (300, 3))
    for k in range(300):
        cols = rng.choice(3, size=2 + k % 2, replace=False)
        y[k, cols] = np.round(2 * y[k, cols]) / 2
    d = rng.normal(size=y.shape)
    d *= 1e-9 / np.linalg.norm(d, axis=1, keepdims=True)
    np.testing.assert_allclose(oracle.phi(sp, y), oracle.phi(sp, y + d), atol=1e-7)


# ------------------------------------------------------ enumeration, grads

@pytest.mark.parametrize("sp", SPL3 + [ZP])
def test_pruned_equals_brute_force(sp):
    E = _ext(sp, 6 if sp.D.max() > 1 else 9)
    dims = (E,) * sp.s
    coeffs = [rng.uniform(-1, 1, tuple(dims[::-1])) for _ in range(sp.n_cosets)]
    hi = (E - 1) * sp.D.max() + 1
    x = rng.uniform(-2, hi + 2, (40, sp.s))  # includes boundary and outside points
    f1 = oracle.evaluate(sp, dims, coeffs, x)
    f2 = oracle.evaluate(sp, dims, coeffs, x, brute=True)
    assert np.array_equal(f1, f2)


@pytest.mark.parametrize("sp", SPL3)
def test_gradient_matches_central_differences(sp):
    E = _ext(sp, 8)
    dims = (E,) * 3
    coeffs = [rng.uniform(-1, 1, (E, E, E)) for _ in range(sp.n_cosets)]
    x = _interior(sp, E, 20)
    _, g = oracle.evaluate(sp, dims, coeffs, x, grad=True)
    h = 1e-4
    fd = np.zeros_like(g)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd[:, a] = (oracle.evaluate(sp, dims, coeffs, x + e) - oracle.evaluate(sp, dims, coeffs, x - e)) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=1e-6)


@pytest.mark.parametrize("sp", SPL3)
def test_gradient_exact_for_affine_data(sp):
    E = _ext(sp, 8)
    dims = (E,) * 3
    pos = oracle.site_positions(sp, dims).astype(np.float64)
    a = np.array([0.3, -1.1, 0.45])
    coeffs = [c.reshape(E, E, E) for c in (pos @ a - 2.0).reshape(sp.n_cosets, -1)]
    x = _interior(sp, E, 20)
    _, g = oracle.evaluate(sp, dims, coeffs, x, grad=True)
    np.testing.assert_allclose(g, np.broadcast_to(a, g.shape), atol=1e-12)


@pytest.mark.parametrize("sp", SPL3)
def test_backward_coef_fd_and_moments(sp):
    """MSE loss is quadratic in c, so central differences in c are exact."""
    E = _ext(sp, 7)
    dims = (E,) * 3
    coeffs = [rng.uniform(-1, 1, (E, E, E)) for _ in range(sp.n_cosets)]
    x = _interior(sp, E, 60)
    target = rng.uniform(-1, 1, len(x))

    def loss(cs):
        f = oracle.evaluate(sp, dims, cs, x)
        return 0.5 * np.sum((f - target) ** 2)

    f = oracle.evaluate(sp, dims, coeffs, x)
    g = f - target
    dc = oracle.backward(sp, dims, x, g)
    flat = np.concatenate([d.reshape(-1) for d in dc])
    # sum rules: sum_n dL/dc_n = sum g, sum_n n dL/dc_n = sum g x
    pos = oracle.site_positions(sp, dims).astype(np.float64)
    np.testing.assert_allclose(flat.sum(), g.sum(), atol=1e-11)
    np.testing.assert_allclose(pos.T @ flat, x.T @ g, atol=1e-10)
    # exact central differences at a few sites with nonzero gradient
    nz = np.flatnonzero(np.abs(flat) > 1e-3)
    for k in rng.choice(nz, size=4, replace=False):
        m, r = divmod(int(k), E ** 3)
        h = 0.25
        cp = [c.copy() for c in coeffs]
        cm = [c.copy() for c in coeffs]
        cp[m].reshape(-1)[r] += h
        cm[m].reshape(-1)[r] -= h
        fd = (loss(cp) - loss(cm)) / (2 * h)
        assert abs(fd - flat[k]) < 1e-10 * max(1.0, abs(fd))


def test_backward_x_is_g_times_grad():
    sp = BCC8
    E = _ext(sp, 7)
    dims = (E,) * 3
    coeffs = [rng.uniform(-1, 1, (E, E, E)) for _ in range(2)]
    x = _interior(sp, E, 10)
    g = rng.normal(size=len(x))
    dx = oracle.backward_x(sp, dims, coeffs, x, g)
    _, gr = oracle.evaluate(sp, dims, coeffs, x, grad=True)
    np.testing.assert_allclose(dx, g[:, None] * gr, atol=1e-15)


# ------------------------------------------------------------ Hessians

HESS = [TRICUBIC, BCC8, FCC6, TRIQUADRATIC, CC7, BCC7, CC6]   # C^1 and smoother after removing a direction


def test_tricubic_hessian_closed_form():
    """phi's Hessian for the tensor-product cubic B-spline: products of the
    textbook first and second derivatives of the centred cubic B-spline."""
    def d1(t):
        a = np.abs(t)
        return np.sign(t) * np.where(a <= 1, -2 * a + 1.5 * a ** 2, np.where(a <= 2, -0.5 * (2 - a) ** 2, 0))

    def d2(t):
        a = np.abs(t)
        return np.where(a <= 1, -2 + 3 * a, np.where(a <= 2, 2 - a, 0))

    E = 9
    dims = (E,) * 3
    coeffs = [np.zeros((E, E, E))]
    coeffs[0][4, 4, 4] = 1.0          # phi(x - n), n = (4, 4, 4)
    y = rng.uniform(-2.3, 2.3, (300, 3))
    _, _, H = oracle.evaluate_hessian(TRICUBIC, dims, coeffs, y + 4.0)
    b = [beta3(y[:, i]) for i in range(3)]
    g = [d1(y[:, i]) for i in range(3)]
    h = [d2(y[:, i]) for i in range(3)]
    ref = np.zeros((y.shape[0], 3, 3))
    for i in range(3):
        for j in range(3):
            f = [b[0], b[1], b[2]]
            if i == j:
                f[i] = h[i]
            else:
                f[i], f[j] = g[i], g[j]
            ref[:, i, j] = f[0] * f[1] * f[2]
    np.testing.assert_allclose(H, ref, atol=1e-12)


@pytest.mark.parametrize("sp", HESS)
def test_hessian_symmetric_and_matches_gradient_differences(sp):
    E = _ext(sp, 8)
    dims = (E,) * 3
    coeffs = [rng.uniform(-1, 1, (E, E, E)) for _ in range(sp.n_cosets)]
    x = _interior(sp, E, 20)
    f, g, H = oracle.evaluate_hessian(sp, dims, coeffs, x)
    f0, g0 = oracle.evaluate(sp, dims, coeffs, x, grad=True)
    np.testing.assert_allclose(f, f0, atol=1e-14)
    np.testing.assert_allclose(g, g0, atol=1e-13)
    np.testing.assert_allclose(H, H.transpose(0, 2, 1), atol=1e-12)
    h = 1e-5
    fd = np.zeros_like(H)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd[:, :, a] = (oracle.evaluate(sp, dims, coeffs, x + e, grad=True)[1]
                       - oracle.evaluate(sp, dims, coeffs, x - e, grad=True)[1]) / (2 * h)
    np.testing.assert_allclose(H, fd, atol=1e-7)


@pytest.mark.parametrize("sp", HESS)
def test_hessian_exact_for_quadratic_data(sp):
    """c_n = n^T Q n + b.n + a gives f = q(x) + const for these splines
    (quadratics are reproduced up to the second-moment constant), so the
    Hessian is exactly 2Q."""
    E = _ext(sp, 10)
    dims = (E,) * 3
    pos = oracle.site_positions(sp, dims).astype(np.float64)
    Q = np.array([[0.3, -0.1, 0.05], [-0.1, -0.2, 0.15], [0.05, 0.15, 0.4]])
    b = np.array([0.2, -0.3, 0.1])
    vals = np.einsum("ni,ij,nj->n", pos, Q, pos) + pos @ b + 1.0
    coeffs = [c.reshape(E, E, E) for c in vals.reshape(sp.n_cosets, -1)]
    x = _interior(sp, E, 30)
    _, _, H = oracle.evaluate_hessian(sp, dims, coeffs, x)
    np.testing.assert_allclose(H, np.broadcast_to(2 * Q, H.shape), atol=1e-10)


def test_hessian_refused_for_c0_splines():
    """Removing two directions of the trilinear / linear BCC splines stops
    them spanning: no classical Hessian, and the oracle says so."""
    E = 6
    for sp in (TRILINEAR, BCC4):
        coeffs = [np.ones((E, E, E)) for _ in range(sp.n_cosets)]
        with pytest.raises(RuntimeError):
            oracle.evaluate_hessian(sp, (E,) * 3, coeffs, np.full((1, 3), 5.3))
