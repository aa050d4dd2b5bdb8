// Point location, symmetry transform and stencil addressing (Sec. 4.1.2 to
// Sec. 4.2, Algorithm 1): everything a query point needs before the
// coefficient fetches.  Written as __host__ __device__ so the host library can
// run the same arithmetic for its bounds diagnostics.
//
// Internal coefficient layout: the per-coset grids, each surrounded by a zero
// halo of `pad` sites, are interleaved (all cosets of one index idx are
// adjacent) and cut into bricks of 2^lb[0] x 2^lb[1] x 2^lb[2] indices, so
// that the few cache lines a stencil touches hold as many of its taps as
// possible.  With i = idx + pad (non-negative), the byte offset of site idx
// in coset m is separable per axis:
//     m * es + sum_a f_a(i_a),   f_a(i) = (i >> lb[a]) * bs[a] + (i & (2^lb[a] - 1)) * is[a]
// Every brick and every site are powers of two bytes, so is[a] = 2^lis[a]
// and bs[a] = nbs[a] * 2^lbb with nbs the brick-count stride (< 2^24); the
// kernels form sum_a (i_a >> lb[a]) * nbs[a] with 24-bit multiplies and one
// shift.
// where idx = floor((n - shift_m) / D).  For D = 2 lattices floor(n/2)
// equals (n - shift_m)/2 for the coset the site belongs to.
#pragma once

#include <stdint.h>

#ifndef __HIP_DEVICE_COMPILE__
#include <math.h>
#endif

#include "generated/all.h"

#ifndef LSP_HD
#define LSP_HD __host__ __device__ __forceinline__
#endif

namespace lsp {

// Spline kinds, in the order of the generated kind table (generated/all.h).
enum Kind : int {
    kTricubic = 0, kBcc8 = 1, kFcc6 = 2, kTrilinear = 3, kBcc4 = 4, kTriquadratic = 5, kCc7 = 6, kBcc7 = 7,
    kCc6 = 8
};
static_assert(gen::kNumKinds == 9, "kind table and Kind enum disagree");

// Expands X(k) for every spline kind (compile-time dispatch).
#define LSP_FOR_EACH_KIND(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

template <int KIND> using TablesOf = typename gen::SplineOf<KIND>::T;
template <int KIND> using PolyOf = typename gen::SplineOf<KIND>::P;

enum Lattice : int { kLatCC = 0, kLatBCC = 1, kLatFCC = 2 };
enum Roe : int { kRoeFloor = 0, kRoeRound = 1, kRoeVoronoi = 2 };
enum Sym : int { kSymNone = 0, kSymSigns = 1, kSymSignedPerm = 2 };

// Geometry of one volume as the kernels see it.  Strides are in bytes.
struct VolGeom {
    int es;                 // bytes per coefficient
    int pad;                // halo in coset units
    int kmin[3], kmax[3];   // ROE lattice points k with any stored tap
    int lb[3];              // log2 of the brick extent per axis
    int nbs[3];             // bricks between neighbouring bricks along each axis
    int lis[3];             // log2 of the bytes between neighbouring sites in a brick
    int lbb;                // log2 of the bytes per brick
};

// 24-bit products (full-rate on the GPU); operands are below 2^24 here.
LSP_HD int mul24u(int a, int b) {
#ifdef __HIP_DEVICE_COMPILE__
    return (int)__umul24((unsigned)a, (unsigned)b);
#else
    return a * b;
#endif
}
LSP_HD int mul24s(int a, int b) {
#ifdef __HIP_DEVICE_COMPILE__
    return __mul24(a, b);
#else
    return a * b;
#endif
}

// Brick part (in bricks) and in-brick part (in bytes) of one axis.
LSP_HD int brick_term(int i, int lb, int nbs) { return mul24u(i >> lb, nbs); }
LSP_HD int inner_term(int i, int lb, int lis) { return (i & ((1 << lb) - 1)) << lis; }

LSP_HD int site_offset(const VolGeom& g, const int i[3], int coset) {
    int br = 0, in = 0;
    for (int a = 0; a < 3; ++a) {
        br += brick_term(i[a], g.lb[a], g.nbs[a]);
        in += inner_term(i[a], g.lb[a], g.lis[a]);
    }
    return (br << g.lbb) + in + coset * g.es;
}

// Result of locating one point.
struct Loc {
    float y[3];        // coordinates in the reference sub-region frame
    int bidx[2][3];    // padded index origin per reference axis, for even / odd offsets
    int cb[4];         // coset byte offset per tap parity class
    int s[3];          // +-1: reflection of each reference axis
    int lb[3], nbs[3], lis[3];  // layout of the global axis behind each reference axis
    int lbb;           // log2 of the bytes per brick
    int axis[3];       // global axis of each reference axis
    float sgn[3];      // sign of each reference axis (reflection)
    int region;        // reference sub-region (polynomial) index
    int k[3];          // the ROE lattice point (origin for inactive points)
    bool active;       // some stencil tap lies in the stored lattice
    bool nan;          // a coordinate was NaN
};

// The layout is wave-uniform: on the device the per-axis values are taken
// into scalar registers first, so that the per-lane choice below is a
// register select and never becomes a per-lane load from the kernel
// arguments (a dependent memory round trip ahead of every gather).
LSP_HD int uniform_int(int v) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_readfirstlane(v);
#else
    return v;
#endif
}

LSP_HD void set_axis_layout(const VolGeom& g, Loc& L) {
    int lb[3], nbs[3], lis[3];
    for (int a = 0; a < 3; ++a) {
        lb[a] = uniform_int(g.lb[a]);
        nbs[a] = uniform_int(g.nbs[a]);
        lis[a] = uniform_int(g.lis[a]);
    }
    for (int r = 0; r < 3; ++r) {
        const int a = L.axis[r];
        L.lb[r] = a == 0 ? lb[0] : (a == 1 ? lb[1] : lb[2]);
        L.nbs[r] = a == 0 ? nbs[0] : (a == 1 ? nbs[1] : nbs[2]);
        L.lis[r] = a == 0 ? lis[0] : (a == 1 ? lis[1] : lis[2]);
    }
    L.lbb = g.lbb;
}

// Coordinates are clamped to +-2^22 before rounding so the integer
// conversions below stay defined; such points are outside any volume.
#define LSP_XCLAMP 4194304.0

template <class PT>
LSP_HD PT clampc(PT v) {
    return v < (PT)-LSP_XCLAMP ? (PT)-LSP_XCLAMP : (v > (PT)LSP_XCLAMP ? (PT)LSP_XCLAMP : v);
}

LSP_HD float fl_floor(float v) { return floorf(v); }
LSP_HD double fl_floor(double v) { return floor(v); }
LSP_HD float fl_rint(float v) { return rintf(v); }
LSP_HD double fl_rint(double v) { return rint(v); }
LSP_HD bool is_nan(float v) { return v != v; }
LSP_HD bool is_nan(double v) { return v != v; }

template <class PT>
LSP_HD void finish_common(const PT x[3], const PT k[3], const VolGeom& g, Loc& L, int ki[3],
                          float d[3]) {
    L.nan = is_nan(x[0]) || is_nan(x[1]) || is_nan(x[2]);
    bool act = !L.nan;
    for (int a = 0; a < 3; ++a) {
        ki[a] = (int)k[a];
        act = act && ki[a] >= g.kmin[a] && ki[a] <= g.kmax[a];
    }
    L.active = act;
    for (int a = 0; a < 3; ++a) {
        // inactive points take the ROE of the origin (a site of every
        // lattice here) so that every fetch stays inside the buffer
        d[a] = act ? (float)(x[a] - k[a]) : 0.0f;
        if (!act) ki[a] = 0;
        L.k[a] = ki[a];
    }
}

// Symmetry element of a located point in the encoding of the generated
// transposed-stencil tables: 0 without symmetry; the sign bits (bit r set when
// reference axis r is reflected) for reflections only; and
// (axis[0] * 3 + axis[1]) * 8 + sign bits for signed permutations.
template <int KIND>
LSP_HD int sym_id(const Loc& L) {
    constexpr int S = TablesOf<KIND>::kSymmetry;
    if (S == kSymNone) return 0;
    const int bits = (L.sgn[0] < 0.0f ? 1 : 0) | (L.sgn[1] < 0.0f ? 2 : 0) | (L.sgn[2] < 0.0f ? 4 : 0);
    if (S == kSymSigns) return bits;
    return (L.axis[0] * 3 + L.axis[1]) * 8 + bits;
}

// The signed permutation y = sort_desc(|x - k|) (Sec. 4.1.3): a 3-comparator
// network, descending by |d|, carrying each axis' index origins (even / odd
// offsets), global axis and sign into the reference frame.
LSP_HD void signed_perm_to_loc(float m[3], int b0[3], int b1[3], int ax[3], float sg[3], Loc& L) {
#define LSP_CSWAP(i, j)                                                           \
    {                                                                             \
        const bool sw = m[i] < m[j];                                              \
        const float tm = sw ? m[j] : m[i], um = sw ? m[i] : m[j];                 \
        const int t0 = sw ? b0[j] : b0[i], u0 = sw ? b0[i] : b0[j];               \
        const int t1 = sw ? b1[j] : b1[i], u1 = sw ? b1[i] : b1[j];               \
        const int ta = sw ? ax[j] : ax[i], ua = sw ? ax[i] : ax[j];               \
        const float ts = sw ? sg[j] : sg[i], us = sw ? sg[i] : sg[j];             \
        m[i] = tm; m[j] = um; b0[i] = t0; b0[j] = u0; b1[i] = t1; b1[j] = u1;     \
        ax[i] = ta; ax[j] = ua; sg[i] = ts; sg[j] = us;                           \
    }
    LSP_CSWAP(0, 1)
    LSP_CSWAP(1, 2)
    LSP_CSWAP(0, 1)
#undef LSP_CSWAP
    for (int r = 0; r < 3; ++r) {
        L.y[r] = m[r];
        L.bidx[0][r] = b0[r];
        L.bidx[1][r] = b1[r];
        L.axis[r] = ax[r];
        L.sgn[r] = sg[r];
        L.s[r] = sg[r] < 0.0f ? -1 : 1;
    }
}

// Z^3 with a parallelepiped ROE (Sec. 4.1.2): the unit cube [0,1)^3 via
// floor, or the centred cube [-1/2,1/2)^3 via floor(x + 1/2).  Without
// symmetry the cube is the sub-region; with signed permutations (SORTED)
// y = sort_desc(|x - k|) lands in the wedge 0 <= y2 <= y1 <= y0 <= 1/2.
template <class PT, bool CENTRED, bool SORTED>
LSP_HD void locate_cc(const PT xin[3], const VolGeom& g, Loc& L) {
    PT x[3], k[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = is_nan(xin[a]) ? xin[a] : clampc(xin[a]);
        k[a] = is_nan(x[a]) ? (PT)0 : fl_floor(CENTRED ? x[a] + (PT)0.5 : x[a]);
    }
    int ki[3];
    float d[3];
    finish_common(x, k, g, L, ki, d);
    if (SORTED) {
        float m[3], sg[3];
        int b0[3], b1[3], ax[3];
        for (int a = 0; a < 3; ++a) {
            const bool neg = d[a] < 0.0f;
            b0[a] = b1[a] = ki[a] + g.pad;
            m[a] = neg ? -d[a] : d[a];
            sg[a] = neg ? -1.0f : 1.0f;
            ax[a] = a;
        }
        signed_perm_to_loc(m, b0, b1, ax, sg, L);
    } else {
        for (int a = 0; a < 3; ++a) {
            L.bidx[0][a] = L.bidx[1][a] = ki[a] + g.pad;
            L.y[a] = d[a];
            L.s[a] = 1;
            L.axis[a] = a;
            L.sgn[a] = 1.0f;
        }
    }
    L.cb[0] = L.cb[1] = L.cb[2] = L.cb[3] = 0;
    set_axis_layout(g, L);
    L.region = 0;
}

// BCC lattice 2Z^3 u (2Z^3 + 1): Voronoi ROE (nearest lattice point: the
// nearer of the nearest even and the nearest odd point), then the signed
// permutation y = sort_desc(|x - k|) into the reference wedge
// 0 <= y2 <= y1 <= y0 (Sec. 4.1.2, 4.1.3, Fig. 1's transform column).
template <class PT>
LSP_HD void locate_bcc(const PT xin[3], const VolGeom& g, Loc& L) {
    PT x[3], ke[3], ko[3], k[3];
    PT de = 0, dodd = 0;
    for (int a = 0; a < 3; ++a) {
        x[a] = is_nan(xin[a]) ? (PT)0 : clampc(xin[a]);
        ke[a] = (PT)2 * fl_rint(x[a] * (PT)0.5);
        ko[a] = (PT)2 * fl_rint((x[a] - (PT)1) * (PT)0.5) + (PT)1;
        de += (x[a] - ke[a]) * (x[a] - ke[a]);
        dodd += (x[a] - ko[a]) * (x[a] - ko[a]);
    }
    const bool odd = dodd < de;
    for (int a = 0; a < 3; ++a) k[a] = odd ? ko[a] : ke[a];
    PT xr[3] = {xin[0], xin[1], xin[2]};
    for (int a = 0; a < 3; ++a) if (!is_nan(xr[a])) xr[a] = x[a];
    int ki[3];
    float d[3];
    finish_common(xr, k, g, L, ki, d);
    const int q = ki[0] & 1;
    float m[3];
    int b0[3], b1[3], ax[3];
    float sg[3];
    for (int a = 0; a < 3; ++a) {
        const int K = ki[a] >> 1;   // floor(k/2)
        const bool neg = d[a] < 0.0f;
        b0[a] = K + g.pad;                          // even offsets: floor((k + s o)/2) = K + s o/2
        b1[a] = K + g.pad + q - (neg ? 1 : 0);      // odd offsets:  K + q - [s < 0] + s floor(o/2)
        m[a] = neg ? -d[a] : d[a];
        sg[a] = neg ? -1.0f : 1.0f;
        ax[a] = a;
    }
    signed_perm_to_loc(m, b0, b1, ax, sg, L);
    L.cb[0] = q * g.es;         // taps with all-even offsets stay in the coset of k
    L.cb[1] = (1 - q) * g.es;   // taps with all-odd offsets are in the other coset
    L.cb[2] = L.cb[3] = L.cb[0];
    set_axis_layout(g, L);
    L.region = 0;
}

// Coset index of an FCC parity pattern (bit0 x, bit1 y, bit2 z):
// 000 -> 0, 110 -> 1, 101 -> 2, 011 -> 3 (the order of the coset shifts).
LSP_HD int fcc_coset(int p) { return (14400 >> (2 * p)) & 3; }

// Index of an FCC tap parity pattern among {000, 110, 101, 011}.
LSP_HD constexpr int fcc_class(int p) { return p == 0 ? 0 : (p == 3 ? 1 : (p == 5 ? 2 : 3)); }

// FCC lattice {n : sum n even}: Voronoi ROE by rounding every coordinate and,
// when the sum is odd, re-rounding the coordinate with the largest residual
// the other way (Conway and Sloane's decoder for D3); the reflections
// y = |x - k| map into the positive octant, where the plane
// y0 + y1 + y2 = 1 splits the two reference sub-regions.
template <class PT>
LSP_HD void locate_fcc(const PT xin[3], const VolGeom& g, Loc& L) {
    PT x[3], k[3], res[3];
    int par = 0;
    for (int a = 0; a < 3; ++a) {
        x[a] = is_nan(xin[a]) ? (PT)0 : clampc(xin[a]);
        k[a] = fl_rint(x[a]);
        res[a] = x[a] - k[a];
        par += (int)k[a];
    }
    PT ar[3];
    for (int a = 0; a < 3; ++a) ar[a] = res[a] < (PT)0 ? -res[a] : res[a];
    const int j = (ar[0] >= ar[1]) ? ((ar[0] >= ar[2]) ? 0 : 2) : ((ar[1] >= ar[2]) ? 1 : 2);
    if (par & 1) {
        for (int a = 0; a < 3; ++a)
            if (a == j) k[a] += res[a] >= (PT)0 ? (PT)1 : (PT)-1;
    }
    PT xr[3] = {xin[0], xin[1], xin[2]};
    for (int a = 0; a < 3; ++a) if (!is_nan(xr[a])) xr[a] = x[a];
    int ki[3];
    float d[3];
    finish_common(xr, k, g, L, ki, d);
    const int q = (ki[0] & 1) | ((ki[1] & 1) << 1) | ((ki[2] & 1) << 2);
    const int pats[4] = {0, 3, 5, 6};
    for (int a = 0; a < 3; ++a) {
        const bool neg = d[a] < 0.0f;
        const int K = ki[a] >> 1;
        L.bidx[0][a] = K + g.pad;                                   // even component of o
        L.bidx[1][a] = K + g.pad + ((q >> a) & 1) - (neg ? 1 : 0);  // odd component of o
        L.y[a] = neg ? -d[a] : d[a];
        L.s[a] = neg ? -1 : 1;
        L.sgn[a] = neg ? -1.0f : 1.0f;
        L.axis[a] = a;
    }
    for (int c = 0; c < 4; ++c) L.cb[c] = fcc_coset(q ^ pats[c]) * g.es;
    set_axis_layout(g, L);
    L.region = 0;
}

// Region of evaluation, symmetry transform and reference sub-region of a
// point for the spline KIND (the preamble of Algorithm 1 up to the table
// lookups): several reference sub-regions are told apart by the generated
// plane tests.
template <int KIND, class PT>
LSP_HD void locate(const PT x[3], const VolGeom& g, Loc& L) {
    using T = TablesOf<KIND>;
    if (T::kLattice == kLatCC) {
        constexpr bool SORTED = T::kSymmetry == kSymSignedPerm;
        if (T::kRoe == kRoeRound) locate_cc<PT, true, SORTED>(x, g, L);
        else locate_cc<PT, false, SORTED>(x, g, L);
    } else if (T::kLattice == kLatBCC) {
        locate_bcc(x, g, L);
    } else {
        locate_fcc(x, g, L);
    }
    if constexpr (T::kRegions > 1) L.region = PolyOf<KIND>::region(L.y[0], L.y[1], L.y[2]);
}

// Byte offset of the tap with reference-frame offset o (a lattice vector)
// and parity pattern par: along each reference axis r the padded index is the
// origin for the parity of o_r plus s_r * floor(o_r / D); the per-axis terms
// of the separable layout are summed and the coset of the tap added.
template <int KIND>
LSP_HD int tap_offset(const Loc& L, int o0, int o1, int o2, int par) {
    constexpr int LAT = TablesOf<KIND>::kLattice;
    const int o[3] = {o0, o1, o2};
    // For stencils of more than 32 taps each axis contributes its brick and
    // in-brick bytes as one term, which depends only on that axis' offset
    // component: with the offsets known at compile time the terms are shared
    // by every tap with the same component and a tap costs one three-way add
    // plus its coset (measured on MI355X: 9% faster for the 53-tap spline,
    // 6% for the 38-tap one; the smaller stencils run faster with the brick
    // and in-brick sums kept apart).
    constexpr bool FOLD = TablesOf<KIND>::kTaps > 32;
    int br = 0, in = 0, off = 0;
    for (int r = 0; r < 3; ++r) {
        int i;
        if (LAT == kLatCC)
            i = L.bidx[0][r] + (TablesOf<KIND>::kSymmetry == kSymNone ? o[r] : mul24s(L.s[r], o[r]));
        else if (LAT == kLatBCC) i = L.bidx[par ? 1 : 0][r] + mul24s(L.s[r], o[r] >> 1);
        else i = L.bidx[o[r] & 1][r] + mul24s(L.s[r], o[r] >> 1);
        if (FOLD) {
            off += (brick_term(i, L.lb[r], L.nbs[r]) << L.lbb) + inner_term(i, L.lb[r], L.lis[r]);
        } else {
            br += brick_term(i, L.lb[r], L.nbs[r]);
            in += inner_term(i, L.lb[r], L.lis[r]);
        }
    }
    const int cls = (LAT == kLatCC) ? 0 : ((LAT == kLatBCC) ? (par ? 1 : 0) : fcc_class(par));
    return (FOLD ? off : (br << L.lbb) + in) + L.cb[cls];
}

// Coset index of a lattice site from the parities of its coordinates.
template <int KIND>
LSP_HD int coset_of_parity(int p0, int p1, int p2) {
    constexpr int LAT = TablesOf<KIND>::kLattice;
    if (LAT == kLatCC) return 0;
    if (LAT == kLatBCC) return p0;
    return fcc_coset(p0 | (p1 << 1) | (p2 << 2));
}

}  // namespace lsp
