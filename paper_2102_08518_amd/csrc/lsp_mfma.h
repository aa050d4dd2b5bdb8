// Matrix-core evaluation of a spline with one reference sub-region.
//
// After the symmetry transform (Sec. 4.2) every point evaluates the same
// reference polynomial, whose monomial coefficients are a constant linear map
// of the point's own stencil values: A = W c (monomials x taps).  Over a
// wavefront this is the product of one constant matrix with the 32 x 64
// matrix of gathered coefficients (one column per lane), which the matrix
// cores evaluate with v_mfma_f32_32x32x16_{bf16,f16}:
//   * the generator scales W by the least common denominator Q of its
//     entries; Wq = Q W is an integer matrix whose entries are exact in bf16
//     and fp16 (checked when the tables are generated);
//   * FP32 coefficients are split exactly into three bf16 parts
//     c = c0 + c1 + c2 (the top, middle and low 8 significand bits), so every
//     product Wq_mj c_j is exact and only the FP32 accumulation rounds; bf16
//     and fp16 coefficients go in as stored (one pass);
//   * the B operand of a 32x32 MFMA holds 32 points, split over the two lane
//     halves by K.  One v_permlane32_swap per operand dword turns "each lane
//     holds all taps of its own point" into that layout for the two 32-point
//     groups of the wavefront, and one swap per result dword turns the
//     results back, so each lane ends with all rows of A for its own point;
//   * the polynomial in A is then evaluated per lane in Horner form.
// Per point this replaces the ~800 FMAs of W c with about 200 VALU
// operations of operand preparation.
#pragma once

#include "lsp_kernels.h"

namespace lsp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

template <int KIND> using MfmaOf = typename gen::SplineOf<KIND>::M;

// The matrix-core path is used for splines whose polynomial has a Wq form and
// more than 16 taps (below that the per-lane FMAs are already few).
template <int KIND>
constexpr bool mfma_eligible() {
    if constexpr (MfmaOf<KIND>::kOk) return TablesOf<KIND>::kTaps > 16;
    return false;
}

// One 32x32x16 product: bf16 operands for FP32 and bf16 coefficients, fp16
// for fp16 coefficients.
template <class CT> struct MfmaOp {
    static __device__ __forceinline__ f32x16_t run(u32x4_t a, u32x4_t b, f32x16_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                      __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
    }
    // 16-bit encoding of a small integer (exact)
    static __device__ __forceinline__ unsigned enc(int v) {
        return __builtin_bit_cast(unsigned, (float)v) >> 16;
    }
};
template <> struct MfmaOp<f16_t> {
    static __device__ __forceinline__ f32x16_t run(u32x4_t a, u32x4_t b, f32x16_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a),
                                                     __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ unsigned enc(int v) {
        return (unsigned)__builtin_bit_cast(unsigned short, (_Float16)(float)v);
    }
};

// v_permlane32_swap: lanes 32..63 of a trade places with lanes 0..31 of b.
// (The results are copied out element by element: a bit cast applied to a
// vector subscript expression reads element 0 instead.)
__device__ __forceinline__ void swap_halves(unsigned& a, unsigned& b) {
    const auto sw = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    const unsigned x = sw[0];
    const unsigned y = sw[1];
    a = x;
    b = y;
}

// Low half: top 16 bits of a; high half: top 16 bits of b.
__device__ __forceinline__ unsigned pack_hi16(unsigned a, unsigned b) {
    return __builtin_amdgcn_perm(b, a, 0x07060302u);
}

// A operand for row tile t, K-step s: lane l holds Wq[32t + l%32][16s + 8(l/32) + j],
// j = 0..7, as packed 16-bit pairs.  The weights are small integers.
template <int KIND, class CT>
__device__ __forceinline__ u32x4_t weight_operand(int t, int s, int lane) {
    using M = MfmaOf<KIND>;
    const int row = 32 * t + (lane & 31);
    const int col = 16 * s + 8 * (lane >> 5);
    u32x4_t w;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const unsigned lo = MfmaOp<CT>::enc(M::kWq[row][col + 2 * q]);
        const unsigned hi = MfmaOp<CT>::enc(M::kWq[row][col + 2 * q + 1]);
        w[q] = lo | (hi << 16);
    }
    return w;
}

// The point's stencil values (byte offsets off[0..NTAP), zero beyond) as
// packed 16-bit pairs: for FP32 coefficients the exact three-way bf16 split
// into parts 0..2, else the stored encoding.
template <class CT> struct StencilParts;
template <> struct StencilParts<float> {
    static constexpr int kParts = 3;
    template <int NT, int NTAP>
    static __device__ __forceinline__ void build(__amdgpu_buffer_rsrc_t r, const int* off,
                                                 unsigned (*v)[NT / 2]) {
#pragma unroll
        for (int j = 0; j < NT; j += 2) {
            unsigned u0[2], u1[2], u2[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const unsigned u = j + e < NTAP ? __builtin_amdgcn_raw_buffer_load_b32(r, off[j + e], 0, 0) : 0u;
                const float c = __builtin_bit_cast(float, u);
                const float r1 = c - __builtin_bit_cast(float, u & 0xffff0000u);
                const unsigned v1 = __builtin_bit_cast(unsigned, r1);
                const float r2 = r1 - __builtin_bit_cast(float, v1 & 0xffff0000u);
                u0[e] = u;
                u1[e] = v1;
                u2[e] = __builtin_bit_cast(unsigned, r2);
            }
            v[0][j / 2] = pack_hi16(u0[0], u0[1]);
            v[1][j / 2] = pack_hi16(u1[0], u1[1]);
            v[2][j / 2] = pack_hi16(u2[0], u2[1]);
        }
    }
};
template <class CT16> struct StencilParts16 {
    static constexpr int kParts = 1;
    template <int NT, int NTAP>
    static __device__ __forceinline__ void build(__amdgpu_buffer_rsrc_t r, const int* off,
                                                 unsigned (*v)[NT / 2]) {
#pragma unroll
        for (int j = 0; j < NT; j += 2) {
            const unsigned a = j < NTAP ? (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, off[j], 0, 0) : 0u;
            const unsigned b = j + 1 < NTAP ? (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, off[j + 1], 0, 0) : 0u;
            v[0][j / 2] = (a & 0xffffu) | (b << 16);
        }
    }
};
template <> struct StencilParts<bf16_t> : StencilParts16<bf16_t> {};
template <> struct StencilParts<f16_t> : StencilParts16<f16_t> {};

// The point's stencil values already in FP32 registers (zero beyond NTAP),
// packed the same way: FP32 coefficients split three ways, 16-bit ones
// re-encoded exactly (the FP32 values are conversions of them).
template <class CT> struct PackParts;
template <> struct PackParts<float> {
    template <int NT, int NTAP>
    static __device__ __forceinline__ void pack(const float* c, unsigned (*v)[NT / 2]) {
#pragma unroll
        for (int j = 0; j < NT; j += 2) {
            unsigned u0[2], u1[2], u2[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const float cj = j + e < NTAP ? c[j + e] : 0.0f;
                const unsigned u = __builtin_bit_cast(unsigned, cj);
                const float r1 = cj - __builtin_bit_cast(float, u & 0xffff0000u);
                const unsigned v1 = __builtin_bit_cast(unsigned, r1);
                const float r2 = r1 - __builtin_bit_cast(float, v1 & 0xffff0000u);
                u0[e] = u;
                u1[e] = v1;
                u2[e] = __builtin_bit_cast(unsigned, r2);
            }
            v[0][j / 2] = pack_hi16(u0[0], u0[1]);
            v[1][j / 2] = pack_hi16(u1[0], u1[1]);
            v[2][j / 2] = pack_hi16(u2[0], u2[1]);
        }
    }
};
template <> struct PackParts<bf16_t> {
    template <int NT, int NTAP>
    static __device__ __forceinline__ void pack(const float* c, unsigned (*v)[NT / 2]) {
#pragma unroll
        for (int j = 0; j < NT; j += 2) {
            const unsigned a = j < NTAP ? __builtin_bit_cast(unsigned, c[j]) : 0u;
            const unsigned b = j + 1 < NTAP ? __builtin_bit_cast(unsigned, c[j + 1]) : 0u;
            v[0][j / 2] = pack_hi16(a, b);
        }
    }
};
template <> struct PackParts<f16_t> {
    template <int NT, int NTAP>
    static __device__ __forceinline__ void pack(const float* c, unsigned (*v)[NT / 2]) {
#pragma unroll
        for (int j = 0; j < NT; j += 2) {
            const unsigned a = j < NTAP ? __builtin_bit_cast(unsigned short, (_Float16)c[j]) : 0u;
            const unsigned b = j + 1 < NTAP ? __builtin_bit_cast(unsigned short, (_Float16)c[j + 1]) : 0u;
            v[0][j / 2] = a | (b << 16);
        }
    }
};

// Matrix products, results back to one point per lane, polynomial and store
// for a located point whose packed stencil values are v.  Every lane of the
// wave executes this; lanes with valid == false store nothing.
template <int KIND, class CT, int MODE>
__device__ __forceinline__ void mfma_finish(const Loc& L, unsigned (*v)[16], int o, bool valid,
                                            const u32x4_t (&W)[2][2], float* __restrict__ out,
                                            float* __restrict__ grad) {
    using T = TablesOf<KIND>;
    using M = MfmaOf<KIND>;
    constexpr int NS = (T::kTaps + 15) / 16;      // K-steps used
    constexpr int NR = (M::kRows + 31) / 32;      // row tiles used
    constexpr int NP = StencilParts<CT>::kParts;

    // B operands: group 0 = points of lanes 0..31, group 1 = lanes 32..63.
    f32x16_t acc[2][NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        acc[0][t] = f32x16_t{};
        acc[1][t] = f32x16_t{};
    }
#pragma unroll
    for (int p = NP - 1; p >= 0; --p) {  // smallest part first
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            u32x4_t b0, b1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // each lane's own taps 16s+0..7 and 16s+8..15
                unsigned y = v[p][8 * s + q], x = v[p][8 * s + 4 + q];
                swap_halves(y, x);
                b0[q] = y;
                b1[q] = x;
            }
#pragma unroll
            for (int t = 0; t < NR; ++t) {
                acc[0][t] = MfmaOp<CT>::run(W[t][s], b0, acc[0][t]);
                acc[1][t] = MfmaOp<CT>::run(W[t][s], b1, acc[1][t]);
            }
        }
    }
    // Results back to one point per lane: register i of tile t holds row
    // 32t + 8(i/4) + 4h + i%4 for lane half h.
    float A[32 * NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float e0 = acc[0][t][i];
            const float e1 = acc[1][t][i];
            unsigned lo = __builtin_bit_cast(unsigned, e0), hi = __builtin_bit_cast(unsigned, e1);
            swap_halves(lo, hi);
            A[32 * t + 8 * (i / 4) + (i % 4)] = __builtin_bit_cast(float, lo);
            A[32 * t + 8 * (i / 4) + 4 + (i % 4)] = __builtin_bit_cast(float, hi);
        }
    }
    constexpr float invq = 1.0f / (float)M::kQ;
    const float qnan = __builtin_nanf("");
    const float fill = L.nan ? qnan : 0.0f;
    if (MODE == kValue) {
        const float f = M::value(A, L.y[0], L.y[1], L.y[2]) * invq;
        if (valid) out[o] = L.active ? f : fill;
    } else {
        float gr[3], gx[3];
        const float f = M::value_grad(A, L.y[0], L.y[1], L.y[2], gr[0], gr[1], gr[2]) * invq;
#pragma unroll
        for (int a = 0; a < 3; ++a) gr[a] *= invq;
        grad_to_global(L, gr, gx);
        if (valid) {
            if (out) out[o] = L.active ? f : fill;
#pragma unroll
            for (int a = 0; a < 3; ++a) grad[3 * (size_t)o + a] = L.active ? gx[a] : fill;
        }
    }
}

// One point per lane, taps gathered from the coefficient buffer.  Full
// wavefronts only: lanes without a point (valid == false) compute a dummy
// point and store nothing.  Results for the point x go to index o.
template <int KIND, class CT, class PT, int MODE>
__device__ __forceinline__ void eval_mfma_wave(const PT x[3], int o, bool valid,
                                               const u32x4_t (&W)[2][2],
                                               __amdgpu_buffer_rsrc_t r, const VolGeom& g,
                                               float* __restrict__ out, float* __restrict__ grad) {
    using T = TablesOf<KIND>;
    constexpr int NT = 32;  // taps padded to two K-steps
    constexpr int NP = StencilParts<CT>::kParts;
    Loc L;
    locate<KIND>(x, g, L);
    int off[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j)
        off[j] = j < T::kTaps ? tap_offset<KIND>(L, T::kOff[j][0], T::kOff[j][1], T::kOff[j][2],
                                                 T::kParity[j])
                              : 0;
    unsigned v[NP][NT / 2];
    StencilParts<CT>::template build<NT, T::kTaps>(r, off, v);
    mfma_finish<KIND, CT, MODE>(L, v, o, valid, W, out, grad);
}

template <int KIND, class CT>
__device__ __forceinline__ void load_weight_operands(u32x4_t (&W)[2][2]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s) W[t][s] = weight_operand<KIND, CT>(t, s, lane);
}

// Direct order: block b handles points [b * 256 * ppt, (b + 1) * 256 * ppt),
// 256 at a time.  blockDim.x == 256.
template <int KIND, class CT, class PT, int MODE>
__global__ __launch_bounds__(256) void k_eval_mfma(const PT* __restrict__ pts, int N, int ppt,
                                                   const void* __restrict__ coef, unsigned nbytes,
                                                   VolGeom g, float* __restrict__ out,
                                                   float* __restrict__ grad) {
    u32x4_t W[2][2];
    load_weight_operands<KIND, CT>(W);
    const __amdgpu_buffer_rsrc_t r = make_rsrc(coef, nbytes);
    const int wave_lane = threadIdx.x & 63;
    for (int it = 0; it < ppt; ++it) {
        const long long base = ((long long)blockIdx.x * ppt + it) * 256 + (threadIdx.x & ~63);
        if (base >= N) break;  // uniform over the wavefront
        const int p = (int)base + wave_lane;
        const bool valid = p < N;
        PT x[3] = {PT(0), PT(0), PT(0)};
        if (valid) load_point(pts, p, x);
        eval_mfma_wave<KIND, CT, PT, MODE>(x, p, valid, W, r, g, out, grad);
    }
}

}  // namespace lsp
