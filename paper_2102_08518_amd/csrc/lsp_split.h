// Several lanes per point for the separable (tensor-product) splines: for
// launches too small to fill the GPU with one lane per point, and for the
// tricubic spline at every size (its one-lane kernel needs registers for 64
// taps and runs at 4 waves per SIMD).
//
// A point's stencil is an S x S x S block (S = 2, 3, 4) whose union order
// runs x fastest, then y, then z, so the taps of z-slab l are
// [S*S*l, S*S*(l+1)).  Four lanes of one quad share a point: lane l < S
// gathers slab l and contracts it with the 1D weights of the point (the
// generated y-only phase, PolyOf<K>::pre), giving its part of f (and of the
// gradient); the quad then adds its four parts with two DPP quad
// permutations.  The per-lane work is a quarter of the one-lane kernel's, so
// four times as many wavefronts hide the gather latency.
// Results equal the one-lane kernel's up to the order of the final additions.
#pragma once

#include "lsp_kernels.h"

namespace lsp {

constexpr int kSplitLanes = 4;
// A launch holds fewer than 2^32 work-items, so the four-lanes-per-point
// kernels cover more than 2^29 points in launches of 2^29 points each.
constexpr int kSplitChunk = 1 << 29;

template <int KIND>
constexpr int split_extent() {
    using T = TablesOf<KIND>;
    if constexpr (!T::kTensor) return 0;
    return T::kTaps == 8 ? 2 : (T::kTaps == 27 ? 3 : (T::kTaps == 64 ? 4 : 0));
}

template <int KIND>
constexpr bool split_eligible() {
    return split_extent<KIND>() > 0;
}

// Default largest point count for four lanes per point, measured on MI355X
// (value and gradient, 2^14 .. 2^20 points, 32^3 and 128^3 volumes): the
// tricubic one-lane kernel is latency-bound at every size (VGPRs allow 4
// waves per SIMD; four lanes per point run at 8 and are up to 1.7x faster),
// the triquadratic one breaks even, the trilinear one is faster from 2^18
// points on.
template <int KIND>
constexpr int split_default_maxn() {
    constexpr int S = split_extent<KIND>();
    return S == 4 ? 0x7fffffff : (S == 3 ? (1 << 18) : (S == 2 ? (1 << 17) : 0));
}

// v summed over the four lanes of its quad (every lane gets the sum).
__device__ __forceinline__ float quad_sum(float v) {
    // quad_perm [1,0,3,2] then [2,3,0,1]
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    return v;
}

// The part of point x that lane l (of its quad) computes, summed over the
// quad; lane 0 writes the results for output index o.  MODE kValue,
// kValueGrad or kGradX (as for k_eval, so that a gradient and the dL/dx
// formed from it agree bit for bit).  Every lane must call this (the quad
// sums need all four lanes active); lanes with has == false take part with
// the point x = 0 and write nothing.
template <int KIND, class CT, class PT, int MODE>
__device__ __forceinline__ void eval_split_at(const PT x[3], long long o, bool has, int l,
                                              const void* __restrict__ coef, unsigned nbytes,
                                              const VolGeom& g, float* __restrict__ out,
                                              float* __restrict__ grad,
                                              const float* __restrict__ gin) {
    using T = TablesOf<KIND>;
    using P = PolyOf<KIND>;
    constexpr int S = split_extent<KIND>();
    constexpr int S2 = S * S;
    Loc L;
    locate<KIND>(x, g, L);
    const __amdgpu_buffer_rsrc_t r = make_rsrc(coef, nbytes);
    float w[P::kPre];
    P::template pre<MODE == kValue ? 0 : 1>(L.y[0], L.y[1], L.y[2], w);
    // this lane's slab (lanes past the last slab repeat slab 0 and add 0)
    const bool mine = l < S;
    const int ls = mine ? l : 0;
    int off[S2];
#pragma unroll
    for (int j = 0; j < S2; ++j)
        off[j] = tap_offset<KIND>(L, T::kOff[j][0], T::kOff[j][1], T::kOff[j][2] + ls, 0);
    __builtin_amdgcn_sched_barrier(0);
    float c[S2];
#pragma unroll
    for (int j = 0; j < S2; ++j) c[j] = Coef<CT>::ld(r, off[j]);
    // 1D weights of this slab along z (registers, no dynamic indexing)
    float wz = 0.0f, dz = 0.0f;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        wz = ls == q ? w[2 * S + q] : wz;
        if (MODE != kValue) dz = ls == q ? w[5 * S + q] : dz;
    }
    if (!mine) {
        wz = 0.0f;
        dz = 0.0f;
    }
    // w[(order * 3 + axis) * S + a]
    float rv = 0.0f, rx = 0.0f, ry = 0.0f;
#pragma unroll
    for (int b = 0; b < S; ++b) {
        float s = c[S * b] * w[0];
        float sd = 0.0f;
        if (MODE != kValue) sd = c[S * b] * w[3 * S];
#pragma unroll
        for (int a = 1; a < S; ++a) {
            s = fmaf(c[a + S * b], w[a], s);
            if (MODE != kValue) sd = fmaf(c[a + S * b], w[3 * S + a], sd);
        }
        rv = fmaf(s, w[S + b], rv);
        if (MODE != kValue) {
            ry = fmaf(s, w[4 * S + b], ry);
            rx = fmaf(sd, w[S + b], rx);
        }
    }
    const float f = quad_sum(rv * wz);
    const float qnan = __builtin_nanf("");
    const float fill = L.nan ? qnan : 0.0f;
    if (MODE == kValue) {
        if (has && l == 0) out[o] = L.active ? f : fill;
    } else {
        float gr[3] = {quad_sum(rx * wz), quad_sum(ry * wz), quad_sum(rv * dz)};
        float gx[3];
        grad_to_global(L, gr, gx);
        if (has && l == 0) {
            float scale = 1.0f;
            if (MODE == kGradX) scale = gin[o];
            if (MODE == kValueGrad && out) out[o] = L.active ? f : fill;
#pragma unroll
            for (int a = 0; a < 3; ++a) grad[3 * o + a] = L.active ? scale * gx[a] : fill;
        }
    }
}

// Thread t handles point t / 4, slab t % 4.
template <int KIND, class CT, class PT, int MODE>
__global__ __launch_bounds__(256) void k_eval_split(const PT* __restrict__ pts, int N,
                                                    const void* __restrict__ coef, unsigned nbytes,
                                                    VolGeom g, float* __restrict__ out,
                                                    float* __restrict__ grad,
                                                    const float* __restrict__ gin) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long i = t >> 2;
    const bool has = i < N;
    PT x[3] = {PT(0), PT(0), PT(0)};
    if (has) load_point(pts, (int)i, x);
    eval_split_at<KIND, CT, PT, MODE>(x, i, has, (int)(t & 3), coef, nbytes, g, out, grad, gin);
}

// Largest point count for four lanes per point: the caller's setting, or
// (-1) the spline's default.
template <int KIND>
inline int split_limit(int requested) {
    return requested >= 0 ? requested : split_default_maxn<KIND>();
}

}  // namespace lsp
