// Forward and value+gradient kernels: one thread per query point, the four
// steps of Algorithm 1 -- locate and transform (lsp_locate.h), fetch the
// stencil coefficients, evaluate the reference sub-region polynomial in
// Horner form (generated code), write the result.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "lsp_launch.h"
#include "lsp_locate.h"

namespace lsp {

// Buffer resource over the internal coefficient buffer: raw loads whose byte
// offset is outside [0, nbytes) return 0 instead of touching memory, which is
// also exactly the zero padding of the convolution sum.
#define LSP_RSRC_FLAGS 0x00020000

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes,
                                             LSP_RSRC_FLAGS);
}

struct bf16_t { unsigned short b; };
struct f16_t { unsigned short b; };

template <class CT> struct Coef;
template <> struct Coef<float> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
};
template <> struct Coef<bf16_t> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int off) {
        const unsigned h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return __builtin_bit_cast(float, h << 16);
    }
};
template <> struct Coef<f16_t> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int off) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return (float)__builtin_bit_cast(_Float16, h);
    }
};

// Whether the tap loads are also fenced off from the arithmetic after them.
// With the fence the polynomial starts only once every load is issued; without
// it the scheduler may start consuming the first taps among the last loads.
// Chosen per spline and mode from measurements on MI355X (the analogue of the
// paper's per-architecture parameter exploration, Sec. 5): the fence pays
// for the 7-direction splines and the BCC8 gradient; the separable splines and
// the BCC8 value do better without it.
template <int KIND, int MODE>
constexpr bool fence_after_loads() {
    return !TablesOf<KIND>::kTensor && !(KIND == kBcc8 && MODE == kValue);
}

// Fetch every tap of the union stencil (Algorithm 1's memory lookups through
// the permuted stencil pi').  The gathers are latency-bound, so every address
// is formed first and the loads are then issued back to back.  Left to itself
// the scheduler interleaves them with address arithmetic or, to save
// registers, waits on the first loads before issuing the last (a second
// memory round trip per point).
template <int KIND, class CT, bool FENCE_AFTER>
__device__ __forceinline__ void gather(const Loc& L, __amdgpu_buffer_rsrc_t r, float* c) {
    using T = TablesOf<KIND>;
    int off[T::kTaps];
#pragma unroll
    for (int j = 0; j < T::kTaps; ++j)
        off[j] = tap_offset<KIND>(L, T::kOff[j][0], T::kOff[j][1], T::kOff[j][2], T::kParity[j]);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (FENCE_AFTER) {
        // the polynomial waits for every load: table order, which keeps the
        // loads of neighbouring taps together
#pragma unroll
        for (int j = 0; j < T::kTaps; ++j) c[j] = Coef<CT>::ld(r, off[j]);
        __builtin_amdgcn_sched_barrier(0);
    } else {
        // the polynomial starts while loads are in flight, and loads complete
        // in issue order: issue them in the order the polynomial first reads
        // the taps (generated)
#pragma unroll
        for (int q = 0; q < T::kTaps; ++q) c[T::kIssue[q]] = Coef<CT>::ld(r, off[T::kIssue[q]]);
    }
}

// Reference polynomial value and gradient (the unrolled reference
// sub-region loop of Sec. 4.3, generated per spline; two reference
// sub-regions either branch or evaluate both and select).  For the
// tensor-product splines w holds the 1D weights formed from y before the
// gather (PolyOf<KIND>::pre), so that work overlaps the loads in flight.
template <int KIND, bool PREDICATED>
__device__ __forceinline__ float poly_value(const float* c, const Loc& L, const float* w) {
    if constexpr (PolyOf<KIND>::kPre > 0) return PolyOf<KIND>::value_pre(c, w);
    else return PolyOf<KIND>::template value<PREDICATED>(c, L.y[0], L.y[1], L.y[2], L.region);
}

template <int KIND, bool PREDICATED>
__device__ __forceinline__ float poly_value_grad(const float* c, const Loc& L, const float* w, float* g) {
    if constexpr (PolyOf<KIND>::kPre > 0) return PolyOf<KIND>::value_grad_pre(c, w, g[0], g[1], g[2]);
    else
        return PolyOf<KIND>::template value_grad<PREDICATED>(c, L.y[0], L.y[1], L.y[2], L.region, g[0],
                                                              g[1], g[2]);
}

template <int KIND, bool PREDICATED>
__device__ __forceinline__ float poly_value_grad_hess(const float* c, const Loc& L, const float* w, float* g,
                                                      float* h) {
    if constexpr (PolyOf<KIND>::kPre > 0)
        return PolyOf<KIND>::value_grad_hess_pre(c, w, g[0], g[1], g[2], h);
    else
        return PolyOf<KIND>::template value_grad_hess<PREDICATED>(c, L.y[0], L.y[1], L.y[2], L.region,
                                                                   g[0], g[1], g[2], h);
}

// Hessian back to global axes: with y = G (x - k), G a signed permutation,
// d2f/dx_a dx_b = sgn[r] sgn[s] d2f/dy_r dy_s for axis[r] = a, axis[s] = b.
// hr, hg: (00, 01, 02, 11, 12, 22).
__device__ __forceinline__ float sym3(const float* hr, int i, int j) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    return lo == 0 ? (hi == 0 ? hr[0] : (hi == 1 ? hr[1] : hr[2]))
                   : (lo == 1 ? (hi == 1 ? hr[3] : hr[4]) : hr[5]);
}

__device__ __forceinline__ void hess_to_global(const Loc& L, const float* hr, float* hg) {
    int rr[3];
    float sg[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rr[a] = L.axis[0] == a ? 0 : (L.axis[1] == a ? 1 : 2);
        sg[a] = rr[a] == 0 ? L.sgn[0] : (rr[a] == 1 ? L.sgn[1] : L.sgn[2]);
    }
    hg[0] = sym3(hr, rr[0], rr[0]);
    hg[1] = sg[0] * sg[1] * sym3(hr, rr[0], rr[1]);
    hg[2] = sg[0] * sg[2] * sym3(hr, rr[0], rr[2]);
    hg[3] = sym3(hr, rr[1], rr[1]);
    hg[4] = sg[1] * sg[2] * sym3(hr, rr[1], rr[2]);
    hg[5] = sym3(hr, rr[2], rr[2]);
}

// Gradient back to global axes: y = G (x - k) with G a signed permutation,
// so df/dx = G^T df/dy, i.e. component axis[r] is sgn[r] * df/dy_r.
__device__ __forceinline__ void grad_to_global(const Loc& L, const float* gr, float* gx) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float v = 0.0f;
#pragma unroll
        for (int r = 0; r < 3; ++r) v = (L.axis[r] == a) ? L.sgn[r] * gr[r] : v;
        gx[a] = v;
    }
}



template <class PT>
__device__ __forceinline__ void load_point(const PT* __restrict__ pts, int i, PT x[3]) {
    x[0] = pts[3 * (size_t)i + 0];
    x[1] = pts[3 * (size_t)i + 1];
    x[2] = pts[3 * (size_t)i + 2];
}

// One query point, all of Algorithm 1 (x read at index i, results written
// at index o):
// MODE kValue:     out[o] = f(x_i)
// MODE kValueGrad: out[o] = f(x_i) (if out), grad[3o..] = grad f(x_i)
// MODE kGradX:     grad[3o..] = gin[o] * grad f(x_i)        (dL/dx)
// MODE kValueGradHess: out[o], grad[3o..] (each if non-null), hess[6o..] =
//                  the Hessian (xx, xy, xz, yy, yz, zz)
// Evaluates the point x (coordinates already loaded) and writes its results
// to output index o.
template <int KIND, class CT, class PT, int MODE, bool PREDICATED>
__device__ __forceinline__ void eval_at(const PT x[3], int o, const void* __restrict__ coef,
                                        unsigned nbytes, const VolGeom& g,
                                        float* __restrict__ out, float* __restrict__ grad,
                                        const float* __restrict__ gin,
                                        float* __restrict__ hess = nullptr) {
    using T = TablesOf<KIND>;
    using P = PolyOf<KIND>;
    Loc L;
    locate<KIND>(x, g, L);
    const __amdgpu_buffer_rsrc_t r = make_rsrc(coef, nbytes);
    float w[P::kPre > 0 ? P::kPre : 1];
    if constexpr (P::kPre > 0)
        P::template pre<MODE == kValue ? 0 : (MODE == kValueGradHess ? 2 : 1)>(L.y[0], L.y[1], L.y[2], w);
    float c[T::kTaps];
    gather<KIND, CT, fence_after_loads<KIND, MODE>()>(L, r, c);
    const float qnan = __builtin_nanf("");
    if (MODE == kValue) {
        const float f = poly_value<KIND, PREDICATED>(c, L, w);
        out[o] = L.active ? f : (L.nan ? qnan : 0.0f);
    } else if (MODE == kValueGradHess) {
        float gr[3], gx[3], hr[6], hx[6];
        const float f = poly_value_grad_hess<KIND, PREDICATED>(c, L, w, gr, hr);
        grad_to_global(L, gr, gx);
        hess_to_global(L, hr, hx);
        const float fill = L.nan ? qnan : 0.0f;
        if (out) out[o] = L.active ? f : fill;
        if (grad)
#pragma unroll
            for (int a = 0; a < 3; ++a) grad[3 * (size_t)o + a] = L.active ? gx[a] : fill;
#pragma unroll
        for (int a = 0; a < 6; ++a) hess[6 * (size_t)o + a] = L.active ? hx[a] : fill;
    } else {
        float gr[3], gx[3];
        const float f = poly_value_grad<KIND, PREDICATED>(c, L, w, gr);
        grad_to_global(L, gr, gx);
        const float fill = L.nan ? qnan : 0.0f;
        float scale = 1.0f;
        if (MODE == kGradX) scale = gin[o];
        if (MODE == kValueGrad && out) out[o] = L.active ? f : fill;
#pragma unroll
        for (int a = 0; a < 3; ++a) grad[3 * (size_t)o + a] = L.active ? scale * gx[a] : fill;
    }
}

template <int KIND, class CT, class PT, int MODE, bool PREDICATED>
__device__ __forceinline__ void eval_point(const PT* __restrict__ pts, int i, int o,
                                           const void* __restrict__ coef, unsigned nbytes,
                                           const VolGeom& g, float* __restrict__ out,
                                           float* __restrict__ grad,
                                           const float* __restrict__ gin,
                                           float* __restrict__ hess = nullptr) {
    PT x[3];
    load_point(pts, i, x);
    eval_at<KIND, CT, PT, MODE, PREDICATED>(x, o, coef, nbytes, g, out, grad, gin, hess);
}

template <int KIND, class CT, class PT, int MODE, bool PREDICATED>
__global__ __launch_bounds__(256) void k_eval(const PT* __restrict__ pts, int N,
                                              const void* __restrict__ coef, unsigned nbytes,
                                              VolGeom g, float* __restrict__ out,
                                              float* __restrict__ grad,
                                              const float* __restrict__ gin,
                                              float* __restrict__ hess) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    eval_point<KIND, CT, PT, MODE, PREDICATED>(pts, i, i, coef, nbytes, g, out, grad, gin, hess);
}

}  // namespace lsp
