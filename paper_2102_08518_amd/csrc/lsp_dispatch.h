// Instantiation and launch of k_eval for one spline kind over coefficient
// type x point type x mode (x predication for the two-polynomial spline).
#pragma once

#include "lsp_kernels.h"
#include "lsp_launch.h"
#include "lsp_mfma.h"
#include "lsp_split.h"

namespace lsp {

constexpr int kBlock = 256;

// Points per thread of the matrix-core kernel: enough blocks to fill the chip
// several times over, the weight operands reused across the rest.
inline int mfma_points_per_thread(int N) {
    const int per = N / (kBlock * 2048);
    return per < 1 ? 1 : (per > 8 ? 8 : per);
}

template <int KIND, class CT, class PT, int MODE, bool PRED>
hipError_t launch_one(const EvalArgs& a) {
    if constexpr (mfma_eligible<KIND>() && (MODE == kValue || MODE == kValueGrad) && !PRED) {
        if (a.mfma) {
            const int ppt = mfma_points_per_thread(a.N);
            const int blocks = (int)(((long long)a.N + kBlock * ppt - 1) / (kBlock * ppt));
            hipLaunchKernelGGL((k_eval_mfma<KIND, CT, PT, MODE>), dim3(blocks), dim3(kBlock), 0,
                               a.stream, static_cast<const PT*>(a.pts), a.N, ppt, a.coef, a.nbytes,
                               a.g, a.out, a.grad);
            return hipGetLastError();
        }
    }
    if constexpr (split_eligible<KIND>() && MODE != kValueGradHess) {
        if (a.N <= split_limit<KIND>(a.split_maxn)) {
            const PT* pts = static_cast<const PT*>(a.pts);
            for (long long s = 0; s < a.N; s += kSplitChunk) {
                const int n = (int)(a.N - s < kSplitChunk ? a.N - s : kSplitChunk);
                const int blocks = (int)(((long long)n * kSplitLanes + kBlock - 1) / kBlock);
                hipLaunchKernelGGL((k_eval_split<KIND, CT, PT, MODE>), dim3(blocks), dim3(kBlock), 0,
                                   a.stream, pts + 3 * s, n, a.coef, a.nbytes, a.g,
                                   a.out ? a.out + s : nullptr, a.grad ? a.grad + 3 * s : nullptr,
                                   a.gin ? a.gin + s : nullptr);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
    }
    const int blocks = (int)(((long long)a.N + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_eval<KIND, CT, PT, MODE, PRED>), dim3(blocks), dim3(kBlock), a.lds_bytes, a.stream,
                       static_cast<const PT*>(a.pts), a.N, a.coef, a.nbytes, a.g, a.out, a.grad,
                       a.gin, a.hess);
    return hipGetLastError();
}

template <int KIND, class CT, class PT, bool PRED>
hipError_t launch_mode(const EvalArgs& a) {
    switch (a.mode) {
        case kValue: return launch_one<KIND, CT, PT, kValue, PRED>(a);
        case kValueGrad: return launch_one<KIND, CT, PT, kValueGrad, PRED>(a);
        case kGradX: return launch_one<KIND, CT, PT, kGradX, PRED>(a);
        case kValueGradHess: return launch_one<KIND, CT, PT, kValueGradHess, PRED>(a);
    }
    return hipErrorInvalidValue;
}

template <int KIND, class CT, bool PRED>
hipError_t launch_pt(const EvalArgs& a) {
    return a.pts_f64 ? launch_mode<KIND, CT, double, PRED>(a) : launch_mode<KIND, CT, float, PRED>(a);
}

template <int KIND, bool PRED>
hipError_t launch_ct(const EvalArgs& a) {
    switch (a.ctype) {
        case kCF32: return launch_pt<KIND, float, PRED>(a);
        case kCBF16: return launch_pt<KIND, bf16_t, PRED>(a);
        case kCF16: return launch_pt<KIND, f16_t, PRED>(a);
    }
    return hipErrorInvalidValue;
}

template <int KIND>
hipError_t launch_kind(const EvalArgs& a) {
    if (a.N <= 0) return hipSuccess;
    if constexpr (TablesOf<KIND>::kRegions > 1) {
        if (a.predicated) return launch_ct<KIND, true>(a);
    }
    return launch_ct<KIND, false>(a);
}

template <int KIND>
hipError_t launch_eval(const EvalArgs& a) {
    return launch_kind<KIND>(a);
}

}  // namespace lsp
