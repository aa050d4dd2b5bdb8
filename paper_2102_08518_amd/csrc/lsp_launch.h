// Internal interface between the host library and the kernel translation
// units (one per spline kind, so they compile in parallel).
#pragma once

#include <hip/hip_runtime_api.h>

#include "lsp_locate.h"

namespace lsp {

enum CoefType : int { kCF32 = 0, kCBF16 = 1, kCF16 = 2 };
enum Mode : int { kValue = 0, kValueGrad = 1, kGradX = 2, kValueGradHess = 3 };

struct EvalArgs {
    int kind;           // Kind
    int ctype;          // CoefType of the internal buffer
    bool pts_f64;       // points in FP64
    int mode;           // Mode
    bool predicated;    // FCC6: evaluate both reference polynomials and select
    const void* pts;
    int N;
    const void* coef;
    unsigned nbytes;
    VolGeom g;
    float* out;
    float* grad;
    float* hess;        // kValueGradHess: N x 6 (xx, xy, xz, yy, yz, zz)
    const float* gin;
    hipStream_t stream;
    unsigned lds_bytes;  // dynamic LDS per workgroup (occupancy control), usually 0
    bool mfma;           // matrix-core path where the spline has one (kValue, kValueGrad)
    int split_maxn;      // separable splines: four lanes per point when N <= split_maxn
                         // (-1: the spline's measured default)
};

// Defined in lsp_dispatch.h and instantiated once per spline kind in its own
// translation unit (eval_<name>.hip).
template <int KIND>
hipError_t launch_eval(const EvalArgs& a);

// Convert one caller coset array (C order [z][y][x], dims X,Y,Z, dtype
// src_dtype as lsp_dtype) into the internal padded buffer.
hipError_t launch_pack(const void* src, int src_dtype, int ctype, void* dst, const int64_t dims[3],
                       const VolGeom& g, int coset, hipStream_t stream);

}  // namespace lsp
