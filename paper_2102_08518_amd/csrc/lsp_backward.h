// Internal interface of the dL/dc pass (deterministic binning plus the
// transposed-stencil gather).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "lsp_locate.h"

namespace lsp {

struct BackwardArgs {
    int kind;
    int ctype;
    bool pts_f64;
    const void* pts;
    int N;
    VolGeom g;
    int n_cosets;
    int dims[3];
    const float* dL_df;
    float* dL_dc;
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
};

size_t backward_workspace_bytes(int kind, int n_cosets, const int64_t dims[3], int pad, int64_t N);
hipError_t launch_backward_coef(const BackwardArgs& a);

// dL_dx[3i + a] = dL_df[i] * grad_f[3i + a].
hipError_t launch_dx_from_grad(long long N, const float* dL_df, const float* grad_f, float* dL_dx,
                               hipStream_t stream);

}  // namespace lsp
