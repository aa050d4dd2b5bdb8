// Internal interface of the binned forward path.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>

#include "lsp_locate.h"

namespace lsp {

constexpr int kMaxBins = 8192;

// Bins are blocks of 2^lb x 2^lb x 2^lb indices of the padded coset grid.
struct BinGeom {
    int lb;
    int nb[3];
    int nbins;
};

struct BinnedArgs {
    int kind;
    int ctype;
    bool pts_f64;
    const void* pts;
    int N;
    const void* coef;
    unsigned nbytes;
    VolGeom g;
    BinGeom bg;
    float* out;    // N
    float* grad;   // N x 3 or nullptr
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
};

size_t binned_workspace_bytes(const BinGeom& bg, int N, bool pts_f64);
hipError_t launch_binned(const BinnedArgs& a);

}  // namespace lsp
