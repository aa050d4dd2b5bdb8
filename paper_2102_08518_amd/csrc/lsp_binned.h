// Internal interface of the binned forward path.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>

#include "lsp_locate.h"

namespace lsp {

// The scatter kernel keeps two ints per bin (plus the sentinel bin) in LDS;
// the bound keeps that within 64 KiB.
constexpr int kMaxBins = 8000;
static_assert(2 * (kMaxBins + 1) * 4 <= 65536, "bin histogram exceeds 64 KiB of LDS");

// Bins are blocks of 2^lb x 2^lb x 2^lb indices of the padded coset grid.
struct BinGeom {
    int lb;
    int nb[3];
    int nbins;
};

// A point in bin order: its coordinates and its index in the caller's arrays.
template <class PT> struct Rec;
template <> struct alignas(16) Rec<float> {
    float x[3];
    int i;
};
template <> struct alignas(16) Rec<double> {
    double x[3];
    int i;
    int pad;
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
    bool mfma;     // matrix-core evaluation where the spline has one
    int split_maxn;  // separable splines: four lanes per record when N <= this (-1: default)
};

size_t binned_workspace_bytes(const BinGeom& bg, int N, bool pts_f64);
hipError_t launch_binned(const BinnedArgs& a);

}  // namespace lsp
