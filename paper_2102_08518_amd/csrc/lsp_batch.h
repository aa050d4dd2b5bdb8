// Internal interface of the batched persistent launch.
#pragma once

#include <hip/hip_runtime_api.h>

#include "lsp_locate.h"

namespace lsp {

struct BatchVol {
    const void* coef;   // internal coefficient buffer
    unsigned nbytes;
    int kind;           // Kind
    int ctype;          // CoefType
    int N;              // points of this volume
    VolGeom g;
    const float* pts;   // N x 3 FP32
    float* val;         // N (nullable when grad is set)
    float* grad;        // N x 3 or nullptr (value only)
};

struct BatchItem {
    int vol;
    int start;
    int count;
};

// Reset the work counter, then run the persistent kernel with `blocks`
// workgroups.  Both are plain kernel launches (graph-capturable).
hipError_t launch_batch(const BatchVol* vols, const BatchItem* items, int n_items, int* counter,
                        int blocks, hipStream_t stream);
int batch_block_threads();

}  // namespace lsp
