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

// The items of one kernel variant (spline kind, storage, value or
// value+gradient): a contiguous range of the item list.
struct BatchGroup {
    int kind;
    int ctype;
    int grad;
    int first;
    int count;
};

// One persistent kernel per group with at most `blocks` workgroups, popping
// items from the group's work counter (device, one int per group), which
// must be zero before the launch and is zero again after it.  Plain kernel
// launches (graph-capturable); groups is host memory.
// split_maxn: the four-lanes-per-point limit of the separable splines, as
// for the direct entry points (-1: each spline's default).
hipError_t launch_batch(const BatchVol* vols, const BatchItem* items, const BatchGroup* groups,
                        int n_groups, int* counters, int blocks, int split_maxn, hipStream_t stream);
// Set n work counters to zero (once, when a plan is created).
hipError_t reset_batch_counters(int* counters, int n, hipStream_t stream);
int batch_block_threads();

}  // namespace lsp
