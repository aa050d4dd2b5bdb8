// Batched evaluation of many volumes of uneven size in one persistent launch.
//
// A plan binds the per-volume descriptors (coefficient buffer, layout,
// points, outputs) and a work list of (volume, tile of points) items.  One
// grid of persistent workgroups pops items from an atomic counter until the
// list is exhausted; inside an item the spline kind, storage type and mode
// are uniform, so the per-point body of the single-volume kernel runs
// without divergence.  The counter is reset by a one-thread kernel that runs
// first on the same stream, so the pair can be captured in a graph and
// replayed.
#include <hip/hip_runtime.h>

#include "lsp_batch.h"
#include "lsp_kernels.h"

namespace lsp {

namespace {

constexpr int kBatchBlock = 256;

__global__ void k_batch_reset(int* counter) { *counter = 0; }

template <int KIND, class CT, int MODE>
__device__ __forceinline__ void run_item(const BatchVol& v, int start, int count) {
    const int end = start + count;
    for (int p = start + (int)threadIdx.x; p < end; p += kBatchBlock)
        eval_point<KIND, CT, float, MODE, false>(v.pts, p, p, v.coef, v.nbytes, v.g, v.val, v.grad,
                                                 nullptr);
}

template <int KIND>
__device__ __forceinline__ void run_kind(const BatchVol& v, int start, int count) {
    const bool grad = v.grad != nullptr;
    switch (v.ctype) {
        case kCF32:
            if (grad) run_item<KIND, float, kValueGrad>(v, start, count);
            else run_item<KIND, float, kValue>(v, start, count);
            break;
        case kCBF16:
            if (grad) run_item<KIND, bf16_t, kValueGrad>(v, start, count);
            else run_item<KIND, bf16_t, kValue>(v, start, count);
            break;
        default:
            if (grad) run_item<KIND, f16_t, kValueGrad>(v, start, count);
            else run_item<KIND, f16_t, kValue>(v, start, count);
            break;
    }
}

__global__ __launch_bounds__(kBatchBlock) void k_batch(const BatchVol* __restrict__ vols,
                                                       const BatchItem* __restrict__ items,
                                                       int n_items, int* __restrict__ counter) {
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;  // uniform across the workgroup
        const BatchItem w = items[it];
        const BatchVol v = vols[w.vol];
        switch (v.kind) {
#define LSP_CASE(k) case k: run_kind<k>(v, w.start, w.count); break;
            LSP_FOR_EACH_KIND(LSP_CASE)
#undef LSP_CASE
        }
    }
}

}  // namespace

hipError_t launch_batch(const BatchVol* vols, const BatchItem* items, int n_items, int* counter,
                        int blocks, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, stream, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(kBatchBlock), 0, stream, vols, items, n_items,
                       counter);
    return hipGetLastError();
}

int batch_block_threads() { return kBatchBlock; }

}  // namespace lsp
