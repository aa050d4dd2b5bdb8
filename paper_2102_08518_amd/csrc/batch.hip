// Batched evaluation of many volumes of uneven size in a few persistent
// launches.
//
// A plan binds the per-volume descriptors (coefficient buffer, layout,
// points, outputs) and a work list of (volume, tile of points) items, grouped
// by kernel variant (spline kind, storage type, value or value+gradient).
// Per group one grid of persistent workgroups pops items from the group's
// atomic counter until its list is exhausted; each variant is its own
// instantiation, so it keeps the registers of the single-volume kernel
// instead of the union of all variants.  Every workgroup makes exactly one
// pop past the end of the list, and the workgroup whose pop is the last of
// all resets the counter to zero: no other workgroup reads it after that, so
// each launch leaves the counter ready for the next one and a graph of the
// launches can be replayed without a separate reset.  The counters start at
// zero when the plan is created.
#include <hip/hip_runtime.h>

#include "lsp_batch.h"
#include "lsp_kernels.h"
#include "lsp_split.h"

namespace lsp {

namespace {

constexpr int kBatchBlock = 256;

__global__ void k_batch_reset(int* counters, int n) {
    for (int i = 0; i < n; ++i) counters[i] = 0;
}

// The points of one item with the per-point body lsp_eval uses for a volume
// of v.N points: four lanes per point for the separable splines up to their
// limit (split_maxn, -1 for the spline's default), else one lane.  The loop
// trip count is uniform over the workgroup, so every lane reaches the quad
// sums of the split body.
template <int KIND, class CT, int MODE>
__device__ __forceinline__ void run_item(const BatchVol& v, int start, int count, int split_maxn) {
    if constexpr (split_eligible<KIND>()) {
        const int lim = split_maxn >= 0 ? split_maxn : split_default_maxn<KIND>();
        if (v.N <= lim) {
            const int lanes = count * kSplitLanes;
#pragma unroll 1
            for (int q = 0; q < lanes; q += kBatchBlock) {
                const int t = q + (int)threadIdx.x;
                const bool has = t < lanes;
                const int p = start + (t >> 2);
                float x[3] = {0.0f, 0.0f, 0.0f};
                if (has) load_point(v.pts, p, x);
                eval_split_at<KIND, CT, float, MODE>(x, p, has, t & 3, v.coef, v.nbytes, v.g, v.val,
                                                     v.grad, nullptr);
            }
            return;
        }
    }
    // offsets within the item, so that no index passes 2^31 - 1 on the way
#pragma unroll 1
    for (int q = (int)threadIdx.x; q < count; q += kBatchBlock)
        eval_point<KIND, CT, float, MODE, false>(v.pts, start + q, start + q, v.coef, v.nbytes, v.g,
                                                 v.val, v.grad, nullptr);
}

template <int KIND, class CT, int MODE>
__global__ __launch_bounds__(kBatchBlock) void k_batch(const BatchVol* __restrict__ vols,
                                                       const BatchItem* __restrict__ items,
                                                       int n_items, int* __restrict__ counter,
                                                       int split_maxn) {
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        // uniform across the workgroup: the item and volume descriptors are
        // then loaded once into scalar registers
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= n_items) {
            // pops return 0 .. n_items + gridDim.x - 1, each once; the largest is the last
            if (threadIdx.x == 0 && it == n_items + (int)gridDim.x - 1) atomicExch(counter, 0);
            break;
        }
        const BatchItem w = items[it];
        // by reference: the layout fields selected per axis are then read
        // from the descriptor in memory, not from a private copy
        const BatchVol& v = vols[w.vol];
        run_item<KIND, CT, MODE>(v, w.start, w.count, split_maxn);
    }
}

template <int KIND, class CT>
hipError_t launch_group_ct(const BatchVol* vols, const BatchItem* items, const BatchGroup& gr,
                           int* counter, int blocks, int split_maxn, hipStream_t stream) {
    const int b = blocks < gr.count ? blocks : gr.count;
    if (gr.grad)
        hipLaunchKernelGGL((k_batch<KIND, CT, kValueGrad>), dim3(b), dim3(kBatchBlock), 0, stream,
                           vols, items + gr.first, gr.count, counter, split_maxn);
    else
        hipLaunchKernelGGL((k_batch<KIND, CT, kValue>), dim3(b), dim3(kBatchBlock), 0, stream, vols,
                           items + gr.first, gr.count, counter, split_maxn);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_group(const BatchVol* vols, const BatchItem* items, const BatchGroup& gr,
                        int* counter, int blocks, int split_maxn, hipStream_t stream) {
    switch (gr.ctype) {
        case kCF32: return launch_group_ct<KIND, float>(vols, items, gr, counter, blocks, split_maxn, stream);
        case kCBF16: return launch_group_ct<KIND, bf16_t>(vols, items, gr, counter, blocks, split_maxn, stream);
        case kCF16: return launch_group_ct<KIND, f16_t>(vols, items, gr, counter, blocks, split_maxn, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_batch(const BatchVol* vols, const BatchItem* items, const BatchGroup* groups,
                        int n_groups, int* counters, int blocks, int split_maxn, hipStream_t stream) {
    if (n_groups <= 0) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int gi = 0; gi < n_groups && e == hipSuccess; ++gi) {
        const BatchGroup& gr = groups[gi];
        if (gr.count <= 0) continue;
        e = hipErrorInvalidValue;
#define LSP_GROUP(k) \
        if (gr.kind == k) e = launch_group<k>(vols, items, gr, counters + gi, blocks, split_maxn, stream);
        LSP_FOR_EACH_KIND(LSP_GROUP)
#undef LSP_GROUP
    }
    return e;
}

hipError_t reset_batch_counters(int* counters, int n, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, stream, counters, n);
    return hipGetLastError();
}

int batch_block_threads() { return kBatchBlock; }

}  // namespace lsp
