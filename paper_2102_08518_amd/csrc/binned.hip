// Forward evaluation in spatially binned order.
//
// For points in random order the gathers of the 64 points of a wavefront
// touch several hundred distinct cache lines, more than the L1 holds, so
// almost every tap becomes an L2 request.  The value at a point does not
// depend on the order in which points are processed, so this path first
// groups the points by coarse blocks of the coset grid (2^lb sites per axis):
//   1. per point its bin (the block holding its ROE lattice point; inactive
//      points go to a last, sentinel bin) and a workgroup-privatised count;
//   2. exclusive scan of the bin counts;
//   3. scatter of the original indices into bin order (workgroup-privatised
//      ranks, one global atomic per touched bin);
//   4. evaluation in bin order: each work-item reads its point through the
//      index and writes the result back to that index.
// The order inside a bin varies from run to run; every output is the same
// function of its own point, so the results are bit-identical to lsp_eval.
#include <hip/hip_runtime.h>

#include "lsp_binned.h"
#include "lsp_kernels.h"

namespace lsp {

namespace {

constexpr int kBinBlk = 256;
constexpr int kPtsPerThr = 16;


template <int KIND, class PT>
__device__ __forceinline__ int bin_of(const PT* __restrict__ pts, int i, const VolGeom& g,
                                      const BinGeom& bg) {
    constexpr int D = TablesOf<KIND>::kD;
    PT x[3];
    load_point(pts, i, x);
    Loc L;
    locate<KIND>(x, g, L);
    if (!L.active) return bg.nbins;
    int b[3];
    for (int a = 0; a < 3; ++a) {
        const int K = (D == 1 ? L.k[a] : (L.k[a] >> 1)) + g.pad;
        b[a] = K >> bg.lb;
    }
    return (b[2] * bg.nb[1] + b[1]) * bg.nb[0] + b[0];
}

__global__ __launch_bounds__(kBinBlk) void k_fill(int* __restrict__ p, int n, int v) {
    for (int t = blockIdx.x * kBinBlk + threadIdx.x; t < n; t += gridDim.x * kBinBlk) p[t] = v;
}

template <int KIND, class PT>
__global__ __launch_bounds__(kBinBlk) void k_bin_count(const PT* __restrict__ pts, int N, VolGeom g,
                                                       BinGeom bg, int* __restrict__ bin,
                                                       int* __restrict__ count) {
    __shared__ int h[kMaxBins + 1];
    for (int t = threadIdx.x; t <= bg.nbins; t += kBinBlk) h[t] = 0;
    __syncthreads();
    const int base = blockIdx.x * kBinBlk * kPtsPerThr;
    for (int k = 0; k < kPtsPerThr; ++k) {
        const int i = base + k * kBinBlk + (int)threadIdx.x;
        if (i < N) {
            const int b = bin_of<KIND>(pts, i, g, bg);
            bin[i] = b;
            atomicAdd(&h[b], 1);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= bg.nbins; t += kBinBlk)
        if (h[t]) atomicAdd(&count[t], h[t]);
}

// start[b] = sum of count[0..b); one workgroup, nbins + 1 <= kMaxBins + 1.
__global__ __launch_bounds__(1024) void k_bin_scan(const int* __restrict__ count, int n,
                                                   int* __restrict__ start) {
    __shared__ int part[1024];
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    int s = 0;
    for (int t = lo; t < hi; ++t) s += count[t];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int t = lo; t < hi; ++t) {
        start[t] = run;
        run += count[t];
    }
}

__global__ __launch_bounds__(kBinBlk) void k_bin_scatter(const int* __restrict__ bin, int N,
                                                         BinGeom bg, const int* __restrict__ start,
                                                         int* __restrict__ cursor,
                                                         int* __restrict__ bidx) {
    __shared__ int h[kMaxBins + 1];
    __shared__ int hb[kMaxBins + 1];
    for (int t = threadIdx.x; t <= bg.nbins; t += kBinBlk) h[t] = 0;
    __syncthreads();
    const int base = blockIdx.x * kBinBlk * kPtsPerThr;
    int b[kPtsPerThr], r[kPtsPerThr];
#pragma unroll
    for (int k = 0; k < kPtsPerThr; ++k) {
        const int i = base + k * kBinBlk + (int)threadIdx.x;
        b[k] = i < N ? bin[i] : 0;
        r[k] = i < N ? atomicAdd(&h[b[k]], 1) : 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= bg.nbins; t += kBinBlk)
        if (h[t]) hb[t] = start[t] + atomicAdd(&cursor[t], h[t]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPtsPerThr; ++k) {
        const int i = base + k * kBinBlk + (int)threadIdx.x;
        if (i < N) bidx[hb[b[k]] + r[k]] = i;
    }
}

template <int KIND, class CT, class PT, int MODE>
__global__ __launch_bounds__(256) void k_eval_binned(const PT* __restrict__ pts,
                                                     const int* __restrict__ bidx, int N,
                                                     const void* __restrict__ coef, unsigned nbytes,
                                                     VolGeom g, float* __restrict__ out,
                                                     float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = bidx[p];
    eval_point<KIND, CT, PT, MODE, false>(pts, i, i, coef, nbytes, g, out, grad, nullptr);
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Parts {
    size_t bin, count, start, cursor, bidx, total;
};

Parts parts(const BinGeom& bg, int N) {
    Parts q{};
    const size_t n = (size_t)(N > 0 ? N : 1);
    size_t o = 0;
    q.bin = o; o += a256(4 * n);
    q.count = o; o += a256(4 * ((size_t)bg.nbins + 1));
    q.start = o; o += a256(4 * ((size_t)bg.nbins + 1));
    q.cursor = o; o += a256(4 * ((size_t)bg.nbins + 1));
    q.bidx = o; o += a256(4 * n);
    q.total = o;
    return q;
}

template <int KIND, class CT, class PT>
hipError_t run(const BinnedArgs& a, const Parts& q) {
    char* ws = static_cast<char*>(a.ws);
    int* bin = reinterpret_cast<int*>(ws + q.bin);
    int* count = reinterpret_cast<int*>(ws + q.count);
    int* start = reinterpret_cast<int*>(ws + q.start);
    int* cursor = reinterpret_cast<int*>(ws + q.cursor);
    int* bidx = reinterpret_cast<int*>(ws + q.bidx);
    const PT* pts = static_cast<const PT*>(a.pts);
    const int N = a.N;
    const int nb1 = a.bg.nbins + 1;
    const int fill_blocks = (nb1 + kBinBlk - 1) / kBinBlk;
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks), dim3(kBinBlk), 0, a.stream, count, nb1, 0);
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks), dim3(kBinBlk), 0, a.stream, cursor, nb1, 0);
    const int chunk = kBinBlk * kPtsPerThr;
    const int cblocks = (N + chunk - 1) / chunk;
    hipLaunchKernelGGL((k_bin_count<KIND, PT>), dim3(cblocks), dim3(kBinBlk), 0, a.stream, pts, N,
                       a.g, a.bg, bin, count);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, a.stream, count, nb1, start);
    hipLaunchKernelGGL(k_bin_scatter, dim3(cblocks), dim3(kBinBlk), 0, a.stream, bin, N, a.bg, start,
                       cursor, bidx);
    const int eblocks = (N + 255) / 256;
    if (a.grad)
        hipLaunchKernelGGL((k_eval_binned<KIND, CT, PT, kValueGrad>), dim3(eblocks), dim3(256), 0,
                           a.stream, pts, bidx, N, a.coef, a.nbytes, a.g, a.out, a.grad);
    else
        hipLaunchKernelGGL((k_eval_binned<KIND, CT, PT, kValue>), dim3(eblocks), dim3(256), 0,
                           a.stream, pts, bidx, N, a.coef, a.nbytes, a.g, a.out, a.grad);
    return hipGetLastError();
}

template <int KIND, class PT>
hipError_t run_ct(const BinnedArgs& a, const Parts& q) {
    switch (a.ctype) {
        case kCF32: return run<KIND, float, PT>(a, q);
        case kCBF16: return run<KIND, bf16_t, PT>(a, q);
        case kCF16: return run<KIND, f16_t, PT>(a, q);
    }
    return hipErrorInvalidValue;
}

}  // namespace

size_t binned_workspace_bytes(const BinGeom& bg, int N, bool pts_f64) {
    (void)pts_f64;
    return parts(bg, N).total;
}

hipError_t launch_binned(const BinnedArgs& a) {
    if (a.N <= 0) return hipSuccess;
    if (a.bg.nbins > kMaxBins) return hipErrorInvalidValue;
    const Parts q = parts(a.bg, a.N);
    if (a.ws_bytes < q.total) return hipErrorInvalidValue;
#define LSP_RUN(k) \
    if (a.kind == k) return a.pts_f64 ? run_ct<k, double>(a, q) : run_ct<k, float>(a, q);
    LSP_FOR_EACH_KIND(LSP_RUN)
#undef LSP_RUN
    return hipErrorInvalidValue;
}

}  // namespace lsp
