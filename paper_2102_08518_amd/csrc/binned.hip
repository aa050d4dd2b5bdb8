// Forward evaluation in spatially binned order.
//
// For points in random order the gathers of the 64 points of a wavefront
// touch several hundred distinct cache lines, more than the L1 holds, so
// almost every tap becomes an L2 request.  The value at a point does not
// depend on the order in which points are processed, so this path first
// groups the points by coarse blocks of the coset grid (2^lb sites per axis):
//   1. per point its bin (the block holding its ROE lattice point; inactive
//      points go to a last, sentinel bin) and a workgroup-privatised count;
//   2. exclusive scan of the bin counts into per-bin cursors;
//   3. scatter of each point's record (coordinates and original index) into
//      bin order (workgroup-privatised ranks, one global atomic per touched
//      bin per workgroup);
//   4. evaluation in bin order: each work-item reads one record, contiguous
//      in memory, and writes its results to the record's original index.
// Moving the coordinates in step 3 (a scattered 16-byte store per point)
// rather than reading them through an index in step 4 (a scattered load that
// costs a full cache line per point) roughly halves the bytes the path moves.
// The order inside a bin varies from run to run; every output is the same
// function of its own point, so the results are bit-identical to lsp_eval.
#include <hip/hip_runtime.h>

#include "lsp_binned.h"
#include "lsp_kernels.h"
#include "lsp_mfma.h"
#include "lsp_split.h"

namespace lsp {

namespace {

// Binning workgroups: 1024 work-items x 16 points.  Large chunks keep the
// number of global counter updates (one per touched bin per workgroup) low,
// and each bin's counter sits on its own 128-byte line so that updates to
// different bins are spread over the L2 channels instead of queueing on a few.
constexpr int kBinBlk = 1024;
constexpr int kPtsPerThr = 16;
constexpr int kCtr = 32;  // ints between consecutive bin counters

// Bin of a located point: the block of 2^lb padded coset indices holding its
// ROE lattice point (coset index floor(k / D)); inactive points go to the
// sentinel bin nbins.
template <int KIND>
__device__ __forceinline__ int bin_index(const Loc& L, const VolGeom& g, const BinGeom& bg) {
    constexpr int D = TablesOf<KIND>::kD;
    if (!L.active) return bg.nbins;
    int b[3];
    for (int a = 0; a < 3; ++a) {
        const int K = (D == 1 ? L.k[a] : (L.k[a] >> 1)) + g.pad;
        b[a] = K >> bg.lb;
    }
    return (b[2] * bg.nb[1] + b[1]) * bg.nb[0] + b[0];
}

template <int KIND, class PT>
__device__ __forceinline__ int bin_of(const PT x[3], const VolGeom& g, const BinGeom& bg) {
    Loc L;
    locate<KIND>(x, g, L);
    return bin_index<KIND>(L, g, bg);
}

// p[t * stride] = 0 for t < n.
__global__ __launch_bounds__(256) void k_zero(int* __restrict__ p, int n, int stride) {
    for (int t = blockIdx.x * 256 + threadIdx.x; t < n; t += gridDim.x * 256) p[(size_t)t * stride] = 0;
}

// Dynamic LDS: nbins + 1 ints.
template <int KIND, class PT>
__global__ __launch_bounds__(kBinBlk) void k_bin_count(const PT* __restrict__ pts, int N, VolGeom g,
                                                       BinGeom bg, int* __restrict__ bin,
                                                       int* __restrict__ count) {
    extern __shared__ int h[];
    for (int t = threadIdx.x; t <= bg.nbins; t += kBinBlk) h[t] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * kBinBlk * kPtsPerThr;
    for (int k = 0; k < kPtsPerThr; ++k) {
        const int i = (int)min(base + k * kBinBlk + (long long)threadIdx.x, (long long)N);
        if (i < N) {
            PT x[3];
            load_point(pts, i, x);
            const int b = bin_of<KIND>(x, g, bg);
            bin[i] = b;
            atomicAdd(&h[b], 1);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= bg.nbins; t += kBinBlk)
        if (h[t]) atomicAdd(&count[t * kCtr], h[t]);
}

// cursor[b kCtr] = sum of count[0..b) (both strided by kCtr); one workgroup,
// n = nbins + 1 <= kMaxBins + 1.
__global__ __launch_bounds__(1024) void k_bin_scan(const int* __restrict__ count, int n,
                                                   int* __restrict__ cursor) {
    __shared__ int part[1024];
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    int s = 0;
    for (int t = lo; t < hi; ++t) s += count[t * kCtr];
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
        cursor[t * kCtr] = run;
        run += count[t * kCtr];
    }
}

// Dynamic LDS: 2 (nbins + 1) ints.  Same chunking as k_bin_count.
template <class PT>
__global__ __launch_bounds__(kBinBlk) void k_bin_scatter(const PT* __restrict__ pts,
                                                         const int* __restrict__ bin, int N,
                                                         BinGeom bg, int* __restrict__ cursor,
                                                         Rec<PT>* __restrict__ rec) {
    extern __shared__ int lds[];
    int* h = lds;
    int* hb = lds + bg.nbins + 1;
    for (int t = threadIdx.x; t <= bg.nbins; t += kBinBlk) h[t] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * kBinBlk * kPtsPerThr;
    int b[kPtsPerThr], r[kPtsPerThr];
#pragma unroll
    for (int k = 0; k < kPtsPerThr; ++k) {
        const int i = (int)min(base + k * kBinBlk + (long long)threadIdx.x, (long long)N);
        b[k] = i < N ? bin[i] : 0;
        r[k] = i < N ? atomicAdd(&h[b[k]], 1) : 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= bg.nbins; t += kBinBlk)
        if (h[t]) hb[t] = atomicAdd(&cursor[t * kCtr], h[t]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPtsPerThr; ++k) {
        const int i = (int)min(base + k * kBinBlk + (long long)threadIdx.x, (long long)N);
        if (i < N) {
            Rec<PT> q;
            load_point(pts, i, q.x);
            q.i = i;
            rec[hb[b[k]] + r[k]] = q;
        }
    }
}

template <int KIND, class CT, class PT, int MODE>
__global__ __launch_bounds__(256) void k_eval_binned(const Rec<PT>* __restrict__ rec, int N,
                                                     const void* __restrict__ coef, unsigned nbytes,
                                                     VolGeom g, float* __restrict__ out,
                                                     float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const Rec<PT> q = rec[p];
    eval_at<KIND, CT, PT, MODE, false>(q.x, q.i, coef, nbytes, g, out, grad, nullptr);
}

// Four lanes per record for the separable splines (the same per-point body
// as the direct entry points, so the results agree bit for bit).
template <int KIND, class CT, class PT, int MODE>
__global__ __launch_bounds__(256) void k_eval_binned_split(const Rec<PT>* __restrict__ rec, int N,
                                                           const void* __restrict__ coef,
                                                           unsigned nbytes, VolGeom g,
                                                           float* __restrict__ out,
                                                           float* __restrict__ grad) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long p = t >> 2;
    const bool has = p < N;
    Rec<PT> q{};
    if (has) q = rec[p];
    eval_split_at<KIND, CT, PT, MODE>(q.x, q.i, has, (int)(t & 3), coef, nbytes, g, out, grad,
                                      nullptr);
}

// Matrix-core evaluation in bin order; block b handles records
// [b * 256 * ppt, (b + 1) * 256 * ppt), 256 at a time.
template <int KIND, class CT, class PT, int MODE>
__global__ __launch_bounds__(256) void k_eval_binned_mfma(const Rec<PT>* __restrict__ rec, int N,
                                                          int ppt, const void* __restrict__ coef,
                                                          unsigned nbytes, VolGeom g,
                                                          float* __restrict__ out,
                                                          float* __restrict__ grad) {
    u32x4_t W[2][2];
    load_weight_operands<KIND, CT>(W);
    const __amdgpu_buffer_rsrc_t r = make_rsrc(coef, nbytes);
    for (int it = 0; it < ppt; ++it) {
        const long long base = ((long long)blockIdx.x * ppt + it) * 256 + (threadIdx.x & ~63);
        if (base >= N) break;  // uniform over the wavefront
        const int p = (int)base + (threadIdx.x & 63);
        const bool valid = p < N;
        Rec<PT> q{};
        if (valid) q = rec[p];
        eval_mfma_wave<KIND, CT, PT, MODE>(q.x, q.i, valid, W, r, g, out, grad);
    }
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Parts {
    size_t bin, count, cursor, rec, total;
};

Parts parts(const BinGeom& bg, int N, bool pts_f64) {
    Parts q{};
    const size_t n = (size_t)(N > 0 ? N : 1);
    size_t o = 0;
    q.bin = o; o += a256(4 * n);
    q.count = o; o += a256(4 * kCtr * ((size_t)bg.nbins + 1));
    q.cursor = o; o += a256(4 * kCtr * ((size_t)bg.nbins + 1));
    q.rec = o; o += a256(n * (pts_f64 ? sizeof(Rec<double>) : sizeof(Rec<float>)));
    q.total = o;
    return q;
}

template <int KIND, class CT, class PT>
hipError_t run(const BinnedArgs& a, const Parts& q) {
    char* ws = static_cast<char*>(a.ws);
    int* bin = reinterpret_cast<int*>(ws + q.bin);
    int* count = reinterpret_cast<int*>(ws + q.count);
    int* cursor = reinterpret_cast<int*>(ws + q.cursor);
    Rec<PT>* rec = reinterpret_cast<Rec<PT>*>(ws + q.rec);
    const PT* pts = static_cast<const PT*>(a.pts);
    const int N = a.N;
    const int nb1 = a.bg.nbins + 1;
    hipLaunchKernelGGL(k_zero, dim3((nb1 + 255) / 256), dim3(256), 0, a.stream, count, nb1, kCtr);
    const int chunk = kBinBlk * kPtsPerThr;
    const int cblocks = (int)(((long long)N + chunk - 1) / chunk);
    hipLaunchKernelGGL((k_bin_count<KIND, PT>), dim3(cblocks), dim3(kBinBlk), nb1 * sizeof(int),
                       a.stream, pts, N, a.g, a.bg, bin, count);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, a.stream, count, nb1, cursor);
    hipLaunchKernelGGL((k_bin_scatter<PT>), dim3(cblocks), dim3(kBinBlk), 2 * nb1 * sizeof(int),
                       a.stream, pts, bin, N, a.bg, cursor, rec);
    if constexpr (mfma_eligible<KIND>()) {
        if (a.mfma) {
            const int ppt = N / (256 * 2048) < 1 ? 1 : (N / (256 * 2048) > 8 ? 8 : N / (256 * 2048));
            const int mblocks = (int)(((long long)N + 256 * ppt - 1) / (256 * ppt));
            if (a.grad)
                hipLaunchKernelGGL((k_eval_binned_mfma<KIND, CT, PT, kValueGrad>), dim3(mblocks),
                                   dim3(256), 0, a.stream, rec, N, ppt, a.coef, a.nbytes, a.g, a.out,
                                   a.grad);
            else
                hipLaunchKernelGGL((k_eval_binned_mfma<KIND, CT, PT, kValue>), dim3(mblocks),
                                   dim3(256), 0, a.stream, rec, N, ppt, a.coef, a.nbytes, a.g, a.out,
                                   a.grad);
            return hipGetLastError();
        }
    }
    if constexpr (split_eligible<KIND>()) {
        if (N <= split_limit<KIND>(a.split_maxn)) {
            // records carry their output index, so a chunk is a range of records
            for (long long s = 0; s < N; s += kSplitChunk) {
                const int n = (int)(N - s < kSplitChunk ? N - s : kSplitChunk);
                const int sblocks = (int)(((long long)n * kSplitLanes + 255) / 256);
                if (a.grad)
                    hipLaunchKernelGGL((k_eval_binned_split<KIND, CT, PT, kValueGrad>), dim3(sblocks),
                                       dim3(256), 0, a.stream, rec + s, n, a.coef, a.nbytes, a.g, a.out,
                                       a.grad);
                else
                    hipLaunchKernelGGL((k_eval_binned_split<KIND, CT, PT, kValue>), dim3(sblocks),
                                       dim3(256), 0, a.stream, rec + s, n, a.coef, a.nbytes, a.g, a.out,
                                       a.grad);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
    }
    const int eblocks = (int)(((long long)N + 255) / 256);
    if (a.grad)
        hipLaunchKernelGGL((k_eval_binned<KIND, CT, PT, kValueGrad>), dim3(eblocks), dim3(256), 0,
                           a.stream, rec, N, a.coef, a.nbytes, a.g, a.out, a.grad);
    else
        hipLaunchKernelGGL((k_eval_binned<KIND, CT, PT, kValue>), dim3(eblocks), dim3(256), 0,
                           a.stream, rec, N, a.coef, a.nbytes, a.g, a.out, a.grad);
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
    return parts(bg, N, pts_f64).total;
}

hipError_t launch_binned(const BinnedArgs& a) {
    if (a.N <= 0) return hipSuccess;
    if (a.bg.nbins > kMaxBins) return hipErrorInvalidValue;
    const Parts q = parts(a.bg, a.N, a.pts_f64);
    if (a.ws_bytes < q.total) return hipErrorInvalidValue;
#define LSP_RUN(k) \
    if (a.kind == k) return a.pts_f64 ? run_ct<k, double>(a, q) : run_ct<k, float>(a, q);
    LSP_FOR_EACH_KIND(LSP_RUN)
#undef LSP_RUN
    return hipErrorInvalidValue;
}

}  // namespace lsp
