// dL/dc of the convolution sum without floating-point atomics:
//
//   dL/dc_n = sum_i g_i phi(x_i - n)
//
// Each point only touches the stencil of its region of evaluation, so the
// pass is organised around ROE cells (the lattice point k of Algorithm 1):
//   1. key every point by its cell (inactive points get a sentinel key);
//   2. stable radix sort of (cell, point index)   -- a library sort;
//   3. cell start offsets by lower-bound search on the sorted keys;
//   4. per cell, partial sums P[u][cell] over the cell's points (sorted
//      order) for every offset v_u of the symmetry-closed stencil U: each
//      point's weights g_i w_j(y_i) (the per-tap polynomials of the reference
//      sub-region) are formed on the fly, and a point with symmetry element G
//      reaches the site cell + v_u through the tap j with G^T o_j = v_u
//      (generated table J[G][u], inverted to u(G, j));
//   5. per stored site n, dL/dc_n = sum over u of P[u][n - v_u].
// Every sum runs in a fixed order (sorted points, then U), so the result is
// bit-reproducible.
#include <hip/hip_runtime.h>

#include <string.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "lsp_backward.h"
#include "lsp_kernels.h"

namespace lsp {

namespace {

constexpr int kBlk = 256;


// Cell grid: the padded per-coset grid of the coefficient layout, one cell
// per lattice point, cell = coset * NC + ((K_z + pad) * PY + K_y + pad) * PX + K_x + pad
// with K = floor(k / D).
struct CellGeom {
    int PX, PY, PZ, NC;
    int pad;
    int ncell;
};


template <int KIND>
__device__ __forceinline__ int cell_of(const int k[3], const CellGeom& cg) {
    constexpr int D = TablesOf<KIND>::kD;
    const int K0 = D == 1 ? k[0] : (k[0] >> 1);
    const int K1 = D == 1 ? k[1] : (k[1] >> 1);
    const int K2 = D == 1 ? k[2] : (k[2] >> 1);
    const int m = coset_of_parity<KIND>(k[0] & 1, k[1] & 1, k[2] & 1);
    return m * cg.NC + ((K2 + cg.pad) * cg.PY + (K1 + cg.pad)) * cg.PX + (K0 + cg.pad);
}

template <int KIND, class PT>
__global__ __launch_bounds__(kBlk) void k_bin_keys(const PT* __restrict__ pts, int N, VolGeom g,
                                                   CellGeom cg, int* __restrict__ keys,
                                                   int* __restrict__ vals) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    if (i >= N) return;
    PT x[3];
    load_point(pts, i, x);
    Loc L;
    locate<KIND>(x, g, L);
    keys[i] = L.active ? cell_of<KIND>(L.k, cg) : cg.ncell;
    vals[i] = i;
}

// off[c] = first sorted position whose key is >= c, for c in [0, ncell].
__global__ __launch_bounds__(kBlk) void k_cell_offsets(const int* __restrict__ keys, int N,
                                                       int ncell, int* __restrict__ off) {
    const int stride = gridDim.x * kBlk;
    for (int c = blockIdx.x * kBlk + threadIdx.x; c <= ncell; c += stride) {
        int lo = 0, hi = N;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (keys[mid] < c) lo = mid + 1;
            else hi = mid;
        }
        off[c] = lo;
    }
}

template <int KIND>
__device__ __forceinline__ void tap_weights(const Loc& L, float* w) {
    PolyOf<KIND>::weights(L.y[0], L.y[1], L.y[2], L.region, w);
}

constexpr int kPartBlk = 128;

// P[u][cell] = sum over the cell's points p (sorted order) of g_p w_j(y_p)
// for the tap j with G_p^T o_j = v_u.  Each thread owns one cell and keeps
// its |U| accumulators in LDS (indexed by u(G, j)); every slot has one owner,
// so the adds happen in program order and the result is reproducible.
template <int KIND, class PT>
__global__ __launch_bounds__(kPartBlk) void k_cell_partials(const PT* __restrict__ pts,
                                                            const int* __restrict__ svals,
                                                            const int* __restrict__ off,
                                                            const float* __restrict__ gin,
                                                            VolGeom g, int ncell,
                                                            float* __restrict__ P) {
    using T = TablesOf<KIND>;
    constexpr int NU = T::kNumU;
    constexpr int NT = T::kTaps;
    constexpr int SLOTS = NU | 1;   // odd stride between threads' slots
    __shared__ __attribute__((aligned(16))) unsigned char Uinv[T::kNumSym * NT];
    __shared__ float acc[kPartBlk * SLOTS];
    for (int t = threadIdx.x; t < T::kNumSym * NU; t += kPartBlk) {
        const int sg = t / NU, u = t % NU;
        const int j = T::kJ[sg][u];
        if (j >= 0) Uinv[sg * NT + j] = (unsigned char)u;
    }
    float* mine = acc + threadIdx.x * SLOTS;
    for (int u = 0; u < NU; ++u) mine[u] = 0.0f;
    __syncthreads();
    const int c = blockIdx.x * kPartBlk + threadIdx.x;
    const int b = c < ncell ? off[c] : 0, e = c < ncell ? off[c + 1] : 0;
    for (int p = b; p < e; ++p) {
        const int i = svals[p];
        PT x[3];
        load_point(pts, i, x);
        Loc L;
        locate<KIND>(x, g, L);
        float w[NT];
        tap_weights<KIND>(L, w);
        const float gi = gin[i];
        const unsigned char* ui = Uinv + sym_id<KIND>(L) * NT;
        if constexpr (NT % 16 == 0) {
            // The taps of one point land in distinct slots (u(G, j) is
            // one-to-one in j for a fixed symmetry G), so all slots are read,
            // updated and written back as independent batches instead of a
            // chain of dependent read-modify-writes; each slot gets the same
            // add.  The row of slot indices is read as 16-byte words (rows
            // are 16-byte aligned).
            int slot[NT];
#pragma unroll
            for (int q = 0; q < NT / 16; ++q) {
                const uint4 v = reinterpret_cast<const uint4*>(ui)[q];
                const unsigned wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int t = 0; t < 16; ++t) slot[16 * q + t] = (wv[t >> 2] >> (8 * (t & 3))) & 0xff;
            }
            float a[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j) a[j] = mine[slot[j]];
#pragma unroll
            for (int j = 0; j < NT; ++j) a[j] += gi * w[j];
#pragma unroll
            for (int j = 0; j < NT; ++j) mine[slot[j]] = a[j];
        } else {
#pragma unroll
            for (int j = 0; j < NT; ++j) mine[ui[j]] += gi * w[j];
        }
    }
    if (c >= ncell) return;
    for (int u = 0; u < NU; ++u) P[(size_t)u * ncell + c] = mine[u];
}

// dL/dx from a saved gradient: one thread per point.
__global__ __launch_bounds__(kBlk) void k_dx_from_grad(int N, const float* __restrict__ gin,
                                                       const float* grad, float* dL_dx) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    if (i >= N) return;
    const float gi = gin[i];
    const float a = grad[3 * (size_t)i], b = grad[3 * (size_t)i + 1], c = grad[3 * (size_t)i + 2];
    dL_dx[3 * (size_t)i] = gi * a;
    dL_dx[3 * (size_t)i + 1] = gi * b;
    dL_dx[3 * (size_t)i + 2] = gi * c;
}

// dL/dc_n = sum_u P[u][n - v_u], one thread per stored site in the canonical
// coset-major C order of the output.
template <int KIND>
__global__ __launch_bounds__(kBlk) void k_site_gather(const float* __restrict__ P, CellGeom cg,
                                                      int X, int Y, int Z, int n_cosets,
                                                      float* __restrict__ dL_dc) {
    using T = TablesOf<KIND>;
    constexpr int D = TablesOf<KIND>::kD;
    const long long per = (long long)X * Y * Z;
    const long long s = (long long)blockIdx.x * kBlk + threadIdx.x;
    if (s >= per * n_cosets) return;
    const int m = (int)(s / per);
    const long long r = s - (long long)m * per;
    const int ix = (int)(r % X);
    const int iy = (int)((r / X) % Y);
    const int iz = (int)(r / ((long long)X * Y));
    // lattice position of the site: D * idx + shift_m
    const int n0 = D * ix + T::kShift[m][0], n1 = D * iy + T::kShift[m][1],
              n2 = D * iz + T::kShift[m][2];
    // every slot's read is independent, so the loop is unrolled whole and all
    // reads can be in flight together; slots outside the cell grid read cell 0
    // and add +0,
    // which leaves the sum unchanged (it starts at +0 and never becomes -0),
    // so the summation order and the result are those of the plain loop
    float acc = 0.0f;
#pragma unroll
    for (int u = 0; u < T::kNumU; ++u) {
        const int c0 = n0 - T::kU[u][0], c1 = n1 - T::kU[u][1], c2 = n2 - T::kU[u][2];
        const int K0 = D == 1 ? c0 : (c0 >> 1);
        const int K1 = D == 1 ? c1 : (c1 >> 1);
        const int K2 = D == 1 ? c2 : (c2 >> 1);
        const bool inside = K0 >= -cg.pad && K0 < cg.PX - cg.pad && K1 >= -cg.pad &&
                            K1 < cg.PY - cg.pad && K2 >= -cg.pad && K2 < cg.PZ - cg.pad;
        const int cm = coset_of_parity<KIND>(c0 & 1, c1 & 1, c2 & 1);
        const int cell = cm * cg.NC + ((K2 + cg.pad) * cg.PY + (K1 + cg.pad)) * cg.PX + (K0 + cg.pad);
        // the read itself stays inside P for every slot (cell 0 when outside)
        const float v = P[(size_t)u * cg.ncell + (inside ? cell : 0)];
        acc += inside ? v : 0.0f;
    }
    dL_dc[s] = acc;
}

struct Layout {
    size_t keys_in, vals_in, keys_out, vals_out, off, P, tmp, total;
    size_t tmp_bytes;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int nu_of(int kind) {
#define LSP_NU(k) if (kind == k) return TablesOf<k>::kNumU;
    LSP_FOR_EACH_KIND(LSP_NU)
#undef LSP_NU
    return 0;
}

CellGeom cell_geom(const int dims[3], int pad, int n_cosets) {
    CellGeom cg{};
    cg.PX = dims[0] + 2 * pad;
    cg.PY = dims[1] + 2 * pad;
    cg.PZ = dims[2] + 2 * pad;
    cg.NC = cg.PX * cg.PY * cg.PZ;
    cg.pad = pad;
    cg.ncell = cg.NC * n_cosets;
    return cg;
}

int key_bits(int ncell) {
    int b = 1;
    while (b < 31 && (1ll << b) <= ncell) ++b;
    return b;
}

bool layout(int kind, int n_cosets, const int dims[3], int pad, long long N, Layout* L) {
    const CellGeom cg = cell_geom(dims, pad, n_cosets);
    size_t tmp = 0;
    const unsigned n = (unsigned)(N > 0 ? N : 1);
    if (rocprim::radix_sort_pairs(nullptr, tmp, (int*)nullptr, (int*)nullptr, (int*)nullptr,
                                  (int*)nullptr, n, 0, key_bits(cg.ncell)) != hipSuccess)
        return false;
    size_t o = 0;
    const size_t nb = align256(sizeof(int) * (size_t)n);
    L->keys_in = o; o += nb;
    L->vals_in = o; o += nb;
    L->keys_out = o; o += nb;
    L->vals_out = o; o += nb;
    L->off = o; o += align256(sizeof(int) * ((size_t)cg.ncell + 1));
    L->P = o; o += align256(sizeof(float) * (size_t)cg.ncell * nu_of(kind));
    L->tmp = o; o += align256(tmp);
    L->tmp_bytes = tmp;
    L->total = o;
    return true;
}

template <int KIND, class CT, class PT>
hipError_t run(const BackwardArgs& a, const Layout& ly) {
    using T = TablesOf<KIND>;
    char* ws = static_cast<char*>(a.ws);
    int* keys_in = reinterpret_cast<int*>(ws + ly.keys_in);
    int* vals_in = reinterpret_cast<int*>(ws + ly.vals_in);
    int* keys_out = reinterpret_cast<int*>(ws + ly.keys_out);
    int* vals_out = reinterpret_cast<int*>(ws + ly.vals_out);
    int* off = reinterpret_cast<int*>(ws + ly.off);
    float* P = reinterpret_cast<float*>(ws + ly.P);
    const CellGeom cg = cell_geom(a.dims, a.g.pad, a.n_cosets);
    const int N = a.N;
    const PT* pts = static_cast<const PT*>(a.pts);
    const int nblk = (int)(((long long)N + kBlk - 1) / kBlk);
    if (N > 0) {
        hipLaunchKernelGGL((k_bin_keys<KIND, PT>), dim3(nblk), dim3(kBlk), 0, a.stream, pts, N, a.g,
                           cg, keys_in, vals_in);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        size_t tmp = ly.tmp_bytes;
        e = rocprim::radix_sort_pairs(ws + ly.tmp, tmp, keys_in, keys_out, vals_in, vals_out,
                                      (unsigned)N, 0, key_bits(cg.ncell), a.stream);
        if (e != hipSuccess) return e;
    }
    {
        long long blocks = ((long long)cg.ncell + 1 + kBlk - 1) / kBlk;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_cell_offsets, dim3((unsigned)blocks), dim3(kBlk), 0, a.stream, keys_out,
                           N, cg.ncell, off);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        const int cblocks = (cg.ncell + kPartBlk - 1) / kPartBlk;
        hipLaunchKernelGGL((k_cell_partials<KIND, PT>), dim3(cblocks), dim3(kPartBlk), 0, a.stream,
                           pts, vals_out, off, a.dL_df, a.g, cg.ncell, P);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const long long sites = (long long)a.dims[0] * a.dims[1] * a.dims[2] * a.n_cosets;
    const long long gblocks = (sites + kBlk - 1) / kBlk;
    hipLaunchKernelGGL((k_site_gather<KIND>), dim3((unsigned)gblocks), dim3(kBlk), 0, a.stream, P, cg,
                       a.dims[0], a.dims[1], a.dims[2], a.n_cosets, a.dL_dc);
    (void)sizeof(T);
    return hipGetLastError();
}

template <int KIND, class CT>
hipError_t run_ct(const BackwardArgs& a, const Layout& ly) {
    return a.pts_f64 ? run<KIND, CT, double>(a, ly) : run<KIND, CT, float>(a, ly);
}

template <int KIND>
hipError_t run_pt(const BackwardArgs& a, const Layout& ly) {
    switch (a.ctype) {
        case kCF32: return run_ct<KIND, float>(a, ly);
        case kCBF16: return run_ct<KIND, bf16_t>(a, ly);
        case kCF16: return run_ct<KIND, f16_t>(a, ly);
    }
    return hipErrorInvalidValue;
}

}  // namespace

size_t backward_workspace_bytes(int kind, int n_cosets, const int64_t dims[3], int pad, int64_t N) {
    const int d[3] = {(int)dims[0], (int)dims[1], (int)dims[2]};
    Layout ly{};
    if (!layout(kind, n_cosets, d, pad, N, &ly)) return (size_t)-1;
    return ly.total;
}

hipError_t launch_dx_from_grad(long long N, const float* dL_df, const float* grad_f, float* dL_dx,
                               hipStream_t stream) {
    if (N <= 0) return hipSuccess;
    if (N > 0x7fffffffLL) return hipErrorInvalidValue;
    const int n = (int)N;
    hipLaunchKernelGGL(k_dx_from_grad, dim3((unsigned)(((long long)n + kBlk - 1) / kBlk)), dim3(kBlk), 0, stream, n, dL_df,
                       grad_f, dL_dx);
    return hipGetLastError();
}

hipError_t launch_backward_coef(const BackwardArgs& a) {
    Layout ly{};
    if (!layout(a.kind, a.n_cosets, a.dims, a.g.pad, a.N, &ly)) return hipErrorInvalidValue;
    if (a.ws_bytes < ly.total) return hipErrorInvalidValue;
#define LSP_RUN(k) if (a.kind == k) return run_pt<k>(a, ly);
    LSP_FOR_EACH_KIND(LSP_RUN)
#undef LSP_RUN
    return hipErrorInvalidValue;
}

}  // namespace lsp
