// Coefficient packing: caller coset arrays (C order [z][y][x]) are converted
// to the storage type and written into the interior of the zero-halo
// internal buffer.  Runs once per lsp_volume_set_coeffs, not on the hot path.
#include <hip/hip_runtime.h>

#include "lsp_launch.h"

namespace lsp {

namespace {

// Float to bfloat16, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
    unsigned b = __builtin_bit_cast(unsigned, f);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (unsigned short)(b >> 16);
}

// Double to float rounding to odd: a correct intermediate for a second
// rounding to a format with at most 22 significand bits (bf16, fp16), so the
// composition is a single round-to-nearest-even of the double.
__device__ __forceinline__ float f64_to_f32_odd(double d) {
    float f = (float)d;
    if ((double)f != d && f == f && !__builtin_isinf(f)) {
        unsigned b = __builtin_bit_cast(unsigned, f);
        const bool away = __builtin_fabs((double)f) > __builtin_fabs(d);
        if (away) b -= 1u;
        b |= 1u;
        f = __builtin_bit_cast(float, b);
    }
    return f;
}

template <int SRC>
__device__ __forceinline__ float src_f32(const void* p, size_t i, bool for_narrow) {
    if (SRC == 0) return static_cast<const float*>(p)[i];
    if (SRC == 1) {
        const double d = static_cast<const double*>(p)[i];
        return for_narrow ? f64_to_f32_odd(d) : (float)d;
    }
    const unsigned short h = static_cast<const unsigned short*>(p)[i];
    if (SRC == 2) return __builtin_bit_cast(float, (unsigned)h << 16);
    return (float)__builtin_bit_cast(_Float16, h);
}

template <int SRC, int DST>
__global__ __launch_bounds__(256) void k_pack(const void* __restrict__ src, void* __restrict__ dst,
                                              long long n, int X, int Y, VolGeom g, int coset) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int x = (int)(i % X);
        const long long r = i / X;
        const int y = (int)(r % Y);
        const int z = (int)(r / Y);
        const float v = src_f32<SRC>(src, (size_t)i, DST != kCF32);
        const int idx[3] = {x + g.pad, y + g.pad, z + g.pad};
        const int off = site_offset(g, idx, coset);
        char* d = static_cast<char*>(dst) + off;
        if (DST == kCF32) {
            *reinterpret_cast<float*>(d) = v;
        } else if (DST == kCBF16) {
            *reinterpret_cast<unsigned short*>(d) = f32_to_bf16(v);
        } else {
            *reinterpret_cast<unsigned short*>(d) = __builtin_bit_cast(unsigned short, (_Float16)v);
        }
    }
}

template <int SRC>
hipError_t pack_src(const void* src, int ctype, void* dst, long long n, int X, int Y,
                    const VolGeom& g, int coset, hipStream_t s) {
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    switch (ctype) {
        case kCF32:
            hipLaunchKernelGGL((k_pack<SRC, kCF32>), dim3((unsigned)blocks), dim3(256), 0, s, src,
                               dst, n, X, Y, g, coset);
            break;
        case kCBF16:
            hipLaunchKernelGGL((k_pack<SRC, kCBF16>), dim3((unsigned)blocks), dim3(256), 0, s, src,
                               dst, n, X, Y, g, coset);
            break;
        case kCF16:
            hipLaunchKernelGGL((k_pack<SRC, kCF16>), dim3((unsigned)blocks), dim3(256), 0, s, src,
                               dst, n, X, Y, g, coset);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pack(const void* src, int src_dtype, int ctype, void* dst, const int64_t dims[3],
                       const VolGeom& g, int coset, hipStream_t stream) {
    const long long n = (long long)dims[0] * dims[1] * dims[2];
    if (n == 0) return hipSuccess;
    const int X = (int)dims[0], Y = (int)dims[1];
    switch (src_dtype) {
        case 0: return pack_src<0>(src, ctype, dst, n, X, Y, g, coset, stream);  // F32
        case 1: return pack_src<1>(src, ctype, dst, n, X, Y, g, coset, stream);  // F64
        case 2: return pack_src<2>(src, ctype, dst, n, X, Y, g, coset, stream);  // BF16
        case 3: return pack_src<3>(src, ctype, dst, n, X, Y, g, coset, stream);  // F16
    }
    return hipErrorInvalidValue;
}

}  // namespace lsp
