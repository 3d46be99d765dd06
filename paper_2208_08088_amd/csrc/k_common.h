// Device helpers shared by the libtsmm kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tsmm {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core product for binary64 / binary32 (one A and one B
// element per lane, four accumulator rows per lane).  Lane 16*q + j
// supplies A(row j, k-slot q) and B(k-slot q, column j) in both types; its
// accumulator element r holds column j of row row(q, r), which is q + 4*r
// for V_MFMA_F64_16X16X4_F64 and 4*q + r for V_MFMA_F32_16X16X4_F32
// (established by an on-device layout probe).
template <typename T> struct Mfma4;
template <> struct Mfma4<double> {
    typedef d4v acc;
    typedef d2v vec;  // one 16-byte vector
    static constexpr int VW = 2;
    static __device__ __forceinline__ int row(int q, int r) { return q + 4 * r; }
    static __device__ __forceinline__ acc op(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma4<float> {
    typedef f4v acc;
    typedef f4v vec;
    static constexpr int VW = 4;
    static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
    static __device__ __forceinline__ acc op(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// The binary64 epilogue RN(RN(alpha*acc) + RN(beta*c)); never fused.
// beta == 0 ignores c (which the caller then never loads).
__device__ __forceinline__ double epilogue(double alpha, double acc, double beta, double c) {
#pragma clang fp contract(off)
    double t = alpha * acc;
    if (beta != 0.0) t = t + beta * c;
    return t;
}

__device__ __forceinline__ float bf16_bits_to_float(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// binary32 -> bfloat16 bits, round to nearest even (finite inputs; a NaN
// input stays a NaN).
__device__ __forceinline__ uint16_t float_to_bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Raw buffer access (the hardware clamps every access against the byte
// count of the resource: out-of-range loads return 0, out-of-range stores
// are dropped).  The range check covers the per-lane offset only, so every
// offset that must be checked goes into `voff`; `aux` 2 marks the access
// non-temporal (streamed once).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// A value that is the same in every lane, moved to scalar registers (the
// compiler cannot always prove it, and a buffer resource must be scalar).
__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, int64_t bytes) {
    const int64_t b = bytes < 0 ? 0 : (bytes > (int64_t)0xFFFFFFFF ? (int64_t)0xFFFFFFFF : bytes);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)(uint32_t)b, 0x00020000);
}

// Byte offset outside any tile-sized resource: an access through it reads
// 0 or is dropped.  Every resource that takes it spans at most 2^30 bytes
// (the planner keeps 16 rows of a strided operand within that).
constexpr int kOOB = 0x40000000;

// Rows of the 16-row tile starting at row0 that exist in an m-row matrix.
__device__ __forceinline__ int64_t tile_rows(int64_t m, int64_t row0) {
    const int64_t r = m - row0;
    return r < 0 ? 0 : (r > 16 ? 16 : r);
}

template <typename T> struct BufIO;
// AUX is the cache policy of a load: 2 (streaming) where each instruction
// covers whole 128-byte lines, 0 (default) where it covers part of a line
// that the next loads of the same wavefront complete (a streaming load
// would not keep the line for them).
template <> struct BufIO<double> {
    template <int AUX = 2>
    static __device__ __forceinline__ d2v load_vec(__amdgpu_buffer_rsrc_t r, int voff) {
        return __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, AUX));
    }
    template <int AUX = 2>
    static __device__ __forceinline__ double load1(__amdgpu_buffer_rsrc_t r, int voff) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, AUX));
    }
    template <int AUX = 2>
    static __device__ __forceinline__ void store1(double v, __amdgpu_buffer_rsrc_t r, int voff) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, 0, AUX);
    }
    template <int AUX = 2>
    static __device__ __forceinline__ void store_vec(d2v v, __amdgpu_buffer_rsrc_t r, int voff) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, 0, AUX);
    }
};
template <> struct BufIO<float> {
    template <int AUX = 2>
    static __device__ __forceinline__ f4v load_vec(__amdgpu_buffer_rsrc_t r, int voff) {
        return __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, AUX));
    }
    template <int AUX = 2>
    static __device__ __forceinline__ float load1(__amdgpu_buffer_rsrc_t r, int voff) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, AUX));
    }
    template <int AUX = 2>
    static __device__ __forceinline__ void store1(float v, __amdgpu_buffer_rsrc_t r, int voff) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, 0, AUX);
    }
    template <int AUX = 2>
    static __device__ __forceinline__ void store_vec(f4v v, __amdgpu_buffer_rsrc_t r, int voff) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, 0, AUX);
    }
};

template <typename T> __device__ __forceinline__ double to_f64(T x) { return (double)x; }
template <typename T> __device__ __forceinline__ T from_f64(double x) { return (T)x; }

}  // namespace tsmm
