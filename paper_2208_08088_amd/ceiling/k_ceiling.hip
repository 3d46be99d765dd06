// Bandwidth ceilings of this device, measured beside the multiply: plain
// streams over buffers far larger than the last-level cache with the same
// 16-byte buffer accesses the multiply kernels use.  They bound what a
// kernel with the same mix of reads and writes can reach, so a multiply's
// rate can be stated as a fraction of them.  Used by the benchmark only;
// the multiply library does not link this code.
//
//   ceiling_read   reads `bytes` (one read stream)
//   ceiling_write  writes `bytes` (one write stream)
//   ceiling_copy   reads `bytes` and writes `bytes` (1 read : 1 write, the
//                  mix of C = A*B at beta = 0 with equal A and C rows)
//   ceiling_mix2   reads 2 x `bytes` and writes `bytes` (2 : 1, the mix at
//                  beta != 0): dst = src ^ dst in place, so each line that
//                  is written was read just before, as C is at beta != 0
//   ceiling_mfma   matrix-core products only, no memory traffic: the
//                  sustained rate of back-to-back binary64 16x16x4 or
//                  bfloat16 32x32x16 products on operands taken from a
//                  buffer (random values, or zeros): the clock of this part
//                  falls with the switching activity of the operands, so
//                  the rate on random data bounds what any kernel of that
//                  product reaches on such data
//
// Every entry point takes device pointers, a byte count that is a multiple
// of the work item (256 lanes x 16 bytes x unroll), the launch shape
// (workgroups, unroll 2/4/8), the cache policy of the loads and of the
// stores (0 default, 1 non-temporal), the item layout (0: the workgroup's
// four wavefronts interleave at 1 KiB, 1: each wavefront owns unroll
// contiguous KiB of the item, as a multiply kernel's wavefront owns its row
// tiles) and a HIP stream, and returns a hipError_t.  Each workgroup walks
// its work items with a grid stride and a two-stage register pipeline: the
// next item's loads are in flight while the current item is stored.  Buffers are addressed through resources of
// 1 GiB windows; loads past a window read 0 without touching memory.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr int64_t kWindow = int64_t(1) << 30;  // bytes addressed through one resource

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)(uint32_t)bytes, 0x00020000);
}

// Byte offset of vector u of this lane within an item (WC: wave-contiguous).
template <int UNROLL, bool WC>
__device__ __forceinline__ int item_off(int u) {
    if constexpr (WC)
        return (int)(threadIdx.x >> 6) * (UNROLL * 1024) + u * 1024 + (int)(threadIdx.x & 63) * 16;
    else
        return u * kBlock * 16 + (int)threadIdx.x * 16;
}

template <int UNROLL, int NR, int LP, bool WC>
__device__ __forceinline__ void load_item(__amdgpu_buffer_rsrc_t r0, __amdgpu_buffer_rsrc_t r1, int base,
                                          u32x4 (&v)[UNROLL]) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int off = base + item_off<UNROLL, WC>(u);
        v[u] = u32x4{0u, 0u, 0u, 0u};
        if constexpr (NR >= 1) v[u] = __builtin_amdgcn_raw_buffer_load_b128(r0, off, 0, LP);
        if constexpr (NR >= 2) v[u] ^= __builtin_amdgcn_raw_buffer_load_b128(r1, off, 0, LP);
    }
}

// LP / SP: cache policy bits of loads / stores (0 or 2 = non-temporal).
template <int UNROLL, int NR, bool WRITE, int LP, int SP, bool WC>
__global__ __launch_bounds__(kBlock) void k_stream(const char *__restrict__ s0, const char *__restrict__ s1,
                                                   char *__restrict__ d, int64_t bytes, u32x4 *__restrict__ sink) {
    constexpr int kItem = kBlock * 16 * UNROLL;  // bytes per work item
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (int64_t w0 = 0; w0 < bytes; w0 += kWindow) {
        const int64_t wb = bytes - w0 < kWindow ? bytes - w0 : kWindow;
        const __amdgpu_buffer_rsrc_t r0 = rsrc(s0 ? s0 + w0 : nullptr, NR >= 1 ? wb : 0);
        const __amdgpu_buffer_rsrc_t r1 = rsrc(s1 ? s1 + w0 : nullptr, NR >= 2 ? wb : 0);
        const __amdgpu_buffer_rsrc_t rd = rsrc(d ? d + w0 : nullptr, WRITE ? wb : 0);
        const int items = (int)(wb / kItem);
        u32x4 v[UNROLL], vn[UNROLL];
        int it = blockIdx.x;
        // offsets stay below 2^31: items * kItem <= 2^30 and the grid adds
        // at most 2^12 items of at most 2^15 bytes
        load_item<UNROLL, NR, LP, WC>(r0, r1, it * kItem, v);
        for (; it < items; it += gridDim.x) {
            // past the last item the offset lies beyond the window: zeros, no traffic
            load_item<UNROLL, NR, LP, WC>(r0, r1, (it + (int)gridDim.x) * kItem, vn);
            const int base = it * kItem;
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                if constexpr (WRITE) {
                    const int off = base + item_off<UNROLL, WC>(u);
                    const u32x4 o = NR == 0 ? u32x4{(uint32_t)off, 1u, 2u, 3u} : v[u];
                    __builtin_amdgcn_raw_buffer_store_b128(o, rd, off, 0, SP);
                } else {
                    acc ^= v[u];
                }
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) v[u] = vn[u];
        }
    }
    if constexpr (!WRITE) sink[(int64_t)blockIdx.x * kBlock + threadIdx.x] = acc;
}

template <int NR, bool WRITE, int LP, int SP, bool WC>
hipError_t launch_u(const char *a, const char *b, char *c, int64_t bytes, int grid, int unroll, u32x4 *k,
                    hipStream_t st) {
    switch (unroll) {
    case 2: hipLaunchKernelGGL((k_stream<2, NR, WRITE, LP, SP, WC>), dim3(grid), dim3(kBlock), 0, st, a, b, c, bytes, k); break;
    case 4: hipLaunchKernelGGL((k_stream<4, NR, WRITE, LP, SP, WC>), dim3(grid), dim3(kBlock), 0, st, a, b, c, bytes, k); break;
    case 8: hipLaunchKernelGGL((k_stream<8, NR, WRITE, LP, SP, WC>), dim3(grid), dim3(kBlock), 0, st, a, b, c, bytes, k); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NR, bool WRITE, int LP, int SP>
hipError_t launch_l(const char *a, const char *b, char *c, int64_t bytes, int grid, int unroll, int layout, u32x4 *k,
                    hipStream_t st) {
    return layout ? launch_u<NR, WRITE, LP, SP, true>(a, b, c, bytes, grid, unroll, k, st)
                  : launch_u<NR, WRITE, LP, SP, false>(a, b, c, bytes, grid, unroll, k, st);
}

template <int NR, bool WRITE>
hipError_t launch(const void *s0, const void *s1, void *d, int64_t bytes, int grid, int unroll, int lpol, int spol,
                  int layout, void *sink, hipStream_t st) {
    if (unroll != 2 && unroll != 4 && unroll != 8) return hipErrorInvalidValue;
    const int64_t item = (int64_t)kBlock * 16 * unroll;
    if (bytes <= 0 || grid < 1 || grid > 4096 || bytes % item != 0 || (lpol != 0 && lpol != 1) ||
        (spol != 0 && spol != 1) || (layout != 0 && layout != 1))
        return hipErrorInvalidValue;
    const char *a = static_cast<const char *>(s0), *b = static_cast<const char *>(s1);
    char *c = static_cast<char *>(d);
    u32x4 *k = static_cast<u32x4 *>(sink);
    if (lpol == 0 && spol == 0) return launch_l<NR, WRITE, 0, 0>(a, b, c, bytes, grid, unroll, layout, k, st);
    if (lpol == 0 && spol == 1) return launch_l<NR, WRITE, 0, 2>(a, b, c, bytes, grid, unroll, layout, k, st);
    if (lpol == 1 && spol == 0) return launch_l<NR, WRITE, 2, 0>(a, b, c, bytes, grid, unroll, layout, k, st);
    return launch_l<NR, WRITE, 2, 2>(a, b, c, bytes, grid, unroll, layout, k, st);
}

typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// Matrix-core ceiling: every lane holds 8 A and 8 B operand vectors read
// from `src` (so their values are the buffer's), and issues 32 products per
// iteration into independent accumulators (consecutive products never
// depend on each other), with a different operand pair for every product.
// The operands and accumulators fit the architectural registers, so the
// loop is the products alone.  KIND 0: binary64 16x16x4 (2048 flops each,
// 8 accumulators); KIND 1: bfloat16 32x32x16 (32768 flops each, 4
// accumulators).  The accumulators go to `sink` so nothing is dropped.
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_mfma(const u32x4 *__restrict__ src, int iters, u32x4 *__restrict__ sink) {
    const int lane = threadIdx.x & 63;
    u32x4 a[8], b[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = src[i * 64 + lane];
        b[i] = src[(8 + i) * 64 + lane];
    }
    u32x4 out = {0u, 0u, 0u, 0u};
    if constexpr (KIND == 0) {
        d4v acc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = d4v{};
        d2v da[8], db[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            da[i] = __builtin_bit_cast(d2v, a[i]);
            db[i] = __builtin_bit_cast(d2v, b[i]);
        }
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const int hx = (u / 8) & 1, hy = ((u / 8) + (u / 16)) & 1;
                acc[u % 8] = __builtin_amdgcn_mfma_f64_16x16x4f64(da[u % 8][hx], db[(u * 3 + 1) % 8][hy], acc[u % 8],
                                                                  0, 0, 0);
            }
        }
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) t += acc[i][r];
        const uint64_t bits = __builtin_bit_cast(uint64_t, t);
        out[0] = (uint32_t)bits;
        out[1] = (uint32_t)(bits >> 32);
    } else {
        f16v acc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = f16v{};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int u = 0; u < 32; ++u)
                acc[u % 4] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8v, a[u % 8]),
                                                                    __builtin_bit_cast(bf8v, b[(u * 3 + 1 + u / 8) % 8]),
                                                                    acc[u % 4], 0, 0, 0);
        }
        float t = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) t += acc[i][r];
        out[0] = __builtin_bit_cast(uint32_t, t);
    }
    sink[(int64_t)blockIdx.x * kBlock + threadIdx.x] = out;
}

}  // namespace

extern "C" {

// src: device memory of 16 * 64 16-byte vectors (the operands); sink:
// grid * 256 16-byte vectors.  kind 0: binary64 16x16x4, 1: bfloat16
// 32x32x16.  Flops: grid * 4 wavefronts * iters * 32 * (2048 or 32768).
int ceiling_mfma(const void *src, void *sink, int kind, int grid, int iters, void *stream) {
    if (!src || !sink || grid < 1 || grid > 4096 || iters < 1 || (kind != 0 && kind != 1))
        return (int)hipErrorInvalidValue;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const u32x4 *s = static_cast<const u32x4 *>(src);
    u32x4 *k = static_cast<u32x4 *>(sink);
    if (kind == 0) hipLaunchKernelGGL(k_mfma<0>, dim3(grid), dim3(kBlock), 0, st, s, iters, k);
    else hipLaunchKernelGGL(k_mfma<1>, dim3(grid), dim3(kBlock), 0, st, s, iters, k);
    return (int)hipGetLastError();
}


// sink: device memory of grid * 256 * 16 bytes (the read stream's result,
// so the loads cannot be dropped).
int ceiling_read(const void *src, int64_t bytes, void *sink, int grid, int unroll, int lpol, int layout,
                 void *stream) {
    if (!src || !sink) return (int)hipErrorInvalidValue;
    return (int)launch<1, false>(src, nullptr, nullptr, bytes, grid, unroll, lpol, 0, layout, sink,
                                 static_cast<hipStream_t>(stream));
}

int ceiling_write(void *dst, int64_t bytes, int grid, int unroll, int spol, int layout, void *stream) {
    if (!dst) return (int)hipErrorInvalidValue;
    return (int)launch<0, true>(nullptr, nullptr, dst, bytes, grid, unroll, 0, spol, layout, nullptr,
                                static_cast<hipStream_t>(stream));
}

int ceiling_copy(const void *src, void *dst, int64_t bytes, int grid, int unroll, int lpol, int spol, int layout,
                 void *stream) {
    if (!src || !dst) return (int)hipErrorInvalidValue;
    return (int)launch<1, true>(src, nullptr, dst, bytes, grid, unroll, lpol, spol, layout, nullptr,
                                static_cast<hipStream_t>(stream));
}

// dst is read and written in place (its second source is itself).
int ceiling_mix2(const void *src, void *dst, int64_t bytes, int grid, int unroll, int lpol, int spol, int layout,
                 void *stream) {
    if (!src || !dst) return (int)hipErrorInvalidValue;
    return (int)launch<2, true>(src, dst, dst, bytes, grid, unroll, lpol, spol, layout, nullptr,
                                static_cast<hipStream_t>(stream));
}

}  // extern "C"
