// Bandwidth ceilings of this device, measured beside the multiply: plain
// streams over buffers far larger than the last-level cache with the same
// 16-byte vector accesses the multiply kernels use.  They bound what a
// kernel with the same mix of reads and writes can reach, so a multiply's
// rate can be stated as a fraction of them.  Used by the benchmark only;
// the multiply library does not link this code.
//
//   ceiling_read   reads `bytes` (one read stream)
//   ceiling_write  writes `bytes` (one write stream)
//   ceiling_copy   reads `bytes` and writes `bytes` (1 read : 1 write, the
//                  mix of C = A*B at beta = 0 with equal A and C rows)
//   ceiling_mix2   reads 2 x `bytes` and writes `bytes` (2 : 1, the mix at
//                  beta != 0)
//
// Every entry point takes device pointers, a byte count that is a multiple
// of 16 * 64 * unroll, the launch shape (workgroups, unroll) and a HIP
// stream, and returns a hipError_t.  Loads and stores go through buffer
// resources of at most 2^31 bytes each (the buffers are walked in windows),
// with the non-temporal policy for whole lines, as in the multiply.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr int64_t kWindow = int64_t(1) << 30;  // bytes addressed through one resource

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)(uint32_t)bytes, 0x00020000);
}

// Work item w of a window: UNROLL consecutive 16-byte vectors per lane,
// 64 lanes per wavefront, wavefronts of the grid interleaved.
template <int UNROLL, int NR, bool WRITE>
__global__ __launch_bounds__(kBlock) void k_stream(const char *__restrict__ s0, const char *__restrict__ s1,
                                                   char *__restrict__ d, int64_t bytes, u32x4 *__restrict__ sink) {
    constexpr int64_t kItem = (int64_t)kBlock * 16 * UNROLL;  // bytes per workgroup step
    u32x4 acc = {0u, 0u, 0u, 0u};
    const int64_t nitems = bytes / kItem;
    for (int64_t w0 = 0; w0 < bytes; w0 += kWindow) {
        const int64_t wb = bytes - w0 < kWindow ? bytes - w0 : kWindow;
        const __amdgpu_buffer_rsrc_t r0 = rsrc(s0 ? s0 + w0 : nullptr, NR >= 1 ? wb : 0);
        const __amdgpu_buffer_rsrc_t r1 = rsrc(s1 ? s1 + w0 : nullptr, NR >= 2 ? wb : 0);
        const __amdgpu_buffer_rsrc_t rd = rsrc(d ? d + w0 : nullptr, WRITE ? wb : 0);
        const int64_t items = wb / kItem;
        (void)nitems;
        for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
            const int base = (int)(it * kItem) + threadIdx.x * 16;
            u32x4 v[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int off = base + u * kBlock * 16;
                v[u] = u32x4{0u, 0u, 0u, 0u};
                if constexpr (NR >= 1) v[u] = __builtin_amdgcn_raw_buffer_load_b128(r0, off, 0, 2);
                if constexpr (NR >= 2) v[u] ^= __builtin_amdgcn_raw_buffer_load_b128(r1, off, 0, 2);
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int off = base + u * kBlock * 16;
                if constexpr (WRITE) {
                    const u32x4 o = NR == 0 ? u32x4{(uint32_t)off, 1u, 2u, 3u} : v[u];
                    __builtin_amdgcn_raw_buffer_store_b128(o, rd, off, 0, 2);
                } else {
                    acc ^= v[u];
                }
            }
        }
    }
    if constexpr (!WRITE) sink[(int64_t)blockIdx.x * kBlock + threadIdx.x] = acc;
}

template <int NR, bool WRITE>
hipError_t launch(const void *s0, const void *s1, void *d, int64_t bytes, int grid, int unroll, void *sink,
                  hipStream_t st) {
    if (bytes <= 0 || grid < 1 || (bytes % ((int64_t)kBlock * 16 * unroll)) != 0 || (kWindow % ((int64_t)kBlock * 16 * unroll)) != 0)
        return hipErrorInvalidValue;
    const char *a = static_cast<const char *>(s0), *b = static_cast<const char *>(s1);
    char *c = static_cast<char *>(d);
    u32x4 *k = static_cast<u32x4 *>(sink);
    switch (unroll) {
    case 1: hipLaunchKernelGGL((k_stream<1, NR, WRITE>), dim3(grid), dim3(kBlock), 0, st, a, b, c, bytes, k); break;
    case 2: hipLaunchKernelGGL((k_stream<2, NR, WRITE>), dim3(grid), dim3(kBlock), 0, st, a, b, c, bytes, k); break;
    case 4: hipLaunchKernelGGL((k_stream<4, NR, WRITE>), dim3(grid), dim3(kBlock), 0, st, a, b, c, bytes, k); break;
    case 8: hipLaunchKernelGGL((k_stream<8, NR, WRITE>), dim3(grid), dim3(kBlock), 0, st, a, b, c, bytes, k); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" {

// sink: device memory of grid * 256 * 16 bytes (the read stream's result,
// so the loads cannot be dropped).
int ceiling_read(const void *src, int64_t bytes, void *sink, int grid, int unroll, void *stream) {
    if (!src || !sink) return (int)hipErrorInvalidValue;
    return (int)launch<1, false>(src, nullptr, nullptr, bytes, grid, unroll, sink, static_cast<hipStream_t>(stream));
}

int ceiling_write(void *dst, int64_t bytes, int grid, int unroll, void *stream) {
    if (!dst) return (int)hipErrorInvalidValue;
    return (int)launch<0, true>(nullptr, nullptr, dst, bytes, grid, unroll, nullptr, static_cast<hipStream_t>(stream));
}

int ceiling_copy(const void *src, void *dst, int64_t bytes, int grid, int unroll, void *stream) {
    if (!src || !dst) return (int)hipErrorInvalidValue;
    return (int)launch<1, true>(src, nullptr, dst, bytes, grid, unroll, nullptr, static_cast<hipStream_t>(stream));
}

int ceiling_mix2(const void *src0, const void *src1, void *dst, int64_t bytes, int grid, int unroll, void *stream) {
    if (!src0 || !src1 || !dst) return (int)hipErrorInvalidValue;
    return (int)launch<2, true>(src0, src1, dst, bytes, grid, unroll, nullptr, static_cast<hipStream_t>(stream));
}

}  // extern "C"
