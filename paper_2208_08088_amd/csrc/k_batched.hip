// Batched op N: many independent tall-and-skinny multiplies, each with its
// own packed B, in ONE persistent launch.
//
// The host cuts every instance into work tiles of kBatchRows rows, orders
// the instances longest first and gives each workgroup one contiguous,
// cost-balanced range of the work-tile sequence (a static schedule: no
// counters or queues, so a launch is deterministic and needs no reset,
// which also makes it safe to capture in a graph and replay).  The
// workgroup walks its range in order; whenever the instance changes it
// copies that instance's packed B into LDS (the per-core resident block of
// B of the paper's Sec. IV-A.2), then its wavefronts stream their rows of
// the tile with the matrix-core body specialised for the instance's
// (k class, n class, mapping): binary32 inputs use the 16x16x4 f32 product
// with the fragments of k_stream.h, bfloat16 inputs the 16x16x32 bf16
// product with the fragments of k_bf16.h.
#include "k_bf16.h"
#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

constexpr int kBatchWaves = 4;
constexpr int kBatchRT = kBatchRows / (16 * kBatchWaves);  // 16-row tiles per wavefront
static_assert(kBatchRT * 16 * kBatchWaves == kBatchRows, "work tile = waves x row tiles");

// Rows row0 .. row0 + 16*kBatchRT of a binary32 instance.
template <int KC, int NT, bool VEC>
__device__ __forceinline__ void tile_f32(const BatchDesc &d, int64_t row0, const float *__restrict__ sB) {
    constexpr int S = KC / 4;
    constexpr int RT = kBatchRT;
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const float *__restrict__ A = static_cast<const float *>(d.A);
    float *__restrict__ C = static_cast<float *>(d.C);
    const int k = d.k, n = d.n;
    const int64_t m = d.m;
    float a[RT][S];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t r0 = uniform64(row0 + 16 * rt);
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + r0 * k, (m - r0) * (int64_t)k * 4);
        if constexpr (VEC) {
#pragma unroll
            for (int p = 0; p < S / 4; ++p) {
                const int col = p * 16 + q * 4;
                f4v v = {};
                if (col < k) v = BufIO<float>::load_vec(ra, (j * k + col) * 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) a[rt][p * 4 + e] = v[e];
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int col = 4 * s + q;
                a[rt][s] = col < k ? BufIO<float>::load1(ra, (j * k + col) * 4) : 0.0f;
            }
        }
    }
    f4v acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = f4v{};
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float b = sB[(s * NT + t) * 64 + lane];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                acc[rt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][s], b, acc[rt][t], 0, 0, 0);
        }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t r0 = uniform64(row0 + 16 * rt);
        const __amdgpu_buffer_rsrc_t rc = make_rsrc(C + r0 * n, (m - r0) * (int64_t)n * 4);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int col = 16 * t + j;
            if (col >= n) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int off = ((4 * q + r) * n + col) * 4;
                const double c = d.beta != 0.0 ? (double)BufIO<float>::load1(rc, off) : 0.0;
                BufIO<float>::store1((float)epilogue(d.alpha, (double)acc[rt][t][r], d.beta, c), rc, off);
            }
        }
    }
}

// Rows row0 .. row0 + 16*kBatchRT of a bfloat16 instance.
template <int KC, int NT, bool VEC>
__device__ __forceinline__ void tile_bf16(const BatchDesc &d, int64_t row0, const u16x8 *__restrict__ sB) {
    constexpr int NCH = KC / 32;
    constexpr int RT = kBatchRT;
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const uint16_t *__restrict__ A = static_cast<const uint16_t *>(d.A);
    float *__restrict__ C = static_cast<float *>(d.C);
    const int k = d.k, n = d.n;
    const int64_t m = d.m;
    u16x8 a[RT][NCH];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t r0 = row0 + 16 * rt;
        const int64_t row = r0 + j;
#pragma unroll
        for (int c = 0; c < NCH; ++c) a[rt][c] = load_a8_bf16<VEC>(A + row * (int64_t)k, 32 * c + 8 * q, k, row < m);
    }
    f4v acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = f4v{};
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const u16x8 b = sB[(c * NT + t) * 64 + lane];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt][t] = mfma_bf16(a[rt][c], b, acc[rt][t]);
        }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t r0 = uniform64(row0 + 16 * rt);
        const __amdgpu_buffer_rsrc_t rc = make_rsrc(C + r0 * n, (m - r0) * (int64_t)n * 4);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int col = 16 * t + j;
            if (col >= n) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int off = ((4 * q + r) * n + col) * 4;
                const double cc = d.beta != 0.0 ? (double)BufIO<float>::load1(rc, off) : 0.0;
                BufIO<float>::store1((float)epilogue(d.alpha, (double)acc[rt][t][r], d.beta, cc), rc, off);
            }
        }
    }
}

#define TSMM_CASE_NT(BODY, KC, V, LDS)                     \
    switch (d.NT) {                                        \
    case 1: BODY<KC, 1, V>(d, r0, LDS); break;             \
    case 2: BODY<KC, 2, V>(d, r0, LDS); break;             \
    case 4: BODY<KC, 4, V>(d, r0, LDS); break;             \
    default: BODY<KC, 8, V>(d, r0, LDS); break;            \
    }

__device__ __forceinline__ void run_tile_f32(const BatchDesc &d, int64_t r0, const float *sB) {
    if (d.vec) {
        switch (d.KC) {
        case 16: TSMM_CASE_NT(tile_f32, 16, true, sB) break;
        case 32: TSMM_CASE_NT(tile_f32, 32, true, sB) break;
        case 64: TSMM_CASE_NT(tile_f32, 64, true, sB) break;
        default: TSMM_CASE_NT(tile_f32, 128, true, sB) break;
        }
    } else {
        switch (d.KC) {
        case 4: TSMM_CASE_NT(tile_f32, 4, false, sB) break;
        case 8: TSMM_CASE_NT(tile_f32, 8, false, sB) break;
        case 16: TSMM_CASE_NT(tile_f32, 16, false, sB) break;
        case 32: TSMM_CASE_NT(tile_f32, 32, false, sB) break;
        case 64: TSMM_CASE_NT(tile_f32, 64, false, sB) break;
        default: TSMM_CASE_NT(tile_f32, 128, false, sB) break;
        }
    }
}

__device__ __forceinline__ void run_tile_bf16(const BatchDesc &d, int64_t r0, const u16x8 *sB) {
    if (d.vec) {
        switch (d.KC) {
        case 32: TSMM_CASE_NT(tile_bf16, 32, true, sB) break;
        case 64: TSMM_CASE_NT(tile_bf16, 64, true, sB) break;
        default: TSMM_CASE_NT(tile_bf16, 128, true, sB) break;
        }
    } else {
        switch (d.KC) {
        case 32: TSMM_CASE_NT(tile_bf16, 32, false, sB) break;
        case 64: TSMM_CASE_NT(tile_bf16, 64, false, sB) break;
        default: TSMM_CASE_NT(tile_bf16, 128, false, sB) break;
        }
    }
}

template <bool BF16>
__global__ __launch_bounds__(64 * kBatchWaves) void k_batched(const BatchDesc *__restrict__ desc,
                                                              const int64_t *__restrict__ inst_start,
                                                              const int64_t *__restrict__ wg_begin,
                                                              const int32_t *__restrict__ wg_inst) {
    extern __shared__ u16x8 sB[];  // the current instance's packed B
    const int64_t begin = wg_begin[blockIdx.x], end = wg_begin[blockIdx.x + 1];
    int inst = wg_inst[blockIdx.x];
    int loaded = -1;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t g = begin; g < end; ++g) {
        while (g >= inst_start[inst + 1]) ++inst;  // the sequence is sorted: inst only grows
        const BatchDesc d = desc[inst];
        if (inst != loaded) {  // uniform across the workgroup: every wavefront walks the same tiles
            __syncthreads();
            const int vecs = BF16 ? (d.KC / 32) * d.NT * 64 : (d.KC / 4) * d.NT * 64 / 4;
            const u16x8 *src = static_cast<const u16x8 *>(d.Bfrag);
            for (int i = threadIdx.x; i < vecs; i += blockDim.x) sB[i] = src[i];
            __syncthreads();
            loaded = inst;
        }
        const int64_t r0 = (g - inst_start[inst]) * kBatchRows + (int64_t)wave * 16 * kBatchRT;
        if (r0 >= d.m) continue;
        if constexpr (BF16) run_tile_bf16(d, r0, sB);
        else run_tile_f32(d, r0, reinterpret_cast<const float *>(sB));
    }
}

size_t batched_lds_bytes(tsmm_dtype dt, int KC, int NT) {
    return dt == TSMM_BF16 ? (size_t)(KC / 32) * NT * 64 * 16 : (size_t)(KC / 4) * NT * 64 * 4;
}

hipError_t prepare_batched(tsmm_dtype dt, size_t lds_bytes) {
    const void *fn = dt == TSMM_BF16 ? (const void *)k_batched<true> : (const void *)k_batched<false>;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_batched(tsmm_dtype dt, const BatchDesc *desc, const int64_t *inst_start,
                          const int64_t *wg_begin, const int32_t *wg_inst, int64_t grid, int block,
                          size_t lds_bytes, hipStream_t s) {
    if (block != 64 * kBatchWaves) return hipErrorInvalidValue;
    if (dt == TSMM_BF16)
        hipLaunchKernelGGL(k_batched<true>, dim3((unsigned)grid), dim3(block), lds_bytes, s, desc, inst_start,
                           wg_begin, wg_inst);
    else
        hipLaunchKernelGGL(k_batched<false>, dim3((unsigned)grid), dim3(block), lds_bytes, s, desc, inst_start,
                           wg_begin, wg_inst);
    return hipGetLastError();
}

}  // namespace tsmm
