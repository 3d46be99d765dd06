// Batched op N: many independent tall-and-skinny multiplies, each with its
// own packed B, in ONE persistent launch.
//
// The host cuts every instance into chunks of chunk_rows rows and orders
// the instances by kernel variant; workgroups take chunks from a counter
// (dynamic schedule, see k_batched).  Binary32 inputs use the 16x16x4 f32
// product and fragments of k_stream.h, bfloat16 inputs the 16x16x32 bf16
// product and fragments of k_bf16.h.
#include "k_bf16.h"
#include "k_common.h"
#include "k_stream.h"
#include "tsmm_internal.h"

namespace tsmm {

// Row tiles per wavefront step of a variant: as many as keep the
// accumulators, the C prefetch and the two A register sets of the software
// pipeline within about 100 registers, up to 8.  Variants that do not
// fit even with one row tile (k or n of 64 and more, which are closer to
// the matrix-core bound) drop the C prefetch.
constexpr int batch_rt(int regs_per_rt) {
    return regs_per_rt * 8 <= 100 ? 8 : (regs_per_rt * 4 <= 100 ? 4 : (regs_per_rt * 2 <= 100 ? 2 : 1));
}
template <int KC, int NT> constexpr int batch_regs_f32() { return 2 * (KC / 4) + 8 * NT; }
template <int KC, int NT> constexpr int batch_regs_bf16() { return 8 * (KC / 32) + 8 * NT; }
template <int KC, int NT> constexpr int batch_rt_f32() { return batch_rt(batch_regs_f32<KC, NT>()); }
template <int KC, int NT> constexpr int batch_rt_bf16() { return batch_rt(batch_regs_bf16<KC, NT>()); }

// Rows [row_a, row_b) of a binary32 instance: the streaming kernel's
// pipelined row steps (k_stream.h) over this segment, with the segment end
// as the row limit (rows past it read 0 and are not written).
template <int KC, int NT, bool VEC, bool IL>
__device__ __forceinline__ void segment_f32(const BatchDesc &d, int64_t row_a, int64_t row_b,
                                            const float *__restrict__ sB, int wave) {
    constexpr int RT = batch_rt_f32<KC, NT>();
    constexpr bool CPRE = batch_regs_f32<KC, NT>() * RT <= 100;
    constexpr int S = KC / 4;
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const float *__restrict__ A = static_cast<const float *>(d.A);
    float *__restrict__ C = static_cast<float *>(d.C);
    const int k = d.k, n = d.n;
    const bool kfull = k == KC;
    const int voff0 = j * k * 4;
    const int64_t tend = (row_b + 15) >> 4;
    const int64_t tstride = (int64_t)kBatchWaves * RT;
    int64_t t = (row_a >> 4) + (int64_t)wave * RT;
    if (t >= tend) return;
    float a0[RT][S], a1[RT][S];
    stream_load_a<float, KC, RT, VEC>(A, row_b, k, k, kfull, t, voff0, q, a0);
    for (; t < tend; t += 2 * tstride) {
        stream_step<float, KC, NT, RT, VEC, IL, CPRE>(A, sB, NT, C, row_b, n, k, k, n, kfull, d.alpha, d.beta, 0, t,
                                                      t + tstride, voff0, q, lane, j, a0, a1);
        stream_step<float, KC, NT, RT, VEC, IL, CPRE>(A, sB, NT, C, row_b, n, k, k, n, kfull, d.alpha, d.beta, 0,
                                                      t + tstride, t + 2 * tstride, voff0, q, lane, j, a1, a0);
    }
}

// The same for a bfloat16 instance (k_bf16.h row steps, one product).
template <int KC, int NT, bool VEC, bool IL>
__device__ __forceinline__ void segment_bf16(const BatchDesc &d, int64_t row_a, int64_t row_b,
                                             const u16x8 *__restrict__ sB, int wave) {
    constexpr int RT = batch_rt_bf16<KC, NT>();
    constexpr bool CPRE = batch_regs_bf16<KC, NT>() * RT <= 100;
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const uint16_t *__restrict__ A = static_cast<const uint16_t *>(d.A);
    float *__restrict__ C = static_cast<float *>(d.C);
    const int k = d.k, n = d.n;
    const int64_t tend = (row_b + 15) >> 4;
    const int64_t tstride = (int64_t)kBatchWaves * RT;
    int64_t t = (row_a >> 4) + (int64_t)wave * RT;
    if (t >= tend) return;
    RawA<0, RT, KC / 32> x0, x1;
    bf16_load_step<uint16_t, KC, RT, 1, VEC>(A, row_b, k, t, j, q, x0);
    for (; t < tend; t += 2 * tstride) {
        bf16_step<uint16_t, KC, NT, RT, 1, VEC, IL, CPRE>(A, sB, NT, nullptr, C, row_b, n, k, d.alpha, d.beta, 0,
                                                          t, t + tstride, j, q, lane, x0, x1);
        bf16_step<uint16_t, KC, NT, RT, 1, VEC, IL, CPRE>(A, sB, NT, nullptr, C, row_b, n, k, d.alpha, d.beta, 0,
                                                          t + tstride, t + 2 * tstride, j, q, lane, x1, x0);
    }
}

// n % 4 == 0 and at least 4 column tiles: interleaved column order
// (16-byte C vectors)
#define TSMM_CASE_NT(BODY, KC, V)                                                                  \
    switch (d.NT) {                                                                                \
    case 1: BODY<KC, 1, V, false>(d, row_a, row_b, sB, wave); break;                               \
    case 2: BODY<KC, 2, V, false>(d, row_a, row_b, sB, wave); break;                               \
    case 4:                                                                                        \
        if (d.il) BODY<KC, 4, V, true>(d, row_a, row_b, sB, wave);                                 \
        else BODY<KC, 4, V, false>(d, row_a, row_b, sB, wave);                                     \
        break;                                                                                     \
    default:                                                                                       \
        if (d.il) BODY<KC, 8, V, true>(d, row_a, row_b, sB, wave);                                 \
        else BODY<KC, 8, V, false>(d, row_a, row_b, sB, wave);                                     \
        break;                                                                                     \
    }

__device__ __forceinline__ void run_segment_f32(const BatchDesc &d, int64_t row_a, int64_t row_b, const float *sB,
                                                int wave) {
    if (d.vec) {
        switch (d.KC) {
        case 16: TSMM_CASE_NT(segment_f32, 16, true) break;
        case 32: TSMM_CASE_NT(segment_f32, 32, true) break;
        case 64: TSMM_CASE_NT(segment_f32, 64, true) break;
        default: TSMM_CASE_NT(segment_f32, 128, true) break;
        }
    } else {
        switch (d.KC) {
        case 4: TSMM_CASE_NT(segment_f32, 4, false) break;
        case 8: TSMM_CASE_NT(segment_f32, 8, false) break;
        case 16: TSMM_CASE_NT(segment_f32, 16, false) break;
        case 32: TSMM_CASE_NT(segment_f32, 32, false) break;
        case 64: TSMM_CASE_NT(segment_f32, 64, false) break;
        default: TSMM_CASE_NT(segment_f32, 128, false) break;
        }
    }
}

__device__ __forceinline__ void run_segment_bf16(const BatchDesc &d, int64_t row_a, int64_t row_b, const u16x8 *sB,
                                                 int wave) {
    if (d.vec) {
        switch (d.KC) {
        case 32: TSMM_CASE_NT(segment_bf16, 32, true) break;
        case 64: TSMM_CASE_NT(segment_bf16, 64, true) break;
        default: TSMM_CASE_NT(segment_bf16, 128, true) break;
        }
    } else {
        switch (d.KC) {
        case 32: TSMM_CASE_NT(segment_bf16, 32, false) break;
        case 64: TSMM_CASE_NT(segment_bf16, 64, false) break;
        default: TSMM_CASE_NT(segment_bf16, 128, false) break;
        }
    }
}

// Dynamic schedule: the work is a sequence of chunks (d.chunk_rows rows of
// one instance, about the same bytes for every instance; instances of one
// kernel variant next to each other).  A
// workgroup takes the next chunk from a counter, loads that instance's
// packed B into LDS when the instance changes (the per-core resident block
// of B of the paper's Sec. IV-A.2), and streams the chunk's rows with the
// software-pipelined row steps of the single-instance kernels, specialised
// for the instance.  Each chunk is computed by exactly one workgroup with
// the same code, so results do not depend on the schedule.  The last
// workgroup to finish puts both counters back to zero, so every launch
// (and every graph replay) starts from a clean state without a memset.
template <bool BF16>
__global__ __launch_bounds__(64 * kBatchWaves) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_batched(
    const BatchDesc *__restrict__ desc, const int64_t *__restrict__ chunk_start, int64_t nchunks,
    int32_t *__restrict__ ctr) {
    extern __shared__ u16x8 sB[];  // the current instance's packed B
    __shared__ int32_t s_chunk;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int inst = 0, loaded = -1;
    for (;;) {
        if (threadIdx.x == 0) s_chunk = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();  // (also: every wavefront is done with the previous chunk and its B)
        const int64_t c = s_chunk;
        if (c >= nchunks) break;
        while (c >= chunk_start[inst + 1]) ++inst;  // a workgroup's chunks only grow
        const BatchDesc d = desc[inst];
        if (inst != loaded) {
            const int vecs = BF16 ? (d.KC / 32) * d.NT * 64 : (d.KC / 4) * d.NT * 64 / 4;
            const u16x8 *src = static_cast<const u16x8 *>(d.Bfrag);
            for (int i = threadIdx.x; i < vecs; i += blockDim.x) sB[i] = src[i];
            loaded = inst;
        }
        __syncthreads();  // B in LDS; every lane has read s_chunk
        const int64_t row_a = (c - chunk_start[inst]) * d.chunk_rows;
        const int64_t row_b = row_a + d.chunk_rows < d.m ? row_a + d.chunk_rows : d.m;
        if constexpr (BF16) run_segment_bf16(d, row_a, row_b, sB, wave);
        else run_segment_f32(d, row_a, row_b, reinterpret_cast<const float *>(sB), wave);
    }
    // the last workgroup out resets the counters for the next launch
    if (threadIdx.x == 0 &&
        __hip_atomic_fetch_add(ctr + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (int32_t)gridDim.x - 1) {
        __hip_atomic_store(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(ctr + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

size_t batched_lds_bytes(tsmm_dtype dt, int KC, int NT) {
    return dt == TSMM_BF16 ? (size_t)(KC / 32) * NT * 64 * 16 : (size_t)(KC / 4) * NT * 64 * 4;
}

hipError_t prepare_batched(tsmm_dtype dt, size_t lds_bytes) {
    const void *fn = dt == TSMM_BF16 ? (const void *)k_batched<true> : (const void *)k_batched<false>;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_batched(tsmm_dtype dt, const BatchDesc *desc, const int64_t *chunk_start, int64_t nchunks,
                          int chunk_rows, int32_t *ctr, int64_t grid, int block, size_t lds_bytes,
                          hipStream_t s) {
    if (block != 64 * kBatchWaves || nchunks < 0 || nchunks >= (int64_t)1 << 31 || chunk_rows < kBatchChunkMin ||
        chunk_rows > kBatchChunkMax || chunk_rows % 16 != 0)
        return hipErrorInvalidValue;
    if (dt == TSMM_BF16)
        hipLaunchKernelGGL(k_batched<true>, dim3((unsigned)grid), dim3(block), lds_bytes, s, desc, chunk_start,
                           nchunks, ctr);
    else
        hipLaunchKernelGGL(k_batched<false>, dim3((unsigned)grid), dim3(block), lds_bytes, s, desc, chunk_start,
                           nchunks, ctr);
    return hipGetLastError();
}

}  // namespace tsmm
