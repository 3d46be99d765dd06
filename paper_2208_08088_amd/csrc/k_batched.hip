// Batched op N: many independent tall-and-skinny multiplies, each with its
// own packed B, in ONE persistent launch.
//
// The host cuts every instance into work tiles of kBatchRows rows, orders
// the instances longest first and gives each workgroup one contiguous,
// cost-balanced range of the work-tile sequence (a static schedule: no
// counters or queues, so a launch is deterministic and needs no reset,
// which also makes it safe to capture in a graph and replay).  The
// workgroup walks its range as one segment per instance it meets: it copies
// that instance's packed B into LDS (the per-core resident block of B of the
// paper's Sec. IV-A.2), then its wavefronts stream the segment's rows with
// the software-pipelined row steps of the single-instance kernels,
// specialised for the instance's (k class, n class, mapping): binary32
// inputs use the 16x16x4 f32 product and fragments of k_stream.h, bfloat16
// inputs the 16x16x32 bf16 product and fragments of k_bf16.h.
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
template <int KC, int NT, bool VEC>
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
    stream_load_a<float, KC, RT, VEC>(A, row_b, k, kfull, t, voff0, q, a0);
    for (; t < tend; t += 2 * tstride) {
        stream_step<float, KC, NT, RT, VEC, CPRE>(A, sB, NT, C, row_b, n, k, kfull, d.alpha, d.beta, 0, t,
                                                  t + tstride, voff0, q, lane, j, a0, a1);
        stream_step<float, KC, NT, RT, VEC, CPRE>(A, sB, NT, C, row_b, n, k, kfull, d.alpha, d.beta, 0,
                                                  t + tstride, t + 2 * tstride, voff0, q, lane, j, a1, a0);
    }
}

// The same for a bfloat16 instance (k_bf16.h row steps, one product).
template <int KC, int NT, bool VEC>
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
    RawA<false, RT, KC / 32> x0, x1;
    bf16_load_step<uint16_t, KC, RT, 1, VEC>(A, row_b, k, t, j, q, x0);
    for (; t < tend; t += 2 * tstride) {
        bf16_step<uint16_t, KC, NT, RT, 1, VEC, CPRE>(A, sB, NT, nullptr, C, row_b, n, k, d.alpha, d.beta, 0, t,
                                                      t + tstride, j, q, lane, x0, x1);
        bf16_step<uint16_t, KC, NT, RT, 1, VEC, CPRE>(A, sB, NT, nullptr, C, row_b, n, k, d.alpha, d.beta, 0,
                                                      t + tstride, t + 2 * tstride, j, q, lane, x1, x0);
    }
}

#define TSMM_CASE_NT(BODY, KC, V)                                       \
    switch (d.NT) {                                                     \
    case 1: BODY<KC, 1, V>(d, row_a, row_b, sB, wave); break;           \
    case 2: BODY<KC, 2, V>(d, row_a, row_b, sB, wave); break;           \
    case 4: BODY<KC, 4, V>(d, row_a, row_b, sB, wave); break;           \
    default: BODY<KC, 8, V>(d, row_a, row_b, sB, wave); break;          \
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

// The workgroup walks its range of work tiles as segments, one per
// instance it meets: B of the instance into LDS, then the rows of the
// segment with a software-pipelined row loop specialised for the instance.
template <bool BF16>
__global__ __launch_bounds__(64 * kBatchWaves) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_batched(const BatchDesc *__restrict__ desc,
                                                              const int64_t *__restrict__ inst_start,
                                                              const int64_t *__restrict__ wg_begin,
                                                              const int32_t *__restrict__ wg_inst) {
    extern __shared__ u16x8 sB[];  // the current instance's packed B
    const int64_t begin = wg_begin[blockIdx.x], end = wg_begin[blockIdx.x + 1];
    int inst = wg_inst[blockIdx.x];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t g = begin; g < end;) {
        while (g >= inst_start[inst + 1]) ++inst;  // the sequence is sorted: inst only grows
        const int64_t g_end = end < inst_start[inst + 1] ? end : inst_start[inst + 1];
        const BatchDesc d = desc[inst];
        __syncthreads();  // every wavefront is done with the previous B
        const int vecs = BF16 ? (d.KC / 32) * d.NT * 64 : (d.KC / 4) * d.NT * 64 / 4;
        const u16x8 *src = static_cast<const u16x8 *>(d.Bfrag);
        for (int i = threadIdx.x; i < vecs; i += blockDim.x) sB[i] = src[i];
        __syncthreads();
        const int64_t row_a = (g - inst_start[inst]) * kBatchRows;
        int64_t row_b = (g_end - inst_start[inst]) * kBatchRows;
        row_b = row_b < d.m ? row_b : d.m;
        if constexpr (BF16) run_segment_bf16(d, row_a, row_b, sB, wave);
        else run_segment_f32(d, row_a, row_b, reinterpret_cast<const float *>(sB), wave);
        g = g_end;
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
