// Batched op N: many independent tall-and-skinny multiplies, each with its
// own packed B, in ONE persistent launch.
//
// The host cuts every instance into work tiles of kBatchRows rows, orders
// the instances longest first and gives each workgroup one contiguous,
// cost-balanced range of the work-tile sequence (a static schedule: no
// counters or queues, so a launch is deterministic and needs no reset,
// which also makes it safe to capture in a graph and replay).  A wavefront
// takes every W-th tile of its workgroup's range, dispatches on the
// instance's (k class, n class, mapping) to a matrix-core body specialised
// for it and streams the tile's rows: binary32 inputs use the 16x16x4 f32
// product with the B fragments of k_stream.h, bfloat16 inputs the 16x16x32
// bf16 product with the fragments of k_bf16.h.  B fragments are read
// through the cache hierarchy (each instance's B is at most 64 KiB).
#include "k_bf16.h"
#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

// One 16-row tile of a binary32 instance (16x16x4 f32 products).
template <int KC, int NT, bool VEC>
__device__ __forceinline__ void tile_f32(const BatchDesc &d, int64_t row0) {
    constexpr int S = KC / 4;
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const float *__restrict__ A = static_cast<const float *>(d.A);
    const float *__restrict__ Bf = static_cast<const float *>(d.Bfrag);
    float *__restrict__ C = static_cast<float *>(d.C);
    const int k = d.k, n = d.n;
    const int64_t m = d.m;
    float a[S];
    {
        const int64_t row = row0 + j;
        const bool rok = row < m;
        const float *arow = A + row * (int64_t)k;
        if constexpr (VEC) {
#pragma unroll
            for (int p = 0; p < S / 4; ++p) {
                const int col = p * 16 + q * 4;
                f4v v = {};
                if (rok && col < k) v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(arow + col));
#pragma unroll
                for (int e = 0; e < 4; ++e) a[p * 4 + e] = v[e];
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int col = 4 * s + q;
                a[s] = (rok && col < k) ? arow[col] : 0.0f;
            }
        }
    }
    f4v acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4v{};
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], Bf[(s * NT + t) * 64 + lane], acc[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = 16 * t + j;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + 4 * q + r;
            if (row < m && col < n) {
                float *pc = C + row * n + col;
                const double c = d.beta != 0.0 ? (double)*pc : 0.0;
                *pc = (float)epilogue(d.alpha, (double)acc[t][r], d.beta, c);
            }
        }
    }
}

// One 16-row tile of a bfloat16 instance (16x16x32 bf16 products).
template <int KC, int NT, bool VEC>
__device__ __forceinline__ void tile_bf16(const BatchDesc &d, int64_t row0) {
    constexpr int NCH = KC / 32;
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const uint16_t *__restrict__ A = static_cast<const uint16_t *>(d.A);
    const u16x8 *__restrict__ Bf = static_cast<const u16x8 *>(d.Bfrag);
    float *__restrict__ C = static_cast<float *>(d.C);
    const int k = d.k, n = d.n;
    const int64_t m = d.m;
    const int64_t row = row0 + j;
    const bool rok = row < m;
    f4v acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4v{};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const u16x8 av = load_a8_bf16<VEC>(A + row * (int64_t)k, 32 * c + 8 * q, k, rok);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma_bf16(av, Bf[(c * NT + t) * 64 + lane], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = 16 * t + j;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t orow = row0 + 4 * q + r;
            if (orow < m && col < n) {
                float *pc = C + orow * n + col;
                const double cc = d.beta != 0.0 ? (double)*pc : 0.0;
                *pc = (float)epilogue(d.alpha, (double)acc[t][r], d.beta, cc);
            }
        }
    }
}

#define TSMM_CASE_NT(BODY, KC, V)                          \
    switch (d.NT) {                                        \
    case 1: BODY<KC, 1, V>(d, r0); break;                  \
    case 2: BODY<KC, 2, V>(d, r0); break;                  \
    case 4: BODY<KC, 4, V>(d, r0); break;                  \
    default: BODY<KC, 8, V>(d, r0); break;                 \
    }

__device__ __forceinline__ void run_tile_f32(const BatchDesc &d, int64_t r0) {
    if (d.vec) {
        switch (d.KC) {
        case 16: TSMM_CASE_NT(tile_f32, 16, true) break;
        case 32: TSMM_CASE_NT(tile_f32, 32, true) break;
        case 64: TSMM_CASE_NT(tile_f32, 64, true) break;
        default: TSMM_CASE_NT(tile_f32, 128, true) break;
        }
    } else {
        switch (d.KC) {
        case 4: TSMM_CASE_NT(tile_f32, 4, false) break;
        case 8: TSMM_CASE_NT(tile_f32, 8, false) break;
        case 16: TSMM_CASE_NT(tile_f32, 16, false) break;
        case 32: TSMM_CASE_NT(tile_f32, 32, false) break;
        case 64: TSMM_CASE_NT(tile_f32, 64, false) break;
        default: TSMM_CASE_NT(tile_f32, 128, false) break;
        }
    }
}

__device__ __forceinline__ void run_tile_bf16(const BatchDesc &d, int64_t r0) {
    if (d.vec) {
        switch (d.KC) {
        case 32: TSMM_CASE_NT(tile_bf16, 32, true) break;
        case 64: TSMM_CASE_NT(tile_bf16, 64, true) break;
        default: TSMM_CASE_NT(tile_bf16, 128, true) break;
        }
    } else {
        switch (d.KC) {
        case 32: TSMM_CASE_NT(tile_bf16, 32, false) break;
        case 64: TSMM_CASE_NT(tile_bf16, 64, false) break;
        default: TSMM_CASE_NT(tile_bf16, 128, false) break;
        }
    }
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_batched(const BatchDesc *__restrict__ desc,
                                                 const int64_t *__restrict__ inst_start,
                                                 const int64_t *__restrict__ wg_begin,
                                                 const int32_t *__restrict__ wg_inst) {
    const int64_t begin = wg_begin[blockIdx.x], end = wg_begin[blockIdx.x + 1];
    int inst = wg_inst[blockIdx.x];
    const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    for (int64_t g = begin + wave; g < end; g += nwave) {
        while (g >= inst_start[inst + 1]) ++inst;  // the sequence is sorted: inst only grows
        const BatchDesc d = desc[inst];
        const int64_t base = (g - inst_start[inst]) * kBatchRows;
#pragma unroll 1
        for (int sub = 0; sub < kBatchRows / 16; ++sub) {
            const int64_t r0 = base + 16 * sub;
            if (r0 >= d.m) break;
            if constexpr (BF16) run_tile_bf16(d, r0);
            else run_tile_f32(d, r0);
        }
    }
}

hipError_t launch_batched(tsmm_dtype dt, const BatchDesc *desc, const int64_t *inst_start,
                          const int64_t *wg_begin, const int32_t *wg_inst, int64_t grid, int block,
                          hipStream_t s) {
    if (dt == TSMM_BF16)
        hipLaunchKernelGGL(k_batched<true>, dim3((unsigned)grid), dim3(block), 0, s, desc, inst_start, wg_begin,
                           wg_inst);
    else
        hipLaunchKernelGGL(k_batched<false>, dim3((unsigned)grid), dim3(block), 0, s, desc, inst_start, wg_begin,
                           wg_inst);
    return hipGetLastError();
}

}  // namespace tsmm
