// op N with bfloat16 matrix-core products (V_MFMA_F32_16X16X32_BF16):
//   - split-bf16 modes for binary32 A and B: every binary32 element is
//     written as a sum of bfloat16 terms (hi, mid[, lo]); A is split in
//     registers as it streams in, B was split once at pack time (with a
//     power-of-two scale per column, undone in the epilogue); the products
//     of term order i + j <= 1 (3 products) or i + j <= 2 (6 products) are
//     accumulated in binary32, the leading hi*hi product in its own
//     accumulator and the correction products in a second one, and the two
//     are added in the binary64 epilogue;
//   - plain bfloat16 inputs (one term, one product), binary32 output.
// Row tiles are walked with a grid stride exactly as in the binary64 /
// binary32 streaming kernel (k_stream.h).
#pragma once

#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

constexpr int kBf16Block = 256;
constexpr int kBf16LdsBudget = 128 * 1024;

__device__ __forceinline__ f4v mfma_bf16(const u16x8 &a, const u16x8 &b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c,
                                                   0, 0, 0);
}

// Load the 8 A values of lane (row, q) for k-chunk c as binary32.
template <typename TA, bool VEC>
__device__ __forceinline__ void load_a8(const TA *__restrict__ arow, int col, int k, bool rok, float (&x)[8]);

template <>
__device__ __forceinline__ void load_a8<float, true>(const float *__restrict__ arow, int col, int k, bool rok,
                                                     float (&x)[8]) {
    f4v v0 = {}, v1 = {};
    if (rok && col < k) v0 = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(arow + col));
    if (rok && col + 4 < k) v1 = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(arow + col + 4));
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        x[e] = v0[e];
        x[4 + e] = v1[e];
    }
}
template <>
__device__ __forceinline__ void load_a8<float, false>(const float *__restrict__ arow, int col, int k, bool rok,
                                                      float (&x)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = (rok && col + e < k) ? arow[col + e] : 0.0f;
}

// bf16 inputs: the 8 raw values (no conversion needed for the product).
template <bool VEC>
__device__ __forceinline__ u16x8 load_a8_bf16(const uint16_t *__restrict__ arow, int col, int k, bool rok) {
    u16x8 v = {};
    if constexpr (VEC) {
        if (rok && col < k) v = __builtin_nontemporal_load(reinterpret_cast<const u16x8 *>(arow + col));
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (rok && col + e < k) ? arow[col + e] : (uint16_t)0;
    }
    return v;
}

// Residual split of 8 binary32 values into TERMS bfloat16 vectors.
template <int TERMS>
__device__ __forceinline__ void split8(const float (&x)[8], u16x8 (&t)[TERMS]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        float r = x[e];
#pragma unroll
        for (int p = 0; p < TERMS; ++p) {
            const uint16_t h = float_to_bf16_bits(r);
            t[p][e] = h;
            if (p + 1 < TERMS) r = r - bf16_bits_to_float(h);
        }
    }
}

// PROD: 1 (plain bf16), 3 (two terms) or 6 (three terms).
template <typename TA, int KC, int NT, int RT, int PROD, bool VEC>
__global__ __launch_bounds__(kBf16Block) void k_splitbf16(const TA *__restrict__ A,
                                                          const uint16_t *__restrict__ Bf,
                                                          const int32_t *__restrict__ exps,
                                                          float *__restrict__ C, int64_t m, int n, int k,
                                                          double alpha, double beta) {
    constexpr int TERMS = PROD == 1 ? 1 : (PROD == 3 ? 2 : 3);
    constexpr int NCH = KC / 32;
    constexpr int FRAG = NCH * NT * TERMS * 64 * 8;  // bf16 elements
    constexpr bool BLDS = FRAG * 2 <= kBf16LdsBudget;
    constexpr bool TWO_ACC = PROD > 1;

    __shared__ u16x8 sB[BLDS ? FRAG / 8 : 1];
    if constexpr (BLDS) {
        const u16x8 *src = reinterpret_cast<const u16x8 *>(Bf);
        for (int idx = threadIdx.x; idx < FRAG / 8; idx += blockDim.x) sB[idx] = src[idx];
        __syncthreads();
    }
    const u16x8 *__restrict__ Bsrc = BLDS ? sB : reinterpret_cast<const u16x8 *>(Bf);

    const int lane = threadIdx.x & 63;
    const int j = lane & 15;
    const int q = lane >> 4;
    const int64_t ntile = (m + 15) >> 4;
    const int wpb = blockDim.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
    const int64_t tstride = (int64_t)gridDim.x * wpb * RT;

    for (int64_t t0 = gw * RT; t0 < ntile; t0 += tstride) {
        f4v acc[RT][NT];
        f4v acc2[TWO_ACC ? RT : 1][TWO_ACC ? NT : 1];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                acc[rt][t] = f4v{};
                if constexpr (TWO_ACC) acc2[rt][t] = f4v{};
            }

        int bofs = 0;
        asm volatile("" : "+v"(bofs));  // B is re-read per row tile, not hoisted

#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            u16x8 at[RT][TERMS];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int64_t row = (t0 + rt) * 16 + j;
                const bool rok = row < m;
                const int col = 32 * c + 8 * q;
                if constexpr (PROD == 1) {
                    at[rt][0] = load_a8_bf16<VEC>(reinterpret_cast<const uint16_t *>(A) + row * (int64_t)k, col, k, rok);
                } else {
                    float x[8];
                    load_a8<float, VEC>(reinterpret_cast<const float *>(A) + row * (int64_t)k, col, k, rok, x);
                    split8<TERMS>(x, at[rt]);
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                u16x8 bt[TERMS];
#pragma unroll
                for (int p = 0; p < TERMS; ++p) bt[p] = Bsrc[bofs + ((c * NT + t) * TERMS + p) * 64 + lane];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    acc[rt][t] = mfma_bf16(at[rt][0], bt[0], acc[rt][t]);
                    if constexpr (PROD >= 3) {
                        acc2[rt][t] = mfma_bf16(at[rt][0], bt[1], acc2[rt][t]);
                        acc2[rt][t] = mfma_bf16(at[rt][1], bt[0], acc2[rt][t]);
                    }
                    if constexpr (PROD == 6) {
                        acc2[rt][t] = mfma_bf16(at[rt][0], bt[2], acc2[rt][t]);
                        acc2[rt][t] = mfma_bf16(at[rt][1], bt[1], acc2[rt][t]);
                        acc2[rt][t] = mfma_bf16(at[rt][2], bt[0], acc2[rt][t]);
                    }
                }
            }
        }

#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int col = 16 * t + j;
            const int e = (PROD > 1 && col < n) ? exps[col] : 0;
            float cv[RT][4];
            if (beta != 0.0) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = (t0 + rt) * 16 + 4 * q + r;
                        cv[rt][r] = (row < m && col < n) ? C[row * n + col] : 0.0f;
                    }
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = (t0 + rt) * 16 + 4 * q + r;
                    if (row < m && col < n) {
                        double s = (double)acc[rt][t][r];
                        if constexpr (TWO_ACC) s = s + (double)acc2[rt][t][r];
                        if (PROD > 1) s = __builtin_ldexp(s, e);
                        const double c = beta != 0.0 ? (double)cv[rt][r] : 0.0;
                        C[row * n + col] = (float)epilogue(alpha, s, beta, c);
                    }
                }
        }
    }
}

template <typename TA, int KC, int NT, int RT, int PROD, bool VEC>
hipError_t run_splitbf16(const void *A, const void *Bf, const int32_t *exps, void *C, int64_t m, int64_t n,
                         int64_t k, double alpha, double beta, int64_t grid, int block, hipStream_t s) {
    hipLaunchKernelGGL((k_splitbf16<TA, KC, NT, RT, PROD, VEC>), dim3((unsigned)grid), dim3(block), 0, s,
                       static_cast<const TA *>(A), static_cast<const uint16_t *>(Bf), exps, static_cast<float *>(C),
                       m, (int)n, (int)k, alpha, beta);
    return hipGetLastError();
}

typedef hipError_t (*Bf16Fn)(const void *, const void *, const int32_t *, void *, int64_t, int64_t, int64_t,
                             double, double, int64_t, int, hipStream_t);
struct Bf16Entry {
    int KC, NT, RT, prod, vec;
    Bf16Fn fn;
};

}  // namespace tsmm

#define TSMM_BE(TA, KC, NT, RT, P, V) {KC, NT, RT, P, V, &tsmm::run_splitbf16<TA, KC, NT, RT, P, V>},
#define TSMM_BE_NT(TA, KC, RT, P, V) \
    TSMM_BE(TA, KC, 1, RT, P, V) TSMM_BE(TA, KC, 2, RT, P, V) TSMM_BE(TA, KC, 4, RT, P, V) TSMM_BE(TA, KC, 8, RT, P, V) \
    TSMM_BE(TA, KC, 16, RT, P, V)
#define TSMM_BE_KC(TA, RT, P, V) \
    TSMM_BE_NT(TA, 32, RT, P, V) TSMM_BE_NT(TA, 64, RT, P, V) TSMM_BE_NT(TA, 128, RT, P, V) TSMM_BE_NT(TA, 256, RT, P, V)
