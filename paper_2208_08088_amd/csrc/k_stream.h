// op N streaming kernel: C = alpha*A*B + beta*C for a tall row-major A
// (m x k) and a small packed B (k x n), binary64 or binary32.
//
// This is the COMPUTE step of Algorithm 1 re-designed for gfx950.  The
// paper's blocking (Sec. IV-A, Fig. 2: TSMM -> GEPB -> GEPB_t -> GEBB_t,
// with n left untiled when it is small, and every core keeping the whole
// block of B in its private cache) maps onto the GPU as
//   - B, packed once in matrix-core fragment order, is copied into LDS by
//     every workgroup (the per-core L1-resident block of B, Eq. (2) with
//     LDS as the capacity); when it is larger than the LDS budget the
//     fragments are read through the L2 instead;
//   - a wavefront owns RT tiles of 16 rows (the m_t rows of a GEBB_t) and
//     walks the row tiles of A with a grid stride, so there is no
//     synchronisation at all after the B copy (Sec. IV-A.2);
//   - each lane loads 16-byte vectors of its row (k-slot mapping in
//     tsmm_internal.h), the 16x16x4 matrix-core product accumulates all n
//     columns, and the binary64 epilogue applies alpha and beta.
#pragma once

#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

constexpr int kStreamBlock = 256;
constexpr int kStreamLdsBudget = 128 * 1024;

template <typename T, int KC, int NT, int RT, bool VEC>
__global__ __launch_bounds__(kStreamBlock) void k_stream(const T *__restrict__ A,
                                                          const T *__restrict__ Bf,
                                                          T *__restrict__ C, int64_t m, int n,
                                                          int k, double alpha, double beta) {
    typedef Mfma4<T> M;
    typedef typename M::acc acc_t;
    typedef typename M::vec vec_t;
    constexpr int VW = M::VW;
    constexpr int S = KC / 4;  // k-steps
    constexpr int FRAG = S * NT * 64;
    constexpr bool BLDS = FRAG * (int)sizeof(T) <= kStreamLdsBudget;
    static_assert(!VEC || (KC % (4 * VW)) == 0, "vector mapping needs KC % (4*VW) == 0");

    __shared__ T sB[BLDS ? FRAG : 1];
    if constexpr (BLDS) {
        for (int idx = threadIdx.x * VW; idx < FRAG; idx += blockDim.x * VW)
            *reinterpret_cast<vec_t *>(&sB[idx]) = *reinterpret_cast<const vec_t *>(&Bf[idx]);
        __syncthreads();
    }
    const T *__restrict__ Bsrc = BLDS ? sB : Bf;

    const int lane = threadIdx.x & 63;
    const int j = lane & 15;
    const int q = lane >> 4;
    const int64_t ntile = (m + 15) >> 4;
    const int wpb = blockDim.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
    const int64_t tstride = (int64_t)gridDim.x * wpb * RT;

    for (int64_t t0 = gw * RT; t0 < ntile; t0 += tstride) {
        T a[RT][S];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t row = (t0 + rt) * 16 + j;
            const bool rok = row < m;
            const T *arow = A + row * (int64_t)k;
            if constexpr (VEC) {
#pragma unroll
                for (int p = 0; p < S / VW; ++p) {
                    const int col = p * 4 * VW + q * VW;
                    vec_t v = {};
                    if (rok && col < k) v = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(arow + col));
#pragma unroll
                    for (int e = 0; e < VW; ++e) a[rt][p * VW + e] = v[e];
                }
            } else {
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const int col = 4 * s + q;
                    a[rt][s] = (rok && col < k) ? arow[col] : T(0);
                }
            }
        }

        // B fragments small enough for registers may be hoisted out of the
        // row loop by the compiler; larger ones are re-read from LDS (or L2)
        // for every row tile, which the opaque offset enforces.
        int bofs = 0;
        if constexpr (S * NT > 32) asm volatile("" : "+v"(bofs));

        acc_t acc[RT][NT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[rt][t] = acc_t{};

#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const T b = Bsrc[bofs + (s * NT + t) * 64 + lane];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt][t] = M::op(a[rt][s], b, acc[rt][t]);
            }
        }

        // epilogue, one column tile at a time: lane (q, j) holds rows
        // M::row(q, r) of column 16t + j
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int col = 16 * t + j;
            T cv[RT][4];
            if (beta != 0.0) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = (t0 + rt) * 16 + M::row(q, r);
                        cv[rt][r] = (row < m && col < n) ? C[row * n + col] : T(0);
                    }
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = (t0 + rt) * 16 + M::row(q, r);
                    if (row < m && col < n) {
                        const double c = beta != 0.0 ? (double)cv[rt][r] : 0.0;
                        C[row * n + col] = (T)epilogue(alpha, (double)acc[rt][t][r], beta, c);
                    }
                }
        }
    }
}

template <typename T, int KC, int NT, int RT, bool VEC>
hipError_t run_stream(const void *A, const void *Bf, void *C, int64_t m, int64_t n, int64_t k,
                      double alpha, double beta, int64_t grid, int block, hipStream_t s) {
    hipLaunchKernelGGL((k_stream<T, KC, NT, RT, VEC>), dim3((unsigned)grid), dim3(block), 0, s,
                       static_cast<const T *>(A), static_cast<const T *>(Bf), static_cast<T *>(C),
                       m, (int)n, (int)k, alpha, beta);
    return hipGetLastError();
}

typedef hipError_t (*StreamFn)(const void *, const void *, void *, int64_t, int64_t, int64_t,
                               double, double, int64_t, int, hipStream_t);
struct StreamEntry {
    int KC, NT, RT, vec;
    StreamFn fn;
};

}  // namespace tsmm

// Instantiation lists: every NT for RT = 1, NT <= 8 for RT = 2, NT <= 4 for
// RT = 4 (accumulators stay within 128 registers).
#define TSMM_SE(T, KC, NT, RT, V) {KC, NT, RT, V, &tsmm::run_stream<T, KC, NT, RT, V>},
#define TSMM_SE_RT1(T, KC, V) \
    TSMM_SE(T, KC, 1, 1, V) TSMM_SE(T, KC, 2, 1, V) TSMM_SE(T, KC, 4, 1, V) TSMM_SE(T, KC, 8, 1, V) TSMM_SE(T, KC, 16, 1, V)
#define TSMM_SE_RT2(T, KC, V) \
    TSMM_SE(T, KC, 1, 2, V) TSMM_SE(T, KC, 2, 2, V) TSMM_SE(T, KC, 4, 2, V) TSMM_SE(T, KC, 8, 2, V)
#define TSMM_SE_RT4(T, KC, V) TSMM_SE(T, KC, 1, 4, V) TSMM_SE(T, KC, 2, 4, V) TSMM_SE(T, KC, 4, 4, V)
#define TSMM_SE_ALL(T, KC, V) TSMM_SE_RT1(T, KC, V) TSMM_SE_RT2(T, KC, V) TSMM_SE_RT4(T, KC, V)
