// Packed A: the PACKA step of Algorithm 1 (alpha folded into A) for a big
// operand that is reused across calls, and the split-bf16 kernels that
// read it.
//   binary64 / binary32, native products: alpha*A rounded to the input
//     type (the product taken in binary64), dense row-major with k columns;
//     the plan's own kernel reads it with alpha = 1.
//   split-bf16 modes: RN32(alpha*A) split ahead of time into its bfloat16
//     terms (hi, mid[, lo]; the same residual split as the kernels apply to
//     a fresh binary32 A), plane p at p * presplit_rows(m) * presplit_ld(k),
//     rows of presplit_ld(k) values, zero padding.  The split-bf16 kernel
//     then loads the terms (16-byte vectors of each plane) instead of
//     splitting binary32 values on every call.
#include "k_bf16.h"

namespace tsmm {

// alpha*A rounded to T.  VEC (rows of A and out 16-byte aligned, k a
// multiple of the vector width): one 16-byte vector per thread and step,
// consecutive threads on consecutive vectors of a row, so that every load
// and store instruction covers whole lines; otherwise one thread per 8
// consecutive columns, element by element.
template <typename T, bool VEC>
__global__ void k_pack_a_scale(const T *__restrict__ A, int64_t lda, T *__restrict__ out, int64_t m, int64_t k,
                               double alpha) {
    if constexpr (VEC) {
        constexpr int VW = 16 / (int)sizeof(T);
        typedef T vec_t __attribute__((ext_vector_type(VW)));
        const int64_t gv = k / VW;
        const int64_t total = m * gv;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
             i += (int64_t)gridDim.x * blockDim.x) {
            const int64_t r = i / gv, c0 = (i - r * gv) * VW;
            const vec_t x = *reinterpret_cast<const vec_t *>(A + r * lda + c0);
            vec_t y;
#pragma unroll
            for (int e = 0; e < VW; ++e) y[e] = (T)(alpha * (double)x[e]);
            *reinterpret_cast<vec_t *>(out + r * k + c0) = y;
        }
    } else {
        const int64_t g8 = (k + 7) / 8;
        const int64_t total = m * g8;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
             i += (int64_t)gridDim.x * blockDim.x) {
            const int64_t r = i / g8, c0 = (i - r * g8) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (c0 + e < k) out[r * k + c0 + e] = (T)(alpha * (double)A[r * lda + c0 + e]);
        }
    }
}

template <typename T>
hipError_t launch_pack_a_scale(const void *A, int64_t lda, void *out, int64_t m, int64_t k, double alpha,
                               hipStream_t s) {
    constexpr int VW = 16 / (int)sizeof(T);
    const bool vec = k % VW == 0 && lda % VW == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(out) % 16 == 0;
    const int64_t work = vec ? m * (k / VW) : m * ((k + 7) / 8);
    const int block = 256;
    const unsigned grid = (unsigned)std::min<int64_t>((work + block - 1) / block, 65536);
    if (vec)
        hipLaunchKernelGGL((k_pack_a_scale<T, true>), dim3(grid), dim3(block), 0, s, static_cast<const T *>(A), lda,
                           static_cast<T *>(out), m, k, alpha);
    else
        hipLaunchKernelGGL((k_pack_a_scale<T, false>), dim3(grid), dim3(block), 0, s, static_cast<const T *>(A), lda,
                           static_cast<T *>(out), m, k, alpha);
    return hipGetLastError();
}

template <int TERMS>
__global__ void k_pack_a_split(const float *__restrict__ A, int64_t lda, uint16_t *__restrict__ planes, int64_t m,
                               int64_t k, double alpha) {
    const int64_t ld = presplit_ld(k), g8 = ld / 8;
    const int64_t pstride = presplit_rows(m) * ld;
    const int64_t total = presplit_rows(m) * g8;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / g8, c0 = (i - r * g8) * 8;
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            x[e] = (r < m && c0 + e < k) ? (float)(alpha * (double)A[r * lda + c0 + e]) : 0.0f;
        u16x8 t[TERMS];
        split8<TERMS>(x, t);
#pragma unroll
        for (int p = 0; p < TERMS; ++p) *reinterpret_cast<u16x8 *>(planes + p * pstride + r * ld + c0) = t[p];
    }
}

hipError_t launch_pack_a(tsmm_dtype dt, int terms, const void *A, int64_t lda, void *out, int64_t m, int64_t k,
                         double alpha, hipStream_t s) {
    const int64_t rows = terms > 0 ? presplit_rows(m) : m;
    const int64_t work = rows * ((k + 7) / 8);
    if (work == 0) return hipSuccess;
    const int block = 256;
    const unsigned grid = (unsigned)std::min<int64_t>((work + block - 1) / block, 65536);
    if (terms == 2)
        hipLaunchKernelGGL(k_pack_a_split<2>, dim3(grid), dim3(block), 0, s, static_cast<const float *>(A), lda,
                           static_cast<uint16_t *>(out), m, k, alpha);
    else if (terms == 3)
        hipLaunchKernelGGL(k_pack_a_split<3>, dim3(grid), dim3(block), 0, s, static_cast<const float *>(A), lda,
                           static_cast<uint16_t *>(out), m, k, alpha);
    else if (dt == TSMM_F64)
        return launch_pack_a_scale<double>(A, lda, out, m, k, alpha, s);
    else if (dt == TSMM_F32)
        return launch_pack_a_scale<float>(A, lda, out, m, k, alpha, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Split-bf16 kernels on a pre-split A (uint16_t planes, vector mapping):
// the variants whose registers hold the two sets of A terms, the
// accumulators and B without spilling (checked in the build's register
// report); the planner halves RT or splits the columns to reach one.
#define TSMM_BP(KC, NT, RT, P) {KC, NT, RT, P, 1, 0, &tsmm::run_splitbf16<uint16_t, KC, NT, RT, P, true, false>}, \
    TSMM_BPI(KC, NT, RT, P)
// interleaved columns where a group of 4 column tiles exists
#define TSMM_BPI(KC, NT, RT, P) TSMM_BPI_##NT(KC, RT, P)
#define TSMM_BPI_1(KC, RT, P)
#define TSMM_BPI_2(KC, RT, P)
#define TSMM_BPI_4(KC, RT, P) {KC, 4, RT, P, 1, 1, &tsmm::run_splitbf16<uint16_t, KC, 4, RT, P, true, true>},
#define TSMM_BPI_8(KC, RT, P) {KC, 8, RT, P, 1, 1, &tsmm::run_splitbf16<uint16_t, KC, 8, RT, P, true, true>},
#define TSMM_BPI_16(KC, RT, P) {KC, 16, RT, P, 1, 1, &tsmm::run_splitbf16<uint16_t, KC, 16, RT, P, true, true>},
#define TSMM_BP4(KC, RT, P) TSMM_BP(KC, 1, RT, P) TSMM_BP(KC, 2, RT, P) TSMM_BP(KC, 4, RT, P)
#define TSMM_BP8(KC, RT, P) TSMM_BP4(KC, RT, P) TSMM_BP(KC, 8, RT, P)
#define TSMM_BP16(KC, RT, P) TSMM_BP8(KC, RT, P) TSMM_BP(KC, 16, RT, P)
static const Bf16Entry kPre[] = {
    // two terms, three products
    TSMM_BP16(32, 1, 3) TSMM_BP16(64, 1, 3) TSMM_BP16(128, 1, 3) TSMM_BP8(256, 1, 3)
    TSMM_BP16(32, 2, 3) TSMM_BP8(64, 2, 3) TSMM_BP8(128, 2, 3) TSMM_BP4(256, 2, 3)
    // three terms, six products
    TSMM_BP16(32, 1, 6) TSMM_BP16(64, 1, 6) TSMM_BP8(128, 1, 6) TSMM_BP8(256, 1, 6)
    TSMM_BP8(32, 2, 6) TSMM_BP8(64, 2, 6) TSMM_BP8(128, 2, 6) TSMM_BP(256, 1, 2, 6) TSMM_BP(256, 2, 2, 6)
};

static Bf16Fn find_presplit(int products, int KC, int NT, int RT, bool il) {
    for (const Bf16Entry &e : kPre)
        if (e.KC == KC && e.NT == NT && e.RT == RT && e.prod == products && e.il == (int)il) return e.fn;
    return nullptr;
}

bool splitbf16_presplit_exists(int products, int KC, int NT, int RT, bool il) {
    return find_presplit(products, KC, NT, RT, il) != nullptr;
}

hipError_t launch_splitbf16_presplit(int products, int KC, int NT, int RT, bool il, const void *planes,
                                     const void *Bfrag, const int32_t *exps, void *C, int64_t m, int64_t n, int64_t k,
                                     double beta, int64_t grid, int block, int nt_total, int nsplit, hipStream_t s) {
    Bf16Fn fn = find_presplit(products, KC, NT, RT, il);
    if (!fn || nsplit < 1 || NT * nsplit != nt_total) return hipErrorInvalidValue;
    return fn(planes, Bfrag, exps, C, m, n, k, 1.0, beta, grid, block, nt_total, nsplit, s);
}

}  // namespace tsmm
