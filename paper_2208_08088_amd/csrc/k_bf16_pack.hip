// Packing for the bfloat16 matrix-core kernels, and their dispatch.
//
// Split modes (PACKB of Algorithm 1 for binary32 B): every column j gets a
// power-of-two exponent e_j with 1 <= max_i |B[i][j]| * 2^-e_j < 2; the
// scaled values are split into `terms` bfloat16 residual terms (round to
// nearest even at every step) and stored both row-major (for inspection)
// and in the fragment order of V_MFMA_F32_16X16X32_BF16 (tsmm_internal.h).
// Plain bfloat16 B is only rearranged.
#include "k_bf16.h"

namespace tsmm {

Bf16Fn find_bf16_x1(int KC, int NT, int RT, bool vec, bool il);
Bf16Fn find_bf16_x3(int KC, int NT, int RT, bool vec, bool il);
Bf16Fn find_bf16_x6(int KC, int NT, int RT, bool vec, bool il);

__global__ void k_col_exps(const float *__restrict__ B, int32_t *__restrict__ exps, int64_t k, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float mx = 0.0f;
    bool finite = true;
    for (int64_t i = 0; i < k; ++i) {
        const float a = fabsf(B[i * n + j]);
        if (!isfinite(a)) finite = false;
        else mx = fmaxf(mx, a);
    }
    int e = 0;
    if (finite && mx != 0.0f) {
        int ex;
        (void)frexpf(mx, &ex);
        e = ex - 1;
    }
    exps[j] = e;
}

// One thread per element of B: split (or copy) and scatter into fragments.
template <bool SPLIT>
__global__ void k_pack_bf16(const void *__restrict__ Bv, const int32_t *__restrict__ exps,
                            uint16_t *__restrict__ frag, uint16_t *__restrict__ planes, int64_t k, int64_t n,
                            int NT, int terms, int pg) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= k * n) return;
    const int64_t i = idx / n, jn = idx % n;
    const int c = (int)(i / 32), kk = (int)(i % 32), q = kk / 8, u = kk % 8;
    // column jn sits in tile t, lane column jj (interleave group pg)
    const int t = (int)(pg * (jn / (16 * pg)) + jn % pg), jj = (int)((jn % (16 * pg)) / pg);
    const int lane = 16 * q + jj;
    if constexpr (SPLIT) {
        float r = ldexpf(static_cast<const float *>(Bv)[idx], -exps[jn]);
        for (int p = 0; p < terms; ++p) {
            const uint16_t h = float_to_bf16_bits(r);
            r = r - bf16_bits_to_float(h);
            planes[(int64_t)p * k * n + idx] = h;
            frag[((((int64_t)c * NT + t) * terms + p) * 64 + lane) * 8 + u] = h;
        }
    } else {
        frag[(((int64_t)c * NT + t) * 64 + lane) * 8 + u] = static_cast<const uint16_t *>(Bv)[idx];
    }
}

__global__ void k_unpack_split(const uint16_t *__restrict__ planes, const int32_t *__restrict__ exps,
                               float *__restrict__ out, int64_t k, int64_t n, int terms) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= k * n) return;
    float x = 0.0f;
    for (int p = terms - 1; p >= 0; --p) x = x + bf16_bits_to_float(planes[(int64_t)p * k * n + idx]);
    out[idx] = ldexpf(x, exps[idx % n]);
}

hipError_t launch_pack_bf16(tsmm_dtype dt, const void *B, void *frag, void *planes, int32_t *exps, int64_t k,
                            int64_t n, int KC, int NT, int terms, int pg, hipStream_t s) {
    const size_t frag_bytes = (size_t)KC * NT * 16 * terms * 2;
    hipError_t e = hipMemsetAsync(frag, 0, frag_bytes, s);  // zero padding
    if (e != hipSuccess) return e;
    const int64_t count = k * n;
    const unsigned blocks = (unsigned)((count + 255) / 256);
    if (dt == TSMM_F32) {
        hipLaunchKernelGGL(k_col_exps, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, static_cast<const float *>(B),
                           exps, k, n);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_pack_bf16<true>, dim3(blocks), dim3(256), 0, s, B, (const int32_t *)exps,
                           static_cast<uint16_t *>(frag), static_cast<uint16_t *>(planes), k, n, NT, terms, pg);
    } else {
        hipLaunchKernelGGL(k_pack_bf16<false>, dim3(blocks), dim3(256), 0, s, B, (const int32_t *)nullptr,
                           static_cast<uint16_t *>(frag), (uint16_t *)nullptr, k, n, NT, 1, pg);
    }
    return hipGetLastError();
}

hipError_t launch_unpack_split(const void *planes, const int32_t *exps, void *B_out, int64_t k, int64_t n,
                               int terms, hipStream_t s) {
    const int64_t count = k * n;
    hipLaunchKernelGGL(k_unpack_split, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       static_cast<const uint16_t *>(planes), exps, static_cast<float *>(B_out), k, n, terms);
    return hipGetLastError();
}

static Bf16Fn find_bf16(tsmm_dtype dt, int KC, int NT, int RT, int products, bool vec, bool il) {
    if (dt == TSMM_BF16 && products == 1) return find_bf16_x1(KC, NT, RT, vec, il);
    if (dt == TSMM_F32 && products == 3) return find_bf16_x3(KC, NT, RT, vec, il);
    if (dt == TSMM_F32 && products == 6) return find_bf16_x6(KC, NT, RT, vec, il);
    return nullptr;
}

bool splitbf16_variant_exists(tsmm_dtype dt, int KC, int NT, int RT, int products, bool il) {
    return find_bf16(dt, KC, NT, RT, products, true, il) != nullptr &&
           find_bf16(dt, KC, NT, 1, products, false, il) != nullptr;
}

hipError_t launch_splitbf16(tsmm_dtype dt, int KC, int NT, int RT, int products, bool il, const void *A,
                            const void *Bfrag, const int32_t *exps, void *C, int64_t m, int64_t n, int64_t k,
                            double alpha, double beta, int64_t grid, int block, int nt_total, int nsplit,
                            hipStream_t s) {
    const int vw = dt == TSMM_BF16 ? 8 : 4;  // elements per 16-byte vector
    const bool vec = (k % vw) == 0;
    Bf16Fn fn = find_bf16(dt, KC, NT, vec ? RT : 1, products, vec, il);
    if (!fn || nsplit < 1 || NT * nsplit != nt_total) return hipErrorInvalidValue;
    return fn(A, Bfrag, exps, C, m, n, k, alpha, beta, grid, block, nt_total, nsplit, s);
}

}  // namespace tsmm
