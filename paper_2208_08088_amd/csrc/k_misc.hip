// Packing, scaling and the any-shape fallback kernels of libtsmm, plus the
// dispatch of the streaming-kernel instantiations.
#include "k_common.h"
#include "k_stream.h"
#include "tsmm_internal.h"

namespace tsmm {

StreamFn find_stream_f64(int KC, int NT, int RT, bool vec, int cm);
StreamFn find_stream_f32(int KC, int NT, int RT, bool vec, int cm);

static inline unsigned blocks_for(int64_t count, int block) {
    return (unsigned)((count + block - 1) / block);
}

// ------------------------------------------------------------------ pack
// PACKB of Algorithm 1 (with unit scale): B is copied once into the
// fragment order in which the execute kernels consume it (tsmm_internal.h).

template <typename T>
__global__ void k_pack_frag4(const T *__restrict__ B, T *__restrict__ frag, int64_t k, int64_t n,
                             int KC, int NT, int vec, int pg, int bcol, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int lane = (int)(idx & 63);
    const int t = (int)((idx >> 6) % NT);
    const int s = (int)((idx >> 6) / NT);
    const int q = lane >> 4, j = lane & 15;
    constexpr int VW = 16 / (int)sizeof(T);
    const int64_t col = vec ? (int64_t)(s / VW) * 4 * VW + q * VW + (s % VW) : 4 * (int64_t)s + q;
    const int64_t nc = 16 * pg * (int64_t)(t / pg) + pg * j + t % pg;  // colp(t, j)
    frag[idx] = (col < k && nc < n) ? B[bcol ? col + nc * k : col * n + nc] : T(0);
}

hipError_t launch_pack_frag4(tsmm_dtype dt, bool bcol, const void *B, void *frag, int64_t k, int64_t n,
                             int KC, int NT, bool vec, int pg, hipStream_t s) {
    const int64_t total = (int64_t)(KC / 4) * NT * 64;
    if (dt == TSMM_F64)
        hipLaunchKernelGGL(k_pack_frag4<double>, dim3(blocks_for(total, 256)), dim3(256), 0, s,
                           static_cast<const double *>(B), static_cast<double *>(frag), k, n, KC, NT,
                           (int)vec, pg, (int)bcol, total);
    else if (dt == TSMM_F32)
        hipLaunchKernelGGL(k_pack_frag4<float>, dim3(blocks_for(total, 256)), dim3(256), 0, s,
                           static_cast<const float *>(B), static_cast<float *>(frag), k, n, KC, NT,
                           (int)vec, pg, (int)bcol, total);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ----------------------------------------------------------------- scale
// C = beta*C: the whole result when alpha == 0 or k == 0.

template <typename T> __global__ void k_scale(T *__restrict__ C, int64_t count, double beta) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    C[idx] = beta == 0.0 ? T(0) : (T)epilogue(0.0, 0.0, beta, (double)C[idx]);
}

hipError_t launch_scale(tsmm_dtype out_dt, void *C, int64_t count, double beta, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (out_dt == TSMM_F64)
        hipLaunchKernelGGL(k_scale<double>, dim3(blocks_for(count, 256)), dim3(256), 0, s,
                           static_cast<double *>(C), count, beta);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(blocks_for(count, 256)), dim3(256), 0, s,
                           static_cast<float *>(C), count, beta);
    return hipGetLastError();
}

// ---------------------------------------------------------------- simple
// Any shape, any alignment: one thread per output element, dot product in
// ascending order (binary64 accumulation for binary64, binary32 otherwise).
// This is the conservative fallback a plan uses outside the fragment
// kernels' classes.

template <typename T> struct SimpleIO;
template <> struct SimpleIO<double> {
    typedef double acc;
    static __device__ double ld(const double *p, int64_t i) { return p[i]; }
};
template <> struct SimpleIO<float> {
    typedef float acc;
    static __device__ float ld(const float *p, int64_t i) { return p[i]; }
};
template <> struct SimpleIO<uint16_t> {
    typedef float acc;
    static __device__ float ld(const uint16_t *p, int64_t i) { return bf16_bits_to_float(p[i]); }
};

// Row strides: A lda (op N: A(i, l) at i*lda + l; op T: A(l, i) at
// l*lda + i), B ldb, C ldc.
template <typename Tin, typename Tout, bool TRANS>
__global__ void k_simple(const Tin *__restrict__ A, const Tin *__restrict__ B, Tout *__restrict__ C,
                         int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb, int64_t ldc, double alpha,
                         double beta) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * n) return;
    const int64_t i = idx / n, j = idx % n;
    typedef typename SimpleIO<Tin>::acc Acc;
    Acc s = 0;
    for (int64_t l = 0; l < k; ++l) {
        const Acc a = TRANS ? SimpleIO<Tin>::ld(A, l * lda + i) : SimpleIO<Tin>::ld(A, i * lda + l);
        s = __builtin_fma(a, SimpleIO<Tin>::ld(B, l * ldb + j), s);
    }
    Tout *c = C + i * ldc + j;
    const double cv = beta != 0.0 ? (double)*c : 0.0;
    *c = (Tout)epilogue(alpha, (double)s, beta, cv);
}

template <typename TI, typename TO>
static void simple_t(bool trans, const void *A, const void *B, void *C, int64_t m, int64_t n, int64_t k,
                     int64_t lda, int64_t ldb, int64_t ldc, double alpha, double beta, hipStream_t s) {
    const dim3 g(blocks_for(m * n, 256)), b(256);
    if (trans)
        hipLaunchKernelGGL((k_simple<TI, TO, true>), g, b, 0, s, (const TI *)A, (const TI *)B, (TO *)C, m, n, k,
                           lda, ldb, ldc, alpha, beta);
    else
        hipLaunchKernelGGL((k_simple<TI, TO, false>), g, b, 0, s, (const TI *)A, (const TI *)B, (TO *)C, m, n, k,
                           lda, ldb, ldc, alpha, beta);
}

hipError_t launch_simple_ld(tsmm_dtype dt, bool trans, const void *A, int64_t lda, const void *B, int64_t ldb,
                            void *C, int64_t ldc, int64_t m, int64_t n, int64_t k, double alpha, double beta,
                            hipStream_t s) {
    if (m * n <= 0) return hipSuccess;
    if (dt == TSMM_F64)
        simple_t<double, double>(trans, A, B, C, m, n, k, lda, ldb, ldc, alpha, beta, s);
    else if (dt == TSMM_F32)
        simple_t<float, float>(trans, A, B, C, m, n, k, lda, ldb, ldc, alpha, beta, s);
    else
        simple_t<uint16_t, float>(trans, A, B, C, m, n, k, lda, ldb, ldc, alpha, beta, s);
    return hipGetLastError();
}

static hipError_t simple(tsmm_dtype dt, bool trans, const void *A, const void *B, void *C, int64_t m,
                         int64_t n, int64_t k, double alpha, double beta, hipStream_t s) {
    return launch_simple_ld(dt, trans, A, trans ? m : k, B, n, C, n, m, n, k, alpha, beta, s);
}

hipError_t launch_simple_n(tsmm_dtype dt, const void *A, const void *B, void *C, int64_t m,
                           int64_t n, int64_t k, double alpha, double beta, hipStream_t s) {
    return simple(dt, false, A, B, C, m, n, k, alpha, beta, s);
}
hipError_t launch_simple_t(tsmm_dtype dt, const void *A, const void *B, void *C, int64_t m,
                           int64_t n, int64_t k, double alpha, double beta, hipStream_t s) {
    return simple(dt, true, A, B, C, m, n, k, alpha, beta, s);
}

// ------------------------------------------------------- stream dispatch

static StreamFn find_stream(tsmm_dtype dt, int KC, int NT, int RT, bool vec, int cm) {
    if (dt == TSMM_F64) return find_stream_f64(KC, NT, RT, vec, cm);
    if (dt == TSMM_F32) return find_stream_f32(KC, NT, RT, vec, cm);
    return nullptr;
}

bool stream_variant_exists(tsmm_dtype dt, int KC, int NT, int RT, bool vec, int cm) {
    return find_stream(dt, KC, NT, RT, vec, cm) != nullptr;
}

hipError_t launch_stream(tsmm_dtype dt, int KC, int NT, int RT, bool vec, int cm, const void *A,
                         const void *Bfrag, void *C, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldc,
                         double alpha, double beta, int64_t grid, int block, int nt_total, int nsplit,
                         hipStream_t s) {
    StreamFn fn = find_stream(dt, KC, NT, RT, vec, cm);
    if (!fn || nsplit < 1 || NT * nsplit != nt_total) return hipErrorInvalidValue;
    return fn(A, Bfrag, C, m, n, k, lda, ldc, alpha, beta, grid, block, nt_total, nsplit, s);
}

}  // namespace tsmm
