// op N, binary64, vector-ALU path: C = alpha*A*B + beta*C.
//
// On gfx950 the binary64 fused multiply-add of the vector ALU sustains a
// higher rate than the binary64 16x16x4 matrix-core product (measured on
// MI355X: about 72 vs 48 TFLOP/s), so shapes that are bound by binary64
// arithmetic (k and n of 64 and more) use this kernel.  It is a register-
// blocked GEBB_t in the paper's sense (Sec. IV-B): every lane owns one row
// of a 64-row tile and NB consecutive columns of C as accumulators; the
// A row streams through registers 8 elements at a time (prefetched one
// chunk ahead), and each B element is wave-uniform, so it reaches the FMA
// as a scalar operand (scalar loads of the row-major packed B) and is reused
// by all 64 rows of the tile.  The four wavefronts of a workgroup take
// four column groups of the same rows, so each A row is fetched from HBM
// once per workgroup and re-read from the L1/L2 by the other three.
#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

constexpr int kValuWaves = 4;

template <int NB>
__global__ __launch_bounds__(64 * kValuWaves) void k_valu64(const double *__restrict__ A,
                                                             const double *__restrict__ B,
                                                             double *__restrict__ C, int64_t m, int n, int k,
                                                             double alpha, double beta, int ncg) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cg = (int)blockIdx.y * kValuWaves + wave;  // column group
    if (cg >= ncg) return;
    const int c0 = cg * NB;
    const int64_t ntile = (m + 63) >> 6;

    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t row0 = uniform64(tile * 64);
        int64_t rows = m - row0;
        rows = rows > 64 ? 64 : rows;
        // rows beyond m read 0 and are not written
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + row0 * k, rows * (int64_t)k * 8);
        const __amdgpu_buffer_rsrc_t rc = make_rsrc(C + row0 * n + c0, (rows * (int64_t)n - c0) * 8);
        const __amdgpu_buffer_rsrc_t rl = make_rsrc(C + row0 * n + c0, beta != 0.0 ? (rows * (int64_t)n - c0) * 8 : 0);
        const int aoff = lane * k * 8;
        const int coff = lane * n * 8;

        // C rows for the epilogue, requested first so they arrive under the
        // products
        d2v cv[NB / 2];
#pragma unroll
        for (int j = 0; j < NB / 2; ++j) cv[j] = BufIO<double>::load_vec(rl, coff + 16 * j);

        double acc[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j] = 0.0;

        d2v a_cur[4], a_nxt[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) a_cur[e] = BufIO<double>::load_vec(ra, aoff + 16 * e);
        for (int l0 = 0; l0 < k; l0 += 8) {
            // next chunk of the row (past k the offset leaves the row: the
            // values are unused, and past the last row the resource ends)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                a_nxt[e] = BufIO<double>::load_vec(ra, l0 + 8 < k ? aoff + (l0 + 8) * 8 + 16 * e : kOOB);
            const double *__restrict__ brow = B + (int64_t)l0 * n + c0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const double a = a_cur[e >> 1][e & 1];
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = __builtin_fma(a, brow[e * n + j], acc[j]);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) a_cur[e] = a_nxt[e];
        }

#pragma unroll
        for (int j = 0; j < NB / 2; ++j) {
            d2v v;
            v[0] = epilogue(alpha, acc[2 * j], beta, cv[j][0]);
            v[1] = epilogue(alpha, acc[2 * j + 1], beta, cv[j][1]);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rc, coff + 16 * j, 0, 2);
        }
    }
}

bool valu64_variant_exists(int NB) { return NB == 16 || NB == 32; }

hipError_t launch_valu64(int NB, const double *A, const double *B, double *C, int64_t m, int64_t n, int64_t k,
                         double alpha, double beta, int64_t grid, hipStream_t s) {
    if (!valu64_variant_exists(NB) || n % NB != 0 || k % 8 != 0) return hipErrorInvalidValue;
    const int ncg = (int)(n / NB);
    const dim3 g((unsigned)grid, (unsigned)((ncg + kValuWaves - 1) / kValuWaves)), b(64 * kValuWaves);
    switch (NB) {
    case 16: hipLaunchKernelGGL(k_valu64<16>, g, b, 0, s, A, B, C, m, (int)n, (int)k, alpha, beta, ncg); break;
    default: hipLaunchKernelGGL(k_valu64<32>, g, b, 0, s, A, B, C, m, (int)n, (int)k, alpha, beta, ncg); break;
    }
    return hipGetLastError();
}

}  // namespace tsmm
