// op T split-k: C = alpha*A^T*B + beta*C for A (K x m) and B (K x n), both
// tall, row-major, with a long shared dimension K and small m, n.
//
// The shared dimension is cut into P contiguous row ranges (split-k).
// Pass 1: workgroup p streams its rows of A and B once and accumulates the
// m x n partial product with 16x16x4 binary64 matrix-core products (the
// rows of A and B are the k dimension of the product, so each wavefront
// reads its 4-row groups with full 128-byte row segments), combines its
// wavefronts' partials through LDS in a fixed order and writes W[p].
// Pass 2: C = alpha * (W[0] + W[1] + ... + W[P-1]) + beta*C with the sum
// taken in ascending p, so a plan's result is bitwise repeatable.  The
// kernel boundary is the only synchronisation between workgroups
// (Sec. IV-A.2: no synchronisation inside the computation).
#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

constexpr int kSplitBlock = 256;

template <int MT, int NT, int RG>
__global__ __launch_bounds__(kSplitBlock) void k_splitk_pass1(const double *__restrict__ A,
                                                               const double *__restrict__ B,
                                                               double *__restrict__ W, int64_t K,
                                                               int m, int n, int64_t rows_per_split) {
    constexpr int BM = 16 * MT, BN = 16 * NT;
    __shared__ double red[BM * BN];

    const int p = blockIdx.x;
    const int nbn = (n + BN - 1) / BN;
    const int m0 = (blockIdx.y / nbn) * BM, n0 = (blockIdx.y % nbn) * BN;
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nwave = blockDim.x >> 6;
    const int64_t r0 = (int64_t)p * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < K ? r0 + rows_per_split : K;

    d4v acc[MT][NT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = d4v{};

    bool acol[MT], bcol[NT];
#pragma unroll
    for (int a = 0; a < MT; ++a) acol[a] = m0 + 16 * a + j < m;
#pragma unroll
    for (int b = 0; b < NT; ++b) bcol[b] = n0 + 16 * b + j < n;

    // Wavefront w takes the 4*RG-row groups w, w + nwave, w + 2*nwave, ...
    // of its range.  Software pipeline: the next group's rows are in flight
    // while the current group's products run.  Rows are read through
    // buffer resources whose byte count ends at row r1, so rows past the
    // range read 0.
    const int64_t gstride = (int64_t)nwave * 4 * RG;
    auto load = [&](int64_t g, double (&av)[RG][MT], double (&bv)[RG][NT]) {
        const int64_t rr = uniform64(r0 + g);  // first row of the group
        // the group's rows that exist (at most 4*RG: far below kOOB)
        const int64_t rows = r1 - rr < 4 * RG ? r1 - rr : 4 * RG;
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + rr * m + m0, (rows * m - m0) * 8);
        const __amdgpu_buffer_rsrc_t rb = make_rsrc(B + rr * n + n0, (rows * n - n0) * 8);
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
            const int row = 4 * rg + q;
            // columns past m (n) read through kOOB, which returns 0: no
            // branch around a load (that would make the compiler wait for
            // every outstanding load, the prefetch included, before the
            // products)
#pragma unroll
            for (int a = 0; a < MT; ++a)
                av[rg][a] = BufIO<double>::load1(ra, acol[a] ? (row * m + 16 * a + j) * 8 : kOOB);
#pragma unroll
            for (int b = 0; b < NT; ++b)
                bv[rg][b] = BufIO<double>::load1(rb, bcol[b] ? (row * n + 16 * b + j) * 8 : kOOB);
        }
    };
    auto mma = [&](const double (&av)[RG][MT], const double (&bv)[RG][NT]) {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
            for (int a = 0; a < MT; ++a)
#pragma unroll
                for (int b = 0; b < NT; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rg][a], bv[rg][b], acc[a][b], 0, 0, 0);
    };
    // Ping-pong over two register sets, in pairs of groups with no branch
    // between them (past r1 the resources are empty and reads return 0, so
    // a pair's second group may lie beyond the range); the scheduling
    // barriers keep each prefetch ahead of the products it overlaps.
    double a0[RG][MT], b0[RG][NT], a1[RG][MT], b1[RG][NT];
    int64_t g = (int64_t)__builtin_amdgcn_readfirstlane(wave) * 4 * RG;
    if (r0 + g < r1) load(g, a0, b0);
    for (; r0 + g < r1; g += 2 * gstride) {
        load(g + gstride, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        mma(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(g + 2 * gstride, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
    }

    // combine the wavefronts in the fixed order ((w0 + w1) + w2) + ...
    for (int w = 0; w < nwave; ++w) {
        if (wave == w) {
#pragma unroll
            for (int a = 0; a < MT; ++a)
#pragma unroll
                for (int b = 0; b < NT; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = (16 * a + Mfma4<double>::row(q, r)) * BN + 16 * b + j;
                        red[e] = w == 0 ? acc[a][b][r] : red[e] + acc[a][b][r];
                    }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < BM * BN; e += blockDim.x) {
        const int i = m0 + e / BN, jj = n0 + e % BN;
        if (i < m && jj < n) W[((int64_t)p * m + i) * n + jj] = red[e];
    }
}

// Pass 2: 16 outputs per workgroup; thread (seg, o) sums the partials of
// segment seg (P split into 16 contiguous segments) in ascending order,
// then the 16 segment sums are added in ascending order.  The summation
// tree depends only on P, so a plan's result is bitwise repeatable.
constexpr int kP2Out = 16, kP2Seg = 16;
__global__ __launch_bounds__(kP2Out *kP2Seg) void k_splitk_pass2(const double *__restrict__ W, double *__restrict__ C,
                                                                 int64_t mn, int P, double alpha, double beta) {
    __shared__ double part[kP2Seg][kP2Out];
    const int o = threadIdx.x % kP2Out, seg = threadIdx.x / kP2Out;
    const int64_t e = (int64_t)blockIdx.x * kP2Out + o;
    const int per = (P + kP2Seg - 1) / kP2Seg;
    const int p0 = seg * per, p1 = p0 + per < P ? p0 + per : P;
    double s = 0.0;
    if (e < mn && p0 < p1) {
        s = W[(int64_t)p0 * mn + e];
#pragma unroll 8
        for (int p = p0 + 1; p < p1; ++p) s = s + W[(int64_t)p * mn + e];
    }
    part[seg][o] = s;
    __syncthreads();
    if (seg == 0 && e < mn) {
        double t = part[0][o];
        for (int g = 1; g < kP2Seg; ++g) t = t + part[g][o];
        const double c = beta != 0.0 ? C[e] : 0.0;
        C[e] = epilogue(alpha, t, beta, c);
    }
}

typedef void (*SplitFn)(const double *, const double *, double *, int64_t, int, int, int64_t);
struct SplitEntry {
    int MT, NT, RG;
    SplitFn fn;
};
#define TSMM_SK(MT, NT, RG) {MT, NT, RG, &k_splitk_pass1<MT, NT, RG>},
#define TSMM_SK_RG(MT, NT) TSMM_SK(MT, NT, 1) TSMM_SK(MT, NT, 2) TSMM_SK(MT, NT, 4)
static const SplitEntry kSplit[] = {
    TSMM_SK_RG(1, 1) TSMM_SK_RG(1, 2) TSMM_SK_RG(1, 4) TSMM_SK_RG(2, 1) TSMM_SK_RG(2, 2)
    TSMM_SK_RG(2, 4) TSMM_SK_RG(4, 1) TSMM_SK_RG(4, 2) TSMM_SK_RG(4, 4)
};

static SplitFn find_split(int MT, int NT, int RG) {
    for (const SplitEntry &e : kSplit)
        if (e.MT == MT && e.NT == NT && e.RG == RG) return e.fn;
    return nullptr;
}

bool splitk_variant_exists(int MT, int NT, int RG) { return find_split(MT, NT, RG) != nullptr; }

hipError_t launch_splitk(int MT, int NT, int RG, const double *A, const double *B, double *W,
                         double *C, int64_t K, int64_t m, int64_t n, int P, double alpha,
                         double beta, int block, hipStream_t s) {
    SplitFn fn = find_split(MT, NT, RG);
    if (!fn || P < 1) return hipErrorInvalidValue;
    int64_t rps = (K + P - 1) / P;
    rps = (rps + 15) / 16 * 16;
    const int64_t nbm = (m + 16 * MT - 1) / (16 * MT), nbn = (n + 16 * NT - 1) / (16 * NT);
    hipLaunchKernelGGL(fn, dim3((unsigned)P, (unsigned)(nbm * nbn)), dim3(block), 0, s, A, B, W, K,
                       (int)m, (int)n, rps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t mn = m * n;
    hipLaunchKernelGGL(k_splitk_pass2, dim3((unsigned)((mn + kP2Out - 1) / kP2Out)), dim3(kP2Out * kP2Seg), 0, s,
                       (const double *)W, C, mn, P, alpha, beta);
    return hipGetLastError();
}

}  // namespace tsmm
