// Column-major operands (the layout the paper's analysis assumes):
// C = alpha*A*B + beta*C with A (m x k), B (k x n) and C (m x n) stored
// column by column, m large, k and n small.  binary64 or binary32.
//
// In row-major terms this is C^T = B^T * A^T: a small matrix times a wide
// one.  On the matrix cores the roles of the operands swap with respect to
// the row-major streaming kernel: the packed B (the same 16x16x4 fragment
// image, lane 16*q + j holding B(col(s, q), 16*t + j)) is the product's
// first operand, whose rows are now columns of C, and A streams in as the
// second operand: lane (q, j) supplies A(i, col(s, q)) for an m index i of
// its own.  A column of A is contiguous, so the 16 lanes of one q read 16
// consecutive m indices; each lane loads VW of them as one 16-byte vector
// (VW = 2 binary64, 4 binary32) and feeds them to VW products, one per
// m-tile u, in which lane j stands for m index i0 + VW*j + u.  The
// accumulators of lane (q, j) then hold, for each C column (row of the
// product), VW adjacent m indices: every C access is one 16-byte vector.
//
// A wavefront owns column blocks of 16*VW m indices over all k and the
// workgroup's NT column tiles of C; A moves in chunks of CH k-steps, the
// next chunk in flight while the current one is multiplied.  Column groups
// (nsplit) divide the C columns among workgroups as in the row-major kernel
// when the packed slice would not fit the LDS.
#include "k_common.h"
#include "k_stream.h"  // BlockMap: workgroup -> (row block, column group)
#include "tsmm_internal.h"

namespace tsmm {

constexpr int kColBlock = 256;

template <typename T, int KC> struct ColCfg {
    static constexpr int S = KC / 4;                // k-steps
    // k-steps per A chunk: 8 for binary64 at k classes of 128 and more (a
    // longer prefetch ahead of the matrix-core bound products), else 4
    static constexpr int CH = S < 4 ? S : (sizeof(T) == 8 && KC >= 128 ? 8 : 4);
    static constexpr int NCH = S / CH;              // chunks per column block
};

// The lane's A vectors of chunk c of column block `blk` (k-slot mapping
// col(s, q) = 4*s + q, the packed image's scalar mapping).  The loads keep
// the default cache policy: with column groups, a second wavefront reads
// the same A chunk right after the first, and a streaming (non-temporal)
// load leaves no line in the L2 for it (measured: A read 1.8 to 1.9 times
// from memory with non-temporal loads).  Every load is
// issued, with no branch around it and no select after it (a load under a
// branch makes the compiler wait for every outstanding load, the prefetch
// included, before the products; a select after it waits for the load
// right away): a lane whose vector lies past m (m is a multiple of VW, so a
// vector lies wholly inside or outside) reads A's first vector, whose
// results are never stored; a lane whose column lies past k reads `zp`, 16
// zeros of the packed image (its last k-slot, which lies past k whenever a
// column does), so no infinite A value meets a zero of B.
template <typename T, int KC>
__device__ __forceinline__ void col_load(const T *__restrict__ A, const T *__restrict__ zp, int64_t m, int k,
                                         int64_t lda, int64_t blk, int c, int j, int q,
                                         typename Mfma4<T>::vec (&x)[ColCfg<T, KC>::CH]) {
    typedef typename Mfma4<T>::vec vec_t;
    constexpr int VW = Mfma4<T>::VW;
    constexpr int CH = ColCfg<T, KC>::CH;
    const int64_t i = blk * 16 * VW + VW * j;
#pragma unroll
    for (int e = 0; e < CH; ++e) {
        const int col = 4 * (c * CH + e) + q;
        const T *p = col < k ? (i < m ? A + i + col * lda : A) : zp;
        x[e] = *reinterpret_cast<const vec_t *>(p);
    }
}

// Products of chunk c: CH k-steps x NT column tiles x VW m-tiles (SNT
// column tiles per k-step in LDS; bofs holds the lane and the wavefront
// group's first tile).
template <typename T, int KC, int NT, int SNT>
__device__ __forceinline__ void col_products(const T *__restrict__ sB, int c, int bofs,
                                             const typename Mfma4<T>::vec (&x)[ColCfg<T, KC>::CH],
                                             typename Mfma4<T>::acc (&acc)[Mfma4<T>::VW][NT]) {
    constexpr int VW = Mfma4<T>::VW;
    constexpr int CH = ColCfg<T, KC>::CH;
#pragma unroll
    for (int e = 0; e < CH; ++e) {
        const int s = c * CH + e;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const T b = sB[bofs + (s * SNT + t) * 64];
#pragma unroll
            for (int u = 0; u < VW; ++u) acc[u][t] = Mfma4<T>::op(b, x[e][u], acc[u][t]);
        }
    }
}

// C vectors of column block blk (beta != 0): lane (q, j) reads C columns
// n0 + 16*t + row(q, r) at m indices i0 + VW*j + u, u < VW (one 16-byte
// vector each).  All loads are issued with no branch around them (vectors
// past m or n read C's first vector; their results are never stored).
template <typename T, int NT>
__device__ __forceinline__ void col_load_c(const T *__restrict__ C, int64_t m, int n, int64_t ldc, int64_t blk,
                                           int n0, int j, int q, typename Mfma4<T>::vec (&cv)[NT][4]) {
    typedef Mfma4<T> M;
    typedef typename M::vec vec_t;
    constexpr int VW = M::VW;
    const int64_t i = blk * 16 * VW + VW * j;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = n0 + 16 * t + M::row(q, r);
            const T *p = (i < m && col < n) ? C + i + col * ldc : C;
            cv[t][r] = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(p));
        }
}

// Epilogue of column block blk: lane (q, j) holds C columns n0 + 16*t +
// row(q, r) at m indices i0 + VW*j + u, u < VW (one 16-byte vector); cv
// holds the C values when BC (beta != 0).
template <typename T, int NT, bool BC>
__device__ __forceinline__ void col_epilogue(T *__restrict__ C, int64_t m, int n, int64_t ldc, int64_t blk, int n0,
                                             int j, int q, double alpha, double beta,
                                             const typename Mfma4<T>::acc (&acc)[Mfma4<T>::VW][NT],
                                             const typename Mfma4<T>::vec (&cv)[NT][4]) {
    typedef Mfma4<T> M;
    typedef typename M::vec vec_t;
    constexpr int VW = M::VW;
    const int64_t i = blk * 16 * VW + VW * j;
    if (i >= m) return;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = n0 + 16 * t + M::row(q, r);
            if (col >= n) continue;
            vec_t v;
#pragma unroll
            for (int u = 0; u < VW; ++u)
                v[u] = (T)epilogue(alpha, (double)acc[u][t][r], BC ? beta : 0.0, BC ? (double)cv[t][r][u] : 0.0);
            __builtin_nontemporal_store(v, reinterpret_cast<vec_t *>(C + i + col * ldc));
        }
}

// One column block: zero the accumulators, run the NCH chunks (chunk c in
// buffer (PAR + c) % 2; the load of the chunk after it goes to the other
// buffer), then the epilogue.  nb: the next column block of this wavefront
// (its first chunk is loaded during the last chunk of this one).  BC: the
// block's C vectors are read at the start of the last chunk, before that
// prefetch, so that the epilogue's wait for them does not include it.
template <typename T, int KC, int NT, int SNT, int PAR, bool BC>
__device__ __forceinline__ void col_block(const T *__restrict__ A, const T *__restrict__ zp, const T *__restrict__ sB,
                                          T *__restrict__ C,
                                          int64_t m, int n, int k, int64_t lda, int64_t ldc, int64_t blk, int64_t nb,
                                          int n0, int t0, int lane, int j, int q, double alpha, double beta,
                                          typename Mfma4<T>::vec (&x0)[ColCfg<T, KC>::CH],
                                          typename Mfma4<T>::vec (&x1)[ColCfg<T, KC>::CH]) {
    typedef Mfma4<T> M;
    constexpr int VW = M::VW;
    constexpr int NCH = ColCfg<T, KC>::NCH;
    typename M::acc acc[VW][NT];
    typename M::vec cv[NT][4];
#pragma unroll
    for (int u = 0; u < VW; ++u)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[u][t] = typename M::acc{};
    // the fragments are re-read from LDS for every block: an opaque lane
    // offset keeps the compiler from holding them in registers across blocks
    int bofs = lane + t0 * 64;
    asm volatile("" : "+v"(bofs));
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const bool last = c + 1 == NCH;
        const int64_t lb = last ? nb : blk;
        const int lc = last ? 0 : c + 1;
        if constexpr (BC) {
            if (last) col_load_c<T, NT>(C, m, n, ldc, blk, n0, j, q, cv);
        }
        if (((PAR + c) & 1) == 0) {
            col_load<T, KC>(A, zp, m, k, lda, lb, lc, j, q, x1);
            __builtin_amdgcn_sched_barrier(0);
            col_products<T, KC, NT, SNT>(sB, c, bofs, x0, acc);
        } else {
            col_load<T, KC>(A, zp, m, k, lda, lb, lc, j, q, x0);
            __builtin_amdgcn_sched_barrier(0);
            col_products<T, KC, NT, SNT>(sB, c, bofs, x1, acc);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    col_epilogue<T, NT, BC>(C, m, n, ldc, blk, n0, j, q, alpha, beta, acc, cv);
}

// KC: packed k class; NT: column tiles of C per wavefront; NG: column
// groups inside the workgroup (its wavefronts split into NG groups that
// walk the same column blocks, each over NT tiles of its own, so the
// second group's read of an A chunk follows the first through the cache);
// nt_total: column tiles of the packed image; nsplit: column groups across
// workgroups; BC: beta != 0 (C is read), a kernel of its own so that the
// beta = 0 kernel holds no registers for C.
template <typename T, int KC, int NT, int NG, bool BC>
__global__ __launch_bounds__(kColBlock) void k_colmajor(const T *__restrict__ A, const T *__restrict__ Bf,
                                                         T *__restrict__ C, int64_t m, int n, int k, int64_t lda,
                                                         int64_t ldc, double alpha, double beta, int nt_total,
                                                         int nsplit) {
    typedef Mfma4<T> M;
    typedef typename M::vec vec_t;
    constexpr int VW = M::VW;
    constexpr int S = KC / 4;
    constexpr int SNT = NT * NG;  // column tiles of this workgroup
    constexpr int FRAG = S * SNT * 64;
    constexpr int NCH = ColCfg<T, KC>::NCH;
    const BlockMap bm = block_map(nsplit);

    __shared__ T sB[FRAG];
    for (int idx = threadIdx.x * VW; idx < FRAG; idx += blockDim.x * VW) {
        const int s = idx / (SNT * 64), rem = idx % (SNT * 64);
        *reinterpret_cast<vec_t *>(&sB[idx]) =
            *reinterpret_cast<const vec_t *>(&Bf[(s * nt_total + bm.group * SNT) * 64 + rem]);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const int wpg = (blockDim.x >> 6) / NG;  // wavefronts per column group
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = wave / wpg, wig = wave % wpg;
    const int t0 = grp * NT;                         // first LDS tile of this wavefront's group
    const int n0 = (bm.group * SNT + t0) * 16;       // its first column of C
    const int64_t nblk = (m + 16 * VW - 1) / (16 * VW);
    const int64_t stride = bm.nrb * wpg;
    int64_t blk = bm.rb * wpg + wig;
    if (blk >= nblk) return;
    // 16 zeros (lanes 48..63 of k-step S-1: k-slot KC-1) for columns past k
    const T *zp = Bf + (int64_t)(S - 1) * nt_total * 64 + 48;
    vec_t x0[ColCfg<T, KC>::CH], x1[ColCfg<T, KC>::CH];
    col_load<T, KC>(A, zp, m, k, lda, blk, 0, j, q, x0);
    // Blocks go in pairs: a block of NCH chunks that starts in buffer p
    // leaves the next block's first chunk in buffer (p + NCH) % 2, so after
    // a pair the first chunk is back in x0.  A pair's second block may lie
    // past the last one, where nothing is loaded or stored.
    for (; blk < nblk; blk += 2 * stride) {
        col_block<T, KC, NT, SNT, 0, BC>(A, zp, sB, C, m, n, k, lda, ldc, blk, blk + stride, n0, t0, lane, j, q,
                                         alpha, beta, x0, x1);
        col_block<T, KC, NT, SNT, NCH & 1, BC>(A, zp, sB, C, m, n, k, lda, ldc, blk + stride, blk + 2 * stride, n0,
                                               t0, lane, j, q, alpha, beta, x0, x1);
    }
}

template <typename T, int KC, int NT, int NG>
hipError_t run_colmajor(const void *A, const void *Bf, void *C, int64_t m, int64_t n, int64_t k, int64_t lda,
                        int64_t ldc, double alpha, double beta, int64_t grid, int nt_total, int nsplit,
                        hipStream_t s) {
    if (beta != 0.0)
        hipLaunchKernelGGL((k_colmajor<T, KC, NT, NG, true>), dim3((unsigned)grid), dim3(kColBlock), 0, s,
                           static_cast<const T *>(A), static_cast<const T *>(Bf), static_cast<T *>(C), m, (int)n,
                           (int)k, lda, ldc, alpha, beta, nt_total, nsplit);
    else
        hipLaunchKernelGGL((k_colmajor<T, KC, NT, NG, false>), dim3((unsigned)grid), dim3(kColBlock), 0, s,
                           static_cast<const T *>(A), static_cast<const T *>(Bf), static_cast<T *>(C), m, (int)n,
                           (int)k, lda, ldc, alpha, beta, nt_total, nsplit);
    return hipGetLastError();
}

typedef hipError_t (*ColFn)(const void *, const void *, void *, int64_t, int64_t, int64_t, int64_t, int64_t, double,
                            double, int64_t, int, int, hipStream_t);
struct ColEntry {
    tsmm_dtype dt;
    int KC, NT, NG;
    ColFn fn;
};

// packed slice (KC/4 * NT * NG * 64 values) within 128 KiB of LDS;
// column tiles per wavefront within the registers: 8 only at k class 4 (at
// larger classes the beta != 0 kernel spilled to scratch when compiled),
// else at most 4, and two groups of 4 in one workgroup where the slice
// fits
#define TSMM_COL_NT4(T, DT, KC) {DT, KC, 1, 1, &run_colmajor<T, KC, 1, 1>}, {DT, KC, 2, 1, &run_colmajor<T, KC, 2, 1>}, \
    {DT, KC, 4, 1, &run_colmajor<T, KC, 4, 1>},
#define TSMM_COL_NT8(T, DT, KC) TSMM_COL_NT4(T, DT, KC) {DT, KC, 8, 1, &run_colmajor<T, KC, 8, 1>},
static const ColEntry kColTable[] = {
    TSMM_COL_NT8(double, TSMM_F64, 4) TSMM_COL_NT4(double, TSMM_F64, 8) TSMM_COL_NT4(double, TSMM_F64, 16)
    TSMM_COL_NT4(double, TSMM_F64, 32) TSMM_COL_NT4(double, TSMM_F64, 64) TSMM_COL_NT4(double, TSMM_F64, 128)
    TSMM_COL_NT4(double, TSMM_F64, 256) {TSMM_F64, 128, 4, 2, &run_colmajor<double, 128, 4, 2>},
    TSMM_COL_NT8(float, TSMM_F32, 4) TSMM_COL_NT4(float, TSMM_F32, 8) TSMM_COL_NT4(float, TSMM_F32, 16)
    TSMM_COL_NT4(float, TSMM_F32, 32) TSMM_COL_NT4(float, TSMM_F32, 64) TSMM_COL_NT4(float, TSMM_F32, 128)
    TSMM_COL_NT4(float, TSMM_F32, 256) {TSMM_F32, 128, 4, 2, &run_colmajor<float, 128, 4, 2>},
    {TSMM_F32, 256, 4, 2, &run_colmajor<float, 256, 4, 2>},
};
#undef TSMM_COL_NT4
#undef TSMM_COL_NT8

static const ColEntry *find_col(tsmm_dtype dt, int KC, int NT, int NG) {
    for (const ColEntry &e : kColTable)
        if (e.dt == dt && e.KC == KC && e.NT == NT && e.NG == NG) return &e;
    return nullptr;
}

bool colmajor_variant_exists(tsmm_dtype dt, int KC, int NT, int NG) { return find_col(dt, KC, NT, NG) != nullptr; }

hipError_t launch_colmajor(tsmm_dtype dt, int KC, int NT, int NG, const void *A, const void *Bf, void *C, int64_t m,
                           int64_t n, int64_t k, int64_t lda, int64_t ldc, double alpha, double beta, int64_t grid,
                           int nt_total, int nsplit, hipStream_t s) {
    const ColEntry *e = find_col(dt, KC, NT, NG);
    const int vw = dt == TSMM_F64 ? 2 : 4;
    if (!e || NT * NG * nsplit != nt_total || m % vw != 0 || lda % vw != 0 || ldc % vw != 0 || lda < m || ldc < m)
        return hipErrorInvalidValue;
    return e->fn(A, Bf, C, m, n, k, lda, ldc, alpha, beta, grid, nt_total, nsplit, s);
}

}  // namespace tsmm
