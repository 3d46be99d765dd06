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

// Workgroup -> (row block, column group).  With nsplit column groups, the
// nsplit workgroups that share a row block get ids 8 apart, so they land on
// the same XCD (ids are dealt to the 8 XCDs round robin) at about the same
// time, and the second read of their A rows hits that XCD's L2.
struct BlockMap {
    int group;     // column group of this workgroup
    int64_t rb;    // row-block index among the gridDim.x / nsplit row blocks
    int64_t nrb;   // number of row blocks
};
__device__ __forceinline__ BlockMap block_map(int nsplit) {
    BlockMap b;
    if (nsplit == 1) {
        b.group = 0;
        b.rb = blockIdx.x;
        b.nrb = gridDim.x;
    } else {
        const int64_t slot = blockIdx.x >> 3;
        b.group = (int)(slot % nsplit);
        b.rb = (slot / nsplit) * 8 + (blockIdx.x & 7);
        b.nrb = gridDim.x / nsplit;
    }
    return b;
}

// A rows of row tiles t .. t+RT-1 into registers.  One buffer resource per
// 16-row tile, sized to the tile's rows that exist, so rows beyond m read
// 0; a lane whose columns lie beyond k (ragged k) reads through the offset
// kOOB instead of branching.  voff0 is the lane's row offset j*lda*sizeof(T)
// (lda: the row stride of A in elements, >= k).
template <typename T, int KC, int RT, bool VEC>
__device__ __forceinline__ void stream_load_a(const T *__restrict__ A, int64_t m, int k, int lda, bool kfull,
                                              int64_t t,
                                              int voff0, int q, T (&a)[RT][KC / 4]) {
    typedef typename Mfma4<T>::vec vec_t;
    constexpr int VW = Mfma4<T>::VW;
    constexpr int S = KC / 4;
    constexpr int SZ = (int)sizeof(T);
    // one load instruction covers 64 bytes (vector mapping) of each of 16
    // rows.  Rows of 1 KiB and more are read with the default cache policy,
    // so that the loads of a step share each line through the cache (one
    // streaming load per line part was measured to refetch it: 7% slower at
    // k = 128 binary64); shorter rows stream (measured faster at k <= 32).
    constexpr int AUX = KC * SZ >= 1024 ? 0 : 2;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64((t + rt) * 16);
        // (rows - 1) * lda + k elements; negative (an empty resource) when
        // no row exists, with no branch
        const int rows = (int)tile_rows(m, row0);
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + row0 * lda, (int64_t)(rows * lda - (lda - k)) * SZ);
        if constexpr (VEC) {
#pragma unroll
            for (int p = 0; p < S / VW; ++p) {
                const int col = p * 4 * VW + q * VW;
                const vec_t v = BufIO<T>::template load_vec<AUX>(ra, (kfull || col < k) ? voff0 + col * SZ : kOOB);
#pragma unroll
                for (int e = 0; e < VW; ++e) a[rt][p * VW + e] = v[e];
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int col = 4 * s + q;
                a[rt][s] = BufIO<T>::template load1<AUX>(ra, (kfull || col < k) ? voff0 + col * SZ : kOOB);
            }
        }
    }
}

// The neighbouring lane's value (lane ^ 1): DPP quad permutation [1, 0, 3, 2]
// on both halves of a binary64 value.
__device__ __forceinline__ double lane_pair_swap(double x) {
    const u32x2 w = __builtin_bit_cast(u32x2, x);
    u32x2 r;
    r[0] = (uint32_t)__builtin_amdgcn_mov_dpp((int)w[0], 0xB1, 0xF, 0xF, false);
    r[1] = (uint32_t)__builtin_amdgcn_mov_dpp((int)w[1], 0xB1, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}

// One row step of the streaming kernel: tiles t .. t+RT-1 are multiplied
// with the A rows already in a_use while the rows of tiles tnext.. stream
// into a_load.  C rows are read through a resource that is empty when
// beta == 0 (no traffic, no branch), before the prefetch is issued, so the
// epilogue's wait for them does not include the prefetch.
// How C moves (CM & 3): 0 element by element; 1 interleaved columns (the
// fragments of PG adjacent columns in one lane, 16-byte vectors); 2 lane
// pairs (binary64, one column tile, n even): lanes j and j ^ 1 swap half of
// their accumulators so that each holds two adjacent columns of a row and C
// moves in 16-byte vectors with the plain column order of the packed B.
// CM & 4: the 16-byte C stores take the default cache policy instead of the
// streaming one (chosen at launch for beta == 0 on the memory-bound binary64
// classes: there it was measured 2-13% faster, and 2-3% slower at
// beta != 0, where C is also read).
template <typename T, int KC, int NT, int RT, bool VEC, int CM, bool CPRE = true>
__device__ __forceinline__ void stream_step(const T *__restrict__ A, const T *__restrict__ Bsrc, int bstride,
                                            T *__restrict__ C, int64_t m, int n, int k, int lda, int ldc,
                                            bool kfull, double alpha,
                                            double beta, int col0, int64_t t, int64_t tnext, int voff0, int q,
                                            int lane, int j, const T (&a_use)[RT][KC / 4],
                                            T (&a_load)[RT][KC / 4]) {
    typedef Mfma4<T> M;
    typedef typename M::acc acc_t;
    constexpr int S = KC / 4;
    constexpr int SZ = (int)sizeof(T);

    __amdgpu_buffer_rsrc_t rc[RT], rl[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64((t + rt) * 16);
        const int rows = (int)tile_rows(m, row0);
        const int64_t bytes = (int64_t)(rows * ldc - (ldc - n + col0)) * SZ;
        rc[rt] = make_rsrc(C + row0 * ldc + col0, bytes);
        rl[rt] = make_rsrc(C + row0 * ldc + col0, beta != 0.0 ? bytes : 0);
    }
    // With interleaved columns (CM 1; tsmm_internal.h) tile tt of lane j is
    // column colp(tt) of the column group, a lane holds PG adjacent columns
    // of each row in the tiles of one group, and C moves in 16-byte vectors
    // (n is then a multiple of PG); otherwise element by element.
    constexpr int PG = (CM & 3) == 1 ? Mfma4<T>::VW : 1;
    static_assert((CM & 3) != 1 || NT % PG == 0, "interleave groups must be whole");
    constexpr bool cvec = (CM & 3) == 1;
    constexpr bool PAIR = (CM & 3) == 2;
    constexpr int SAUX = (CM & 4) ? 0 : 2;  // cache policy of the 16-byte C stores
    static_assert(!PAIR || (sizeof(T) == 8 && NT == 1 && CPRE), "lane pairs: binary64, one column tile");
    auto colp = [=](int tt) { return 16 * PG * (tt / PG) + PG * j + tt % PG; };
    // byte offset of accumulator element (tt, r): row M::row(q, r), column
    // colp(tt); kOOB for columns beyond n
    auto coff = [=](int tt, int r) {
        return (col0 + colp(tt) < n) ? (M::row(q, r) * ldc + colp(tt)) * SZ : kOOB;
    };
    // byte offset of the vector of group g (columns colp(PG*g) ..): whole
    // vectors lie inside or outside n when n % PG == 0
    auto voff = [=](int g, int r) {
        return (col0 + colp(PG * g) < n) ? (M::row(q, r) * ldc + colp(PG * g)) * SZ : kOOB;
    };
    // lane pairs: after the swap the even lane of a pair holds row
    // M::row(q, 2p) and the odd lane row M::row(q, 2p + 1), both at columns
    // j & ~1 and j | 1 (whole vectors lie inside or outside n when n is even)
    const int odd = j & 1;
    auto poff = [=](int p) {
        return (col0 + (j & ~1) < n) ? (M::row(q, 2 * p + odd) * ldc + (j & ~1)) * SZ : kOOB;
    };
    T cv[RT][NT][4];
    typename M::vec cp[RT][2];
    if constexpr (CPRE) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            if constexpr (PAIR) {
#pragma unroll
                for (int p = 0; p < 2; ++p) cp[rt][p] = BufIO<T>::load_vec(rl[rt], poff(p));
            } else if constexpr (cvec) {
#pragma unroll
                for (int g = 0; g < NT / PG; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const typename M::vec v = BufIO<T>::load_vec(rl[rt], voff(g, r));
#pragma unroll
                        for (int i = 0; i < PG; ++i) cv[rt][PG * g + i][r] = v[i];
                    }
            } else {
#pragma unroll
                for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) cv[rt][tt][r] = BufIO<T>::load1(rl[rt], coff(tt, r));
            }
        }
    }

    // past the last tile the resource holds no rows: the loads return 0
    // without touching memory
    stream_load_a<T, KC, RT, VEC>(A, m, k, lda, kfull, tnext, voff0, q, a_load);
    // all loads of this step are issued before any product: the scheduler
    // must not sink the prefetch below the products it is meant to overlap
    __builtin_amdgcn_sched_barrier(0);

    // B fragments small enough for registers may be hoisted out of the row
    // loop by the compiler; larger ones are re-read from LDS (or L2) every
    // step, which the opaque offset enforces.
    int bofs = 0;
    if constexpr (S * NT > 32) asm volatile("" : "+v"(bofs));

    acc_t acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[rt][tt] = acc_t{};
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
            const T b = Bsrc[bofs + (s * bstride + tt) * 64 + lane];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt][tt] = M::op(a_use[rt][s], b, acc[rt][tt]);
        }
    }

    // the epilogue (and its wait for C) follows the products
    __builtin_amdgcn_sched_barrier(0);

    // epilogue: lane (q, j) holds rows M::row(q, r) of columns colp(tt).
    // Without the C prefetch (CPRE false: variants whose registers are
    // spoken for), C is read here, and only when beta != 0.
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        if constexpr (PAIR) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const T lo = acc[rt][0][2 * p], hi = acc[rt][0][2 * p + 1];
                const T got = lane_pair_swap(odd ? lo : hi);
                const T c0 = odd ? got : lo, c1 = odd ? hi : got;  // columns j & ~1, j | 1
                typename M::vec v;
                v[0] = (T)epilogue(alpha, (double)c0, beta, (double)cp[rt][p][0]);
                v[1] = (T)epilogue(alpha, (double)c1, beta, (double)cp[rt][p][1]);
                BufIO<T>::template store_vec<SAUX>(v, rc[rt], poff(p));
            }
        } else if constexpr (cvec) {
#pragma unroll
            for (int g = 0; g < NT / PG; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if constexpr (!CPRE) {
                        const typename M::vec v = beta != 0.0 ? BufIO<T>::load_vec(rl[rt], voff(g, r))
                                                              : typename M::vec{};
#pragma unroll
                        for (int i = 0; i < PG; ++i) cv[rt][PG * g + i][r] = v[i];
                    }
                    typename M::vec v;
#pragma unroll
                    for (int i = 0; i < PG; ++i)
                        v[i] = (T)epilogue(alpha, (double)acc[rt][PG * g + i][r], beta, (double)cv[rt][PG * g + i][r]);
                    BufIO<T>::template store_vec<SAUX>(v, rc[rt], voff(g, r));
                }
        } else {
            // the column tiles of one row quad back to back: the parts of a
            // 128-byte line of C reach the cache together
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int tt = 0; tt < NT; ++tt) {
                    if constexpr (!CPRE) cv[rt][tt][r] = beta != 0.0 ? BufIO<T>::load1(rl[rt], coff(tt, r)) : (T)0;
                    BufIO<T>::store1((T)epilogue(alpha, (double)acc[rt][tt][r], beta, (double)cv[rt][tt][r]), rc[rt],
                                     coff(tt, r));
                }
        }
    }
}

// KC: packed k class; NT: 16-column tiles per workgroup (all of n, or one
// column group of it); RT: 16-row tiles per wavefront step; VEC: vector
// k-slot mapping.  nt_total is the number of column tiles of the packed B.
template <typename T, int KC, int NT, int RT, bool VEC, int CM>
__global__ __launch_bounds__(kStreamBlock) void k_stream(const T *__restrict__ A,
                                                          const T *__restrict__ Bf,
                                                          T *__restrict__ C, int64_t m, int n,
                                                          int k, int lda, int ldc, double alpha,
                                                          double beta, int nt_total, int nsplit) {
    typedef Mfma4<T> M;
    typedef typename M::vec vec_t;
    constexpr int VW = M::VW;
    constexpr int S = KC / 4;  // k-steps
    constexpr int FRAG = S * NT * 64;
    constexpr bool BLDS = FRAG * (int)sizeof(T) <= kStreamLdsBudget;
    static_assert(!VEC || (KC % (4 * VW)) == 0, "vector mapping needs KC % (4*VW) == 0");

    const BlockMap bm = block_map(nsplit);
    const int col0 = bm.group * NT * 16;

    __shared__ T sB[BLDS ? FRAG : 1];
    if constexpr (BLDS) {
        // this workgroup's column tiles of every k-step
        for (int idx = threadIdx.x * VW; idx < FRAG; idx += blockDim.x * VW) {
            const int s = idx / (NT * 64), rem = idx % (NT * 64);
            *reinterpret_cast<vec_t *>(&sB[idx]) =
                *reinterpret_cast<const vec_t *>(&Bf[(s * nt_total + bm.group * NT) * 64 + rem]);
        }
        __syncthreads();
    }

    const int lane = threadIdx.x & 63;
    const int j = lane & 15;
    const int q = lane >> 4;
    const int64_t ntile = (m + 15) >> 4;
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t gw = bm.rb * wpb + wave;
    const int64_t tstride = bm.nrb * wpb * RT;
    constexpr int SZ = (int)sizeof(T);

    // Per-lane byte offsets, fixed for the whole kernel.  Rows are addressed
    // through one buffer resource per 16-row tile sized to the rows of the
    // tile that exist, so rows beyond m read 0 and are not written; lanes
    // whose column lies beyond k (ragged k) or n get the offset kOOB, which
    // is outside every tile, instead of a branch.
    const bool kfull = k == KC;
    const int voff0 = j * lda * SZ;

    // Software pipeline, ping-pong over two register sets (the paper's
    // KERNEL_M1 / KERNEL_M2 alternation, Sec. IV-B.2): while one set feeds
    // this step's products, the next step's A rows stream into the other.
    T a0[RT][S], a1[RT][S];
    int64_t t = gw * RT;
    if (t >= ntile) return;
    stream_load_a<T, KC, RT, VEC>(A, m, k, lda, kfull, t, voff0, q, a0);
    const T *__restrict__ Bsrc = BLDS ? sB : Bf + bm.group * NT * 64;
    const int bstride = BLDS ? NT : nt_total;  // column tiles per k-step in Bsrc
    // Steps go in pairs with no branch between them (a branch would let the
    // compiler sink the prefetch past it); a pair's second step may lie past
    // the last tile, where its loads return 0 and its stores are dropped.
    for (; t < ntile; t += 2 * tstride) {
        stream_step<T, KC, NT, RT, VEC, CM>(A, Bsrc, bstride, C, m, n, k, lda, ldc, kfull, alpha, beta, col0, t,
                                            t + tstride, voff0, q, lane, j, a0, a1);
        stream_step<T, KC, NT, RT, VEC, CM>(A, Bsrc, bstride, C, m, n, k, lda, ldc, kfull, alpha, beta, col0,
                                            t + tstride,
                                            t + 2 * tstride, voff0, q, lane, j, a1, a0);
    }
}

template <typename T, int KC, int NT, int RT, bool VEC, int CM>
hipError_t run_stream(const void *A, const void *Bf, void *C, int64_t m, int64_t n, int64_t k, int64_t lda,
                      int64_t ldc, double alpha, double beta, int64_t grid, int block, int nt_total, int nsplit,
                      hipStream_t s) {
    hipLaunchKernelGGL((k_stream<T, KC, NT, RT, VEC, CM>), dim3((unsigned)grid), dim3(block), 0, s,
                       static_cast<const T *>(A), static_cast<const T *>(Bf), static_cast<T *>(C),
                       m, (int)n, (int)k, (int)lda, (int)ldc, alpha, beta, nt_total, nsplit);
    return hipGetLastError();
}

typedef hipError_t (*StreamFn)(const void *, const void *, void *, int64_t, int64_t, int64_t, int64_t, int64_t,
                               double, double, int64_t, int, int, int, hipStream_t);
struct StreamEntry {
    int KC, NT, RT, vec, cm;
    StreamFn fn;
};

}  // namespace tsmm

// Instantiation lists: every NT for RT = 1, NT <= 8 for RT = 2, NT <= 4 for
// RT = 4 (accumulators stay within 128 registers), NT <= 2 for RT = 8.
// TSMM_SE_* instantiate the plain column order; TSMM_SI, TSMM_SIS (scalar
// mapping) and TSMM_SEI*_* the interleaved order, where it applies
// (NT >= VW); TSMM_SP the binary64 lane pairs (NT = 1); TSMM_SID and
// TSMM_SPD the binary64 vector modes with default-policy C stores.
#define TSMM_SE(T, KC, NT, RT, V) {KC, NT, RT, V, 0, &tsmm::run_stream<T, KC, NT, RT, V, 0>},
#define TSMM_SI(T, KC, NT, RT) {KC, NT, RT, 1, 1, &tsmm::run_stream<T, KC, NT, RT, true, 1>},
#define TSMM_SIS(T, KC, NT, RT) {KC, NT, RT, 0, 1, &tsmm::run_stream<T, KC, NT, RT, false, 1>},
#define TSMM_SP(KC, RT, V) {KC, 1, RT, V, 2, &tsmm::run_stream<double, KC, 1, RT, V, 2>},
// the same two C modes with default-policy C stores (beta == 0)
#define TSMM_SID(KC, NT, RT) {KC, NT, RT, 1, 5, &tsmm::run_stream<double, KC, NT, RT, true, 5>},
#define TSMM_SPD(KC, RT) {KC, 1, RT, 1, 6, &tsmm::run_stream<double, KC, 1, RT, true, 6>},
#define TSMM_SE_RT1(T, KC, V) \
    TSMM_SE(T, KC, 1, 1, V) TSMM_SE(T, KC, 2, 1, V) TSMM_SE(T, KC, 4, 1, V) TSMM_SE(T, KC, 8, 1, V) TSMM_SE(T, KC, 16, 1, V)
#define TSMM_SE_RT2(T, KC, V) \
    TSMM_SE(T, KC, 1, 2, V) TSMM_SE(T, KC, 2, 2, V) TSMM_SE(T, KC, 4, 2, V) TSMM_SE(T, KC, 8, 2, V)
#define TSMM_SE_RT4(T, KC, V) TSMM_SE(T, KC, 1, 4, V) TSMM_SE(T, KC, 2, 4, V) TSMM_SE(T, KC, 4, 4, V)
#define TSMM_SE_RT8(T, KC, V) TSMM_SE(T, KC, 1, 8, V) TSMM_SE(T, KC, 2, 8, V)
#define TSMM_SE_ALL(T, KC, V) TSMM_SE_RT1(T, KC, V) TSMM_SE_RT2(T, KC, V) TSMM_SE_RT4(T, KC, V)
// interleaved: binary64 pairs (NT >= 2), binary32 quads (NT >= 4)
#define TSMM_SEI64_RT1(KC) TSMM_SI(double, KC, 2, 1) TSMM_SI(double, KC, 4, 1) TSMM_SI(double, KC, 8, 1) \
    TSMM_SI(double, KC, 16, 1)
#define TSMM_SEI64_RT2(KC) TSMM_SI(double, KC, 2, 2) TSMM_SI(double, KC, 4, 2) TSMM_SI(double, KC, 8, 2)
#define TSMM_SEI64_RT4(KC) TSMM_SI(double, KC, 2, 4) TSMM_SI(double, KC, 4, 4)
#define TSMM_SEI64_ALL(KC) TSMM_SEI64_RT1(KC) TSMM_SEI64_RT2(KC) TSMM_SEI64_RT4(KC)
#define TSMM_SEI32_RT1(KC) TSMM_SI(float, KC, 4, 1) TSMM_SI(float, KC, 8, 1) TSMM_SI(float, KC, 16, 1)
#define TSMM_SEI32_RT2(KC) TSMM_SI(float, KC, 4, 2) TSMM_SI(float, KC, 8, 2)
#define TSMM_SEI32_RT4(KC) TSMM_SI(float, KC, 4, 4)
#define TSMM_SEI32_ALL(KC) TSMM_SEI32_RT1(KC) TSMM_SEI32_RT2(KC) TSMM_SEI32_RT4(KC)
#define TSMM_SIS64_RT1(KC) TSMM_SIS(double, KC, 2, 1) TSMM_SIS(double, KC, 4, 1) TSMM_SIS(double, KC, 8, 1) \
    TSMM_SIS(double, KC, 16, 1)
#define TSMM_SIS32_RT1(KC) TSMM_SIS(float, KC, 4, 1) TSMM_SIS(float, KC, 8, 1) TSMM_SIS(float, KC, 16, 1)
