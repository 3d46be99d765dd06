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

// A rows of row tiles t .. t+RT-1 into registers: one buffer resource per
// 16-row tile (its byte count ends at row m, so rows beyond m read 0);
// kmask bit p (or s) says whether this lane's columns are inside k.
template <typename T, int KC, int RT, bool VEC>
__device__ __forceinline__ void stream_load_a(const T *__restrict__ A, int64_t m, int k, int64_t t, int voffA,
                                              uint32_t kmask, T (&a)[RT][KC / 4]) {
    typedef typename Mfma4<T>::vec vec_t;
    constexpr int VW = Mfma4<T>::VW;
    constexpr int S = KC / 4;
    constexpr int SZ = (int)sizeof(T);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64((t + rt) * 16);
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + row0 * k, (m - row0) * (int64_t)k * SZ);
        if constexpr (VEC) {
#pragma unroll
            for (int p = 0; p < S / VW; ++p) {
                vec_t v = {};
                if (kmask & (1u << p)) v = BufIO<T>::load_vec(ra, voffA + p * 4 * VW * SZ);
#pragma unroll
                for (int e = 0; e < VW; ++e) a[rt][p * VW + e] = v[e];
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) a[rt][s] = (kmask & (1u << s)) ? BufIO<T>::load1(ra, voffA + 4 * s * SZ) : T(0);
        }
    }
}

// KC: packed k class; NT: 16-column tiles per workgroup (all of n, or one
// column group of it); RT: 16-row tiles per wavefront step; VEC: vector
// k-slot mapping.  nt_total is the number of column tiles of the packed B.
template <typename T, int KC, int NT, int RT, bool VEC>
__global__ __launch_bounds__(kStreamBlock) void k_stream(const T *__restrict__ A,
                                                          const T *__restrict__ Bf,
                                                          T *__restrict__ C, int64_t m, int n,
                                                          int k, double alpha, double beta,
                                                          int nt_total, int nsplit) {
    typedef Mfma4<T> M;
    typedef typename M::acc acc_t;
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
    // through one buffer resource per 16-row tile whose byte count ends at
    // the last row of the matrix, so rows beyond m read 0 and are not
    // written; columns beyond k (ragged k) and beyond n are masked here.
    const int voffA = VEC ? (j * k + q * VW) * SZ : (j * k + q) * SZ;
    int voffC[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) voffC[r] = (M::row(q, r) * n + j) * SZ;
    const bool kfull = k == KC;
    uint32_t kmask = 0;  // bit s (or p): this lane's A column is inside k
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int col = VEC ? (s / VW) * 4 * VW + q * VW : 4 * s + q;
        if (kfull || col < k) kmask |= 1u << (VEC ? s / VW : s);
    }
    uint32_t nmask = 0;
#pragma unroll
    for (int t = 0; t < NT; ++t)
        if (col0 + 16 * t + j < n) nmask |= 1u << t;

    // Software pipeline: the A rows of the next step are in flight while
    // this step's products and epilogue run; this step's C rows (beta != 0)
    // are requested before the next A rows, so waiting for them does not
    // wait for the prefetch.
    T a_cur[RT][S], a_nxt[RT][S];
    int64_t t0 = gw * RT;
    if (t0 < ntile) stream_load_a<T, KC, RT, VEC>(A, m, k, t0, voffA, kmask, a_cur);
    for (; t0 < ntile; t0 += tstride) {
        __amdgpu_buffer_rsrc_t rc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t row0 = uniform64((t0 + rt) * 16);
            rc[rt] = make_rsrc(C + row0 * n + col0, ((m - row0) * (int64_t)n - col0) * SZ);
        }
        T cv[RT][NT][4];
        if (beta != 0.0) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        cv[rt][t][r] = (nmask & (1u << t)) ? BufIO<T>::load1(rc[rt], voffC[r] + 16 * t * SZ) : T(0);
        }
        const int64_t t1 = t0 + tstride;
        if (t1 < ntile) stream_load_a<T, KC, RT, VEC>(A, m, k, t1, voffA, kmask, a_nxt);

        // B fragments small enough for registers may be hoisted out of the
        // row loop by the compiler; larger ones are re-read from LDS (or L2)
        // for every row step, which the opaque offset enforces.
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
                const T b = BLDS ? sB[bofs + (s * NT + t) * 64 + lane]
                                 : Bf[bofs + (s * nt_total + bm.group * NT + t) * 64 + lane];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt][t] = M::op(a_cur[rt][s], b, acc[rt][t]);
            }
        }

        // epilogue: lane (q, j) holds rows M::row(q, r) of column 16t + j
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (nmask & (1u << t)) {
                        const double c = beta != 0.0 ? (double)cv[rt][t][r] : 0.0;
                        BufIO<T>::store1((T)epilogue(alpha, (double)acc[rt][t][r], beta, c), rc[rt],
                                         voffC[r] + 16 * t * SZ);
                    }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int s = 0; s < S; ++s) a_cur[rt][s] = a_nxt[rt][s];
    }
}

template <typename T, int KC, int NT, int RT, bool VEC>
hipError_t run_stream(const void *A, const void *Bf, void *C, int64_t m, int64_t n, int64_t k,
                      double alpha, double beta, int64_t grid, int block, int nt_total, int nsplit,
                      hipStream_t s) {
    hipLaunchKernelGGL((k_stream<T, KC, NT, RT, VEC>), dim3((unsigned)grid), dim3(block), 0, s,
                       static_cast<const T *>(A), static_cast<const T *>(Bf), static_cast<T *>(C),
                       m, (int)n, (int)k, alpha, beta, nt_total, nsplit);
    return hipGetLastError();
}

typedef hipError_t (*StreamFn)(const void *, const void *, void *, int64_t, int64_t, int64_t,
                               double, double, int64_t, int, int, int, hipStream_t);
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
#define TSMM_SE_RT8(T, KC, V) TSMM_SE(T, KC, 1, 8, V) TSMM_SE(T, KC, 2, 8, V)
#define TSMM_SE_ALL(T, KC, V) TSMM_SE_RT1(T, KC, V) TSMM_SE_RT2(T, KC, V) TSMM_SE_RT4(T, KC, V)
