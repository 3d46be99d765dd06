// op N with a long shared dimension: C = alpha*A*B + beta*C for a row-major
// A (m x k) whose k is beyond the streaming kernels' packed classes, and a
// packed B (k x n, n <= 256), binary64 or binary32.  This is the paper's
// own workload shape (Sec. V: square A times a tall-and-skinny B), where B
// no longer fits any on-chip store.
//
// Design.  The paper blocks k into k_c slabs so that one slab of packed B
// stays resident in a core's cache while a block of A rows streams past it
// (Sec. IV-A, Eqs. (2)-(3)).  Here a workgroup of four wavefronts owns a
// block of 4*RT row tiles (16 rows each) and ALL n columns: each wavefront
// keeps the RT x NT accumulators of its row tiles in registers for the
// whole k range, and packed B streams through LDS in slabs of 32 k (one
// slab = 8 k-steps x NT fragments), double-buffered and moved by LDS-DMA
// loads that the four wavefronts share.  A rows are read from HBM exactly
// once, straight into registers, one slab ahead.
//
// When the row blocks alone would leave compute units idle, the k range is
// cut into `splitk` contiguous parts: work item (part, row block) writes
// its binary64 partial sums to a workspace in fragment order, and a second
// pass adds the parts in ascending order and applies the binary64 epilogue
// (bitwise repeatable for a given plan).  Items go part-major, so the
// workgroups that run together read the same slabs of B through the L2.
#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

constexpr int kSlabWaves = 4;
constexpr int kSlabSteps = kSlabK / 4;  // 16x16x4 k-steps per slab (kSlabK: tsmm_internal.h)

// This wavefront's share of slab sl of the packed image (NT fragments of
// 64 lanes per k-step, kSlabSteps k-steps) into LDS: 1 KiB per LDS-DMA
// load (lane l's 16 bytes land at base + 16*l).  A slab of fewer than four
// pieces is moved by the first wavefronts, one piece each.
template <typename T, int NT>
__device__ __forceinline__ void slab_dma(__amdgpu_buffer_rsrc_t rb, int64_t sl, int wave, int lane, u32x4 *dst) {
    constexpr int BYTES = kSlabSteps * NT * 64 * (int)sizeof(T);
    constexpr int PIECES = BYTES / 1024;
    static_assert(PIECES * 1024 == BYTES && (PIECES % kSlabWaves == 0 || PIECES < kSlabWaves),
                  "slab must split into whole 1 KiB pieces");
    constexpr int PER = PIECES >= kSlabWaves ? PIECES / kSlabWaves : 1;
    if (PIECES < kSlabWaves && wave >= PIECES) return;
    u32x4 *d = dst + wave * PER * 64;
    // the image offset of a slab stays below 2^32 bytes (checked on the host)
    const int f0 = (int)(sl * BYTES) + wave * PER * 1024;
#pragma unroll
    for (int f = 0; f < PER; ++f)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (__attribute__((address_space(3))) void *)(d + f * 64), 16,
                                                 lane * 16, f0 + f * 1024, 0, 0);
}

// A of row tiles tile0 .. tile0+RT-1 for the kSlabSteps k-steps of slab sl
// (columns past k and rows past m read 0).  The k-slot mapping is the one
// the packed fragments use (tsmm_internal.h): with VEC, load p of lane q
// holds columns 32*sl + 4*VW*p + VW*q + e, e < VW, for k-steps VW*p + e.
template <typename T, int RT, bool VEC>
__device__ __forceinline__ void slab_load_a(const T *__restrict__ A, int64_t m, int k, int lda, int64_t tile0,
                                            int64_t sl, int j, int q, T (&a)[RT][kSlabSteps]) {
    typedef typename Mfma4<T>::vec vec_t;
    constexpr int VW = Mfma4<T>::VW;
    constexpr int SZ = (int)sizeof(T);
    const int cbase = (int)(sl * kSlabK);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64((tile0 + rt) * 16);
        // (rows - 1) * lda + k elements, negative (empty) when no row exists
        const int rows = (int)tile_rows(m, row0);
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + row0 * lda, (int64_t)(rows * lda - (lda - k)) * SZ);
        // rows of a slab are 128 / 256 bytes read by two or four loads, which
        // share each line through the cache (default policy)
        int vo = j * lda * SZ;
        asm volatile("" : "+v"(vo));
        if constexpr (VEC) {
#pragma unroll
            for (int p = 0; p < kSlabSteps / VW; ++p) {
                const int col = cbase + p * 4 * VW + q * VW;
                const vec_t v = BufIO<T>::template load_vec<0>(ra, col < k ? vo + col * SZ : kOOB);
#pragma unroll
                for (int e = 0; e < VW; ++e) a[rt][p * VW + e] = v[e];
            }
        } else {
#pragma unroll
            for (int s = 0; s < kSlabSteps; ++s) {
                const int col = cbase + 4 * s + q;
                a[rt][s] = BufIO<T>::template load1<0>(ra, col < k ? vo + col * SZ : kOOB);
            }
        }
    }
}

// The products of one slab: NT fragments of B per k-step from LDS, RT*NT
// matrix-core products.  The fragments of k-step s + 1 are read into the
// second register set while the products of step s run, one read between
// every RT products (with one wavefront per SIMD nothing else hides the
// LDS latency).
template <typename T, int NT, int RT>
__device__ __forceinline__ void slab_products(const T *__restrict__ sb, const T (&a)[RT][kSlabSteps],
                                              typename Mfma4<T>::acc (&acc)[RT][NT], int lane) {
    T b[2][NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) b[0][t] = sb[t * 64 + lane];
#pragma unroll
    for (int s = 0; s < kSlabSteps; ++s) {
        const int c = s & 1;
        if (s + 1 < kSlabSteps) {
#pragma unroll
            for (int t = 0; t < NT; ++t) b[c ^ 1][t] = sb[((s + 1) * NT + t) * 64 + lane];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt][t] = Mfma4<T>::op(a[rt][s], b[c][t], acc[rt][t]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (s + 1 < kSlabSteps) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, RT, 0);                        // RT products
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// NT: column tiles of the packed image (all of n); RT: 16-row tiles per
// wavefront; VEC: vector k-slot mapping; IL: interleaved column order
// (16-byte C vectors).  nsl: slabs in the packed image; nrb: row blocks;
// items = nrb * splitk.
template <typename T, int NT, int RT, bool VEC, bool IL>
__global__ __launch_bounds__(64 * kSlabWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_slab(
    const T *__restrict__ A, const T *__restrict__ Bf, T *__restrict__ C, double *__restrict__ W, int64_t m, int n,
    int k, int lda, int ldc, int64_t nsl, double alpha, double beta, int splitk, int64_t nrb) {
    typedef Mfma4<T> M;
    typedef typename M::acc acc_t;
    constexpr int SZ = (int)sizeof(T);
    constexpr int SLAB_ELEMS = kSlabSteps * NT * 64;
    __shared__ u32x4 sb0[SLAB_ELEMS * SZ / 16];
    __shared__ u32x4 sb1[SLAB_ELEMS * SZ / 16];

    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t items = nrb * splitk;
    const int64_t ntile = (m + 15) >> 4;
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(Bf, nsl * SLAB_ELEMS * SZ);

    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int part = (int)(item / nrb);
        const int64_t blk = item % nrb;
        const int64_t sl0 = nsl * part / splitk, sl1 = nsl * (part + 1) / splitk;
        const int64_t tile0 = (blk * kSlabWaves + wave) * RT;

        acc_t acc[RT][NT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[rt][t] = acc_t{};

        // every wavefront has finished with both slab buffers (previous item)
        __syncthreads();
        T a0[RT][kSlabSteps], a1[RT][kSlabSteps];
        slab_dma<T, NT>(rb, sl0, wave, lane, sb0);
        slab_load_a<T, RT, VEC>(A, m, k, lda, tile0, sl0, j, q, a0);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's share of the slab and its A
        __syncthreads();                     // every share has landed
        // slabs go in pairs over the two buffers; the pair's second slab may
        // lie past sl1, where nothing is loaded and nothing is multiplied
        for (int64_t sl = sl0; sl < sl1; sl += 2) {
            const bool two = sl + 1 < sl1;
            if (two) {
                slab_dma<T, NT>(rb, sl + 1, wave, lane, sb1);
                slab_load_a<T, RT, VEC>(A, m, k, lda, tile0, sl + 1, j, q, a1);
            }
            slab_products<T, NT, RT>(reinterpret_cast<const T *>(sb0), a0, acc, lane);
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();  // slab sl+1 in LDS; every wavefront is done with slab sl
            if (!two) break;
            if (sl + 2 < sl1) {
                slab_dma<T, NT>(rb, sl + 2, wave, lane, sb0);
                slab_load_a<T, RT, VEC>(A, m, k, lda, tile0, sl + 2, j, q, a0);
            }
            slab_products<T, NT, RT>(reinterpret_cast<const T *>(sb1), a1, acc, lane);
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();
        }

        if (splitk > 1) {
            // binary64 partials in fragment order: W[part][tile][t][lane][r]
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int64_t tile = tile0 + rt;
                if (tile >= ntile) break;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    d4v v;
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = (double)acc[rt][t][r];
                    d4v *dst = reinterpret_cast<d4v *>(W) + ((part * ntile + tile) * NT + t) * 64 + lane;
                    __builtin_nontemporal_store(v, dst);
                }
            }
            continue;
        }

        // direct epilogue: lane (q, j) holds rows M::row(q, r) of columns
        // colp(t); C rows through a resource per row tile (rows past m are
        // dropped), columns past n through kOOB
        constexpr int PG = IL ? M::VW : 1;
        static_assert(!IL || NT % PG == 0, "interleave groups must be whole");
        auto colp = [=](int t) { return 16 * PG * (t / PG) + PG * j + t % PG; };
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t row0 = uniform64((tile0 + rt) * 16);
            const int rows = (int)tile_rows(m, row0);
            const int64_t bytes = (int64_t)(rows * ldc - (ldc - n)) * SZ;
            const __amdgpu_buffer_rsrc_t rc = make_rsrc(C + row0 * ldc, bytes);
            const __amdgpu_buffer_rsrc_t rl = make_rsrc(C + row0 * ldc, beta != 0.0 ? bytes : 0);
            if constexpr (IL) {
#pragma unroll
                for (int g = 0; g < NT / PG; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int off = colp(PG * g) < n ? (M::row(q, r) * ldc + colp(PG * g)) * SZ : kOOB;
                        const typename M::vec c = BufIO<T>::load_vec(rl, off);
                        typename M::vec v;
#pragma unroll
                        for (int i = 0; i < PG; ++i)
                            v[i] = (T)epilogue(alpha, (double)acc[rt][PG * g + i][r], beta, (double)c[i]);
                        BufIO<T>::store_vec(v, rc, off);
                    }
            } else {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int off = colp(t) < n ? (M::row(q, r) * ldc + colp(t)) * SZ : kOOB;
                        const T c = BufIO<T>::load1(rl, off);
                        BufIO<T>::store1((T)epilogue(alpha, (double)acc[rt][t][r], beta, (double)c), rc, off);
                    }
            }
        }
    }
}

// Second pass: C = alpha * (W[0] + W[1] + ... + W[splitk-1]) + beta * C,
// parts added in ascending order in binary64; one thread per (row tile,
// column tile, lane), four accumulator rows each.
template <typename T>
__global__ __launch_bounds__(256) void k_slab_reduce(const double *__restrict__ W, T *__restrict__ C, int64_t m,
                                                     int n, int ldc, int NT, int pg, int splitk, double alpha,
                                                     double beta) {
    typedef Mfma4<T> M;
    const int64_t ntile = (m + 15) >> 4;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ntile * NT * 64) return;
    const int lane = (int)(idx & 63), j = lane & 15, q = lane >> 4;
    const int t = (int)((idx >> 6) % NT);
    const int64_t tile = (idx >> 6) / NT;
    const int col = 16 * pg * (t / pg) + pg * j + t % pg;
    if (col >= n) return;
    const d4v *w = reinterpret_cast<const d4v *>(W);
    const int64_t stride = ntile * NT * 64;
    d4v s = __builtin_nontemporal_load(w + idx);
    for (int p = 1; p < splitk; ++p) {
        s = s + __builtin_nontemporal_load(w + p * stride + idx);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = tile * 16 + M::row(q, r);
        if (row >= m) continue;
        T *c = C + row * ldc + col;
        *c = (T)epilogue(alpha, s[r], beta, beta != 0.0 ? (double)*c : 0.0);
    }
}

template <typename T, int NT, int RT, bool VEC, bool IL>
hipError_t run_slab(const void *A, const void *Bf, void *C, double *W, int64_t m, int64_t n, int64_t k, int64_t lda,
                    int64_t ldc, int64_t nsl, double alpha, double beta, int splitk, int64_t nrb, int64_t grid,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_slab<T, NT, RT, VEC, IL>), dim3((unsigned)grid), dim3(64 * kSlabWaves), 0, s,
                       static_cast<const T *>(A), static_cast<const T *>(Bf), static_cast<T *>(C), W, m, (int)n,
                       (int)k, (int)lda, (int)ldc, nsl, alpha, beta, splitk, nrb);
    return hipGetLastError();
}

typedef hipError_t (*SlabFn)(const void *, const void *, void *, double *, int64_t, int64_t, int64_t, int64_t,
                             int64_t, int64_t, double, double, int, int64_t, int64_t, hipStream_t);
struct SlabEntry {
    tsmm_dtype dt;
    int NT, RT, vec, il;
    SlabFn fn;
};

#define TSMM_SLAB(T, DT, NT, RT)                                        \
    {DT, NT, RT, 0, 0, &run_slab<T, NT, RT, false, false>},             \
    {DT, NT, RT, 1, 0, &run_slab<T, NT, RT, true, false>},              \
    {DT, NT, RT, 0, 1, &run_slab<T, NT, RT, false, true>},              \
    {DT, NT, RT, 1, 1, &run_slab<T, NT, RT, true, true>},
// fewer column tiles than one interleave group: plain order only
#define TSMM_SLAB_PLAIN(T, DT, NT, RT)                                  \
    {DT, NT, RT, 0, 0, &run_slab<T, NT, RT, false, false>},             \
    {DT, NT, RT, 1, 0, &run_slab<T, NT, RT, true, false>},

// Accumulators (RT * NT tiles of 8 binary64 / 4 binary32 registers) plus
// the two A register sets (RT * 8 values each) within about 200 registers:
// larger products spilled to scratch when compiled.
static const SlabEntry kSlabTable[] = {
    TSMM_SLAB(double, TSMM_F64, 16, 1) TSMM_SLAB(double, TSMM_F64, 8, 2) TSMM_SLAB(double, TSMM_F64, 4, 2)
    TSMM_SLAB(double, TSMM_F64, 2, 4) TSMM_SLAB_PLAIN(double, TSMM_F64, 1, 4)
    TSMM_SLAB(float, TSMM_F32, 16, 2) TSMM_SLAB(float, TSMM_F32, 8, 4) TSMM_SLAB(float, TSMM_F32, 4, 4)
    TSMM_SLAB_PLAIN(float, TSMM_F32, 2, 4) TSMM_SLAB_PLAIN(float, TSMM_F32, 1, 4)
};
#undef TSMM_SLAB
#undef TSMM_SLAB_PLAIN

static const SlabEntry *find_slab(tsmm_dtype dt, int NT, int RT, bool vec, bool il) {
    for (const SlabEntry &e : kSlabTable)
        if (e.dt == dt && e.NT == NT && e.RT == RT && e.vec == (int)vec && e.il == (int)il) return &e;
    return nullptr;
}

bool slab_variant_exists(tsmm_dtype dt, int NT, int RT, bool vec, bool il) {
    return find_slab(dt, NT, RT, vec, il) != nullptr;
}

int slab_rows(int RT) { return kSlabWaves * RT * 16; }

hipError_t launch_slab(tsmm_dtype dt, int NT, int RT, bool vec, bool il, const void *A, const void *Bf, void *C,
                       double *W, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldc, int KCimg, double alpha,
                       double beta, int splitk, int64_t grid, hipStream_t s) {
    const SlabEntry *e = find_slab(dt, NT, RT, vec, il);
    if (!e || KCimg % kSlabK != 0 || splitk < 1 || (splitk > 1 && !W)) return hipErrorInvalidValue;
    const int64_t nsl = KCimg / kSlabK;
    // LDS-DMA offsets are 32-bit: the image must stay below 4 GiB
    if ((int64_t)KCimg / 4 * NT * 64 * (dt == TSMM_F64 ? 8 : 4) >= ((int64_t)1 << 32)) return hipErrorInvalidValue;
    const int64_t nrb = (m + slab_rows(RT) - 1) / slab_rows(RT);
    hipError_t err = e->fn(A, Bf, C, W, m, n, k, lda, ldc, nsl, alpha, beta, splitk, nrb, grid, s);
    if (err != hipSuccess || splitk == 1) return err;
    const int64_t threads = ((m + 15) >> 4) * NT * 64;
    const int pg = il ? 16 / (dt == TSMM_F64 ? 8 : 4) : 1;
    if (dt == TSMM_F64)
        hipLaunchKernelGGL(k_slab_reduce<double>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, W,
                           static_cast<double *>(C), m, (int)n, (int)ldc, NT, pg, splitk, alpha, beta);
    else
        hipLaunchKernelGGL(k_slab_reduce<float>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, W,
                           static_cast<float *>(C), m, (int)n, (int)ldc, NT, pg, splitk, alpha, beta);
    return hipGetLastError();
}

}  // namespace tsmm
