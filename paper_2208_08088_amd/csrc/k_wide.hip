// op N for binary32 A and C with n a multiple of 128 (n <= 256) and
// k <= 256: the "wide" kernels, built on the 32x32 matrix-core products
// V_MFMA_F32_32X32X2_F32 (binary32 products) and V_MFMA_F32_32X32X16_BF16
// (split-bf16 modes, 3 or 6 products per element pair as in k_bf16.h).
//
// Design.  At these shapes packed B (up to 384 KiB of bf16 planes) is
// larger than the LDS, and splitting n over workgroups (the streaming
// kernels' column groups) re-reads and re-splits A once per group.  Here
// one wavefront owns RT 32-row tiles across *all* n columns: its RT*NT
// 32x32 accumulators (256 registers at RT*NT = 16) live in the
// accumulation registers, A is loaded and split exactly once, and packed B
// streams through LDS in 32-k slabs that the workgroup's four wavefronts
// share.  Slabs are double-buffered and moved by the LDS-DMA loads
// (global_load_lds_dwordx4: lane l's 16 bytes land at base + 16*l, checked
// on the device), so the copy needs no registers; the next chunk's A and the
// next slab are in flight while the current chunk's products run.  One
// workgroup of four wavefronts per compute unit, persistent over row tiles.
//
// Fragment order (matrix-core lane layout established by an on-device
// probe): in both 32x32 products lane l = 32*q + j supplies A(row j, ...)
// and B(..., column j), and accumulator element r is row 8*(r/4) + 4*q +
// r%4, column j.  The k-slot -> column-of-A assignment is free; it is
// chosen so that each lane reads A as four 16-byte vectors per 32-k chunk:
// load h (0..3) of lane (q, j) holds A[row j][32c + 8h + 4q + u], u < 4.
//   binary32: k-step 4h + u uses slot q <-> column 32c + 8h + 4q + u;
//   bf16:     k-step s (16 wide) takes loads 2s and 2s+1 as its 8 values.
// Columns are permuted within 128-column groups: tile t, lane column j is
// B column 128*(t/4) + 4*j + t%4, so that a lane's accumulators of tiles
// 4g..4g+3 hold four adjacent columns of C and every C access is one
// 16-byte vector.  The packed image (tsmm_internal.h) holds per chunk c a
// slab of F*NT 1 KiB fragments.
#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

constexpr int kWideWaves = 4;

template <int MODE> struct WideCfg {
    static constexpr int TERMS = MODE == 0 ? 1 : (MODE == 3 ? 2 : 3);
    static constexpr int F = MODE == 0 ? 4 : 2 * TERMS;  // fragments per column tile per chunk
};

// Rows of the 32-row tile starting at row0 that exist in an m-row matrix.
__device__ __forceinline__ int64_t tile_rows32(int64_t m, int64_t row0) {
    const int64_t r = m - row0;
    return r < 0 ? 0 : (r > 32 ? 32 : r);
}

// The lane's four A vectors of chunk c for RT row tiles (rows past m and
// columns past k read 0).  The lane offset is made opaque so that the
// compiler recomputes the per-chunk offsets at each use instead of keeping
// all of them live across the tile loop.
template <int RT>
__device__ __forceinline__ void wide_load_a(const float *__restrict__ A, int64_t m, int k, int64_t row_base, int c,
                                            int j, int q, f4v (&x)[RT][4]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64(row_base + 32 * rt);
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + row0 * k, tile_rows32(m, row0) * (int64_t)k * 4);
        int vo = j * k * 4 + q * 16;
        asm volatile("" : "+v"(vo));
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int col = 32 * c + 8 * h;  // uniform part; k % 8 == 0
            x[rt][h] = __builtin_bit_cast(
                f4v, __builtin_amdgcn_raw_buffer_load_b128(ra, col < k ? vo + col * 4 : kOOB, 0, 0));
        }
    }
}

// This wavefront's share of slab c into LDS (LDS-DMA, 16 bytes per lane;
// the fragment offset is a scalar operand, always inside the image).
template <int SLAB>
__device__ __forceinline__ void wide_dma(__amdgpu_buffer_rsrc_t rw, int c, int wave, int lane, u32x4 *dst) {
    constexpr int PER = SLAB / kWideWaves;
    u32x4 *d = dst + wave * PER * 64;
    const int f0 = (c * SLAB + wave * PER) * 1024;
#pragma unroll
    for (int f = 0; f < PER; ++f)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (__attribute__((address_space(3))) void *)(d + f * 64), 16,
                                                 lane * 16, f0 + f * 1024, 0, 0);
}

// Residual split of the lane's 8 values of one bf16 k-step into TERMS
// bfloat16 vectors (round to nearest even at every step; each residual is
// exact in binary32).
template <int TERMS>
__device__ __forceinline__ void wide_split(const f4v &x0, const f4v &x1, u32x4 (&t)[TERMS]) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        f2v r = w < 2 ? f2v{x0[2 * w], x0[2 * w + 1]} : f2v{x1[2 * w - 4], x1[2 * w - 3]};
#pragma unroll
        for (int p = 0; p < TERMS; ++p) {
            const bf2v h = __builtin_convertvector(r, bf2v);
            t[p][w] = __builtin_bit_cast(uint32_t, h);
            if (p + 1 < TERMS) r = r - __builtin_convertvector(h, f2v);
        }
    }
}

__device__ __forceinline__ f16v mfma32_bf16(const u32x4 &a, const u32x4 &b, const f16v &c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0, 0,
                                                   0);
}

// Products of one 32-k chunk from slab `sb`.  The B fragments of step
// i + 1 are read from LDS before the products of step i, and scheduling
// barriers keep the compiler from hoisting further reads (which would only
// raise register pressure).
template <int MODE, int NT, int RT>
__device__ __forceinline__ void wide_chunk(const u32x4 *sb, const f4v (&x)[RT][4], f16v (&acc)[RT][NT], int lane) {
    constexpr int TP = NT / 2;  // pairs of column tiles
    if constexpr (MODE == 0) {
        // step i = h*TP + tp: rows h of the four k-vectors, tiles 2tp, 2tp+1
        constexpr int NS = 4 * TP;
        f4v b[2][2];
        auto rd = [&](int i, f4v (&d)[2]) {
            const int h = i / TP, tp = i % TP;
#pragma unroll
            for (int u = 0; u < 2; ++u) d[u] = __builtin_bit_cast(f4v, sb[(h * NT + 2 * tp + u) * 64 + lane]);
        };
        rd(0, b[0]);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (i + 1 < NS) rd(i + 1, b[(i + 1) & 1]);
            const int h = i / TP, tp = i % TP;
#pragma unroll
            for (int uu = 0; uu < 4; ++uu)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        acc[rt][2 * tp + u] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[rt][h][uu], b[i & 1][u][uu],
                                                                                   acc[rt][2 * tp + u], 0, 0, 0);
            // the next step's LDS reads go out ahead of this step's products
            if (i + 1 < NS) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 8 * RT, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        constexpr int TERMS = WideCfg<MODE>::TERMS;
        // products (A term, B term) of order <= 1 (3 products) or <= 2 (6)
        constexpr int NP = MODE;
        constexpr int PA[6] = {0, 0, 1, 0, 1, 2};
        constexpr int PB[6] = {0, 1, 0, 2, 1, 0};
        constexpr int NS = 2 * TP;  // step i = s*TP + tp
        u32x4 at[RT][2][TERMS];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int s = 0; s < 2; ++s) wide_split<TERMS>(x[rt][2 * s], x[rt][2 * s + 1], at[rt][s]);
        u32x4 b[2][2][TERMS];
        auto rd = [&](int i, u32x4 (&d)[2][TERMS]) {
            const int s = i / TP, tp = i % TP;
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int p = 0; p < TERMS; ++p) d[u][p] = sb[((s * TERMS + p) * NT + 2 * tp + u) * 64 + lane];
        };
        rd(0, b[0]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (i + 1 < NS) rd(i + 1, b[(i + 1) & 1]);
            const int s = i / TP, tp = i % TP;
#pragma unroll
            for (int pr = 0; pr < NP; ++pr)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        acc[rt][2 * tp + u] = mfma32_bf16(at[rt][s][PA[pr]], b[i & 1][u][PB[pr]], acc[rt][2 * tp + u]);
            if (i + 1 < NS) __builtin_amdgcn_sched_group_barrier(0x100, 2 * TERMS, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 2 * NP * RT, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// binary64 epilogue of the wavefront's RT x NT tiles, 16-byte C vectors.
template <int MODE, int NT, int RT>
__device__ __forceinline__ void wide_epilogue(const f16v (&acc)[RT][NT], const int (&ex)[NT / 4][4],
                                              float *__restrict__ C, int64_t m, int n, int64_t row_base,
                                              double alpha, double beta, int j, int q) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64(row_base + 32 * rt);
        const __amdgpu_buffer_rsrc_t rc = make_rsrc(C + row0 * n, tile_rows32(m, row0) * (int64_t)n * 4);
        int vo = (4 * q * n + 4 * j) * 4;  // row 4q, columns 4j.. of the tile (opaque, as in wide_load_a)
        asm volatile("" : "+v"(vo));
#pragma unroll
        for (int g = 0; g < NT / 4; ++g) {
            f4v cv[16];
            if (beta != 0.0) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    cv[r] = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(
                                                        rc, vo + ((8 * (r / 4) + r % 4) * n + 128 * g) * 4, 0, 2));
            } else {
#pragma unroll
                for (int r = 0; r < 16; ++r) cv[r] = f4v{};
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                f4v o;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    double s = (double)acc[rt][4 * g + i][r];
                    if constexpr (MODE != 0) s = __builtin_ldexp(s, ex[g][i]);
                    o[i] = (float)epilogue(alpha, s, beta, (double)cv[r][i]);
                }
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, o), rc,
                                                       vo + ((8 * (r / 4) + r % 4) * n + 128 * g) * 4, 0, 2);
            }
        }
    }
}

// MODE: 0 binary32 products, 3 or 6 split-bf16 products.  KC: packed k
// class (64, 128, 256); NT: 32-column tiles (n / 32); RT: 32-row tiles per
// wavefront.
template <int MODE, int KC, int NT, int RT>
__global__ __launch_bounds__(64 * kWideWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_wide(
    const float *__restrict__ A, const u32x4 *__restrict__ W, const int32_t *__restrict__ exps,
    float *__restrict__ C, int64_t m, int n, int k, double alpha, double beta) {
    constexpr int F = WideCfg<MODE>::F;
    constexpr int NCH = KC / 32;
    constexpr int SLAB = F * NT;
    constexpr int ROWS = kWideWaves * RT * 32;
    static_assert(NCH % 2 == 0 && SLAB % kWideWaves == 0 && NT % 4 == 0, "wide kernel shape");

    __shared__ u32x4 sb0[SLAB * 64];
    __shared__ u32x4 sb1[SLAB * 64];

    const int lane = threadIdx.x & 63;
    const int j = lane & 31;
    const int q = lane >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t ntile = (m + ROWS - 1) / ROWS;
    int64_t tile = blockIdx.x;
    if (tile >= ntile) return;
    const int64_t wrow = (int64_t)wave * RT * 32;

    int ex[NT / 4][4];
#pragma unroll
    for (int g = 0; g < NT / 4; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i) ex[g][i] = MODE != 0 ? exps[128 * g + 4 * j + i] : 0;

    const __amdgpu_buffer_rsrc_t rw = make_rsrc(W, (int64_t)NCH * SLAB * 1024);
    f4v xa[RT][4], xn[RT][4];
    wide_dma<SLAB>(rw, 0, wave, lane, sb0);
    wide_load_a<RT>(A, m, k, tile * ROWS + wrow, 0, j, q, xa);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();

    for (;;) {
        f16v acc[RT][NT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[rt][t] = f16v{};
        const int64_t next = tile + gridDim.x;
        // chunks in pairs: even chunks read sb0 and fill sb1, odd ones the
        // reverse; the chunk after the last is chunk 0 of the next tile (past
        // the last tile its A reads 0 and is never used)
#pragma unroll
        for (int c = 0; c < NCH; c += 2) {
            wide_dma<SLAB>(rw, c + 1, wave, lane, sb1);
            wide_load_a<RT>(A, m, k, tile * ROWS + wrow, c + 1, j, q, xn);
            wide_chunk<MODE, NT, RT>(sb0, xa, acc, lane);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // this wavefront's slab and A loads have landed
            __syncthreads();                     // ... and every wavefront's
            const bool last = c + 2 >= NCH;
            wide_dma<SLAB>(rw, last ? 0 : c + 2, wave, lane, sb0);
            wide_load_a<RT>(A, m, k, (last ? next : tile) * ROWS + wrow, last ? 0 : c + 2, j, q, xa);
            wide_chunk<MODE, NT, RT>(sb1, xn, acc, lane);
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();
        }
        wide_epilogue<MODE, NT, RT>(acc, ex, C, m, n, tile * ROWS + wrow, alpha, beta, j, q);
        tile = next;
        if (tile >= ntile) break;
    }
}

// Packed image of the wide kernels: for chunk c < KC/32, fragment f < F,
// tile t < NT and lane l = 32q + j, one 16-byte vector
//   binary32: f = h:        B[32c + 8h + 4q + u][col(t, j)], u < 4
//   split:    f = s*T + p:  plane p of B[32c + 16s + 8(e/4) + 4q + e%4][col(t, j)], e < 8
// with col(t, j) = 128*(t/4) + 4*j + t%4 and 0 outside k x n.
__global__ void k_pack_wide(const float *__restrict__ Bf32, const uint16_t *__restrict__ planes,
                            u32x4 *__restrict__ W, int64_t k, int64_t n, int KC, int NT, int terms) {
    const int F = terms == 0 ? 4 : 2 * terms;
    const int64_t total = (int64_t)(KC / 32) * F * NT * 64;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= total) return;
    const int lane = (int)(v % 64), frag = (int)((v / 64) % (F * NT));
    const int c = (int)(v / (64 * (int64_t)F * NT));
    const int f = frag / NT, t = frag % NT;
    const int q = lane >> 5, j = lane & 31;
    const int64_t col = 128 * (t / 4) + 4 * j + t % 4;
    u32x4 out = {0, 0, 0, 0};
    if (terms == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = 32 * c + 8 * f + 4 * q + u;
            const float x = (row < k && col < n) ? Bf32[row * n + col] : 0.0f;
            out[u] = __float_as_uint(x);
        }
    } else {
        const int s = f / terms, p = f % terms;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t row = 32 * c + 16 * s + 8 * (e / 4) + 4 * q + e % 4;
            const uint32_t h = (row < k && col < n) ? planes[(int64_t)p * k * n + row * n + col] : 0u;
            out[e / 2] |= h << (16 * (e % 2));
        }
    }
    W[v] = out;
}

size_t wide_image_bytes(int KC, int NT, int terms) {
    const int F = terms == 0 ? 4 : 2 * terms;
    return (size_t)(KC / 32) * F * NT * 1024;
}

hipError_t launch_pack_wide(const void *Bf32, const void *planes, void *W, int64_t k, int64_t n, int KC, int NT,
                            int terms, hipStream_t s) {
    const int64_t total = (int64_t)wide_image_bytes(KC, NT, terms) / 16;
    hipLaunchKernelGGL(k_pack_wide, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       static_cast<const float *>(Bf32), static_cast<const uint16_t *>(planes),
                       static_cast<u32x4 *>(W), k, n, KC, NT, terms);
    return hipGetLastError();
}

template <int MODE, int KC, int NT, int RT>
hipError_t run_wide(const float *A, const void *W, const int32_t *exps, float *C, int64_t m, int64_t n, int64_t k,
                    double alpha, double beta, int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL((k_wide<MODE, KC, NT, RT>), dim3((unsigned)grid), dim3(64 * kWideWaves), 0, s, A,
                       static_cast<const u32x4 *>(W), exps, C, m, (int)n, (int)k, alpha, beta);
    return hipGetLastError();
}

typedef hipError_t (*WideFn)(const float *, const void *, const int32_t *, float *, int64_t, int64_t, int64_t,
                             double, double, int64_t, hipStream_t);
struct WideEntry {
    int mode, KC, NT, RT;
    WideFn fn;
};

#define TSMM_WE(M, KC, NT, RT) {M, KC, NT, RT, &run_wide<M, KC, NT, RT>},
#define TSMM_WE_KC(M, NT, RT) TSMM_WE(M, 64, NT, RT) TSMM_WE(M, 128, NT, RT) TSMM_WE(M, 256, NT, RT)
#define TSMM_WE_M(M) TSMM_WE_KC(M, 8, 2) TSMM_WE_KC(M, 4, 2) TSMM_WE_KC(M, 4, 4)

static const WideEntry kWideTable[] = {TSMM_WE_M(0) TSMM_WE_M(3) TSMM_WE_M(6)};

static WideFn find_wide(int mode, int KC, int NT, int RT) {
    for (const WideEntry &e : kWideTable)
        if (e.mode == mode && e.KC == KC && e.NT == NT && e.RT == RT) return e.fn;
    return nullptr;
}

bool wide_variant_exists(int products, int KC, int NT, int RT) { return find_wide(products, KC, NT, RT) != nullptr; }

int64_t wide_rows_per_wg(int RT) { return (int64_t)kWideWaves * RT * 32; }

hipError_t launch_wide(int products, int KC, int NT, int RT, const void *A, const void *W, const int32_t *exps,
                       void *C, int64_t m, int64_t n, int64_t k, double alpha, double beta, int64_t grid,
                       hipStream_t s) {
    WideFn fn = find_wide(products, KC, NT, RT);
    if (!fn || n != 32 * NT || k > KC || k % 8 != 0 || grid < 1) return hipErrorInvalidValue;
    return fn(static_cast<const float *>(A), W, exps, static_cast<float *>(C), m, n, k, alpha, beta, grid, s);
}

}  // namespace tsmm
