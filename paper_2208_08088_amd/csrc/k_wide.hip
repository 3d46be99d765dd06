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
// workgroup per compute unit, persistent over row tiles, of four wavefronts
// (one per SIMD, RT = 2 or 4) or eight (two per SIMD, RT = 1, 128
// accumulation registers each).
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

template <int MODE> struct WideCfg {
    static constexpr int TERMS = MODE == 0 ? 1 : (MODE == 3 ? 2 : 3);
    static constexpr int F = MODE == 0 ? 4 : 2 * TERMS;  // fragments per column tile per chunk
};

// Rows of the 32-row tile starting at row0 that exist in an m-row matrix.
__device__ __forceinline__ int64_t tile_rows32(int64_t m, int64_t row0) {
    const int64_t r = m - row0;
    return r < 0 ? 0 : (r > 32 ? 32 : r);
}

// The lane's A vectors h0 <= h < h1 of chunk c for RT row tiles (rows past
// m and columns past k read 0).  One load instruction covers 32 bytes of
// each of 32 rows, so the loads keep the default cache policy: the four
// loads of a chunk then share each 128-byte line (streaming loads were
// measured to refetch it).  The lane offset is made opaque so that the
// compiler recomputes the per-chunk offsets at each use instead of keeping
// all of them live across the tile loop.
template <int RT, int H0, int H1>
__device__ __forceinline__ void wide_load_a(const float *__restrict__ A, int64_t m, int k, int64_t row_base, int c,
                                            int j, int q, f4v (&x)[RT][4]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64(row_base + 32 * rt);
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + row0 * k, tile_rows32(m, row0) * (int64_t)k * 4);
        int vo = j * k * 4 + q * 16;
        asm volatile("" : "+v"(vo));
#pragma unroll
        for (int h = H0; h < H1; ++h) {
            const int col = 32 * c + 8 * h;  // uniform part; k % 8 == 0
            x[rt][h] = __builtin_bit_cast(
                f4v, __builtin_amdgcn_raw_buffer_load_b128(ra, col < k ? vo + col * 4 : kOOB, 0, 0));
        }
    }
}

// This wavefront's share of slab c into LDS (LDS-DMA, 16 bytes per lane;
// the fragment offset is a scalar operand, always inside the image); WV
// wavefronts share the slab.
template <int SLAB, int WV>
__device__ __forceinline__ void wide_dma(__amdgpu_buffer_rsrc_t rw, int c, int wave, int lane, u32x4 *dst) {
    constexpr int PER = SLAB / WV;
    u32x4 *d = dst + wave * PER * 64;
    const int f0 = (c * SLAB + wave * PER) * 1024;
#pragma unroll
    for (int f = 0; f < PER; ++f)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (__attribute__((address_space(3))) void *)(d + f * 64), 16,
                                                 lane * 16, f0 + f * 1024, 0, 0);
}

// Residual split of one pair (word w of a bf16 k-step: values 2w, 2w+1 of
// the 8 that the vectors xs[0], xs[1] hold) into TERMS bfloat16 pairs
// (round to nearest even at every step; each residual is exact in
// binary32).
template <int TERMS>
__device__ __forceinline__ void wide_split_pair(const f4v &xa, const f4v &xb, int w, u32x4 (&t)[TERMS]) {
    f2v r = w < 2 ? f2v{xa[2 * w], xa[2 * w + 1]} : f2v{xb[2 * w - 4], xb[2 * w - 3]};
#pragma unroll
    for (int p = 0; p < TERMS; ++p) {
        const bf2v h = __builtin_convertvector(r, bf2v);
        t[p][w] = __builtin_bit_cast(uint32_t, h);
        if (p + 1 < TERMS) r = r - __builtin_convertvector(h, f2v);
    }
}

__device__ __forceinline__ f16v mfma32_bf16(const u32x4 &a, const u32x4 &b, const f16v &c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0, 0,
                                                   0);
}

// Interleave hints for one step: the next step's LDS reads first, then
// matrix-core products with one vector-ALU instruction (split work) after
// each, so that the split runs in the shadow of the products.
template <int NDS, int NMFMA, bool VALU>
__device__ __forceinline__ void wide_step_schedule() {
    if constexpr (NDS > 0) __builtin_amdgcn_sched_group_barrier(0x100, NDS, 0);
#pragma unroll
    for (int z = 0; z < NMFMA; ++z) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if constexpr (VALU) __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Binary32 products of one 32-k chunk from slab `sb` (four k-vectors per
// row tile; step i = h*TP + tp covers vector h and column tiles 2tp, 2tp+1).
// The B fragments of step i + 1 are read from LDS before the products of
// step i.
template <int NT, int RT>
__device__ __forceinline__ void wide_chunk_f32(const u32x4 *sb, const f4v (&x)[RT][4], f16v (&acc)[RT][NT],
                                               int lane) {
    constexpr int TP = NT / 2;
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
        if (i + 1 < NS) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 8 * RT, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Split-bf16 products of one half chunk (bf16 k-step s of chunk c) from
// slab `sb`, with the A terms `at` of that k-step.  Interleaved with the
// products, the half splits the next k-step's values (xs[.][0..1], the two
// vectors of one bf16 k-step) into `an`: in the first half the second
// k-step of this chunk, in the second half the first k-step of the next
// chunk.  The B fragments of the next step (of this half or the next) are
// read one step ahead through `b`.
template <int MODE, int NT, int RT>
__device__ __forceinline__ void wide_half_split(const u32x4 *sb, int s, bool prefetch_next_half,
                                                const u32x4 (&at)[RT][WideCfg<MODE>::TERMS], const f4v (&xs0)[RT],
                                                const f4v (&xs1)[RT], u32x4 (&an)[RT][WideCfg<MODE>::TERMS],
                                                u32x4 (&b)[2][2][WideCfg<MODE>::TERMS], f16v (&acc)[RT][NT],
                                                int lane) {
    constexpr int TERMS = WideCfg<MODE>::TERMS;
    constexpr int NP = MODE;  // products (A term, B term) of order <= 1 (3) or <= 2 (6)
    constexpr int PA[6] = {0, 0, 1, 0, 1, 2};
    constexpr int PB[6] = {0, 1, 0, 2, 1, 0};
    constexpr int TP = NT / 2;
    constexpr int WPS = 4 / TP;  // split pairs per step (4 pairs per k-step)
    auto rd = [&](int s2, int tp, u32x4 (&d)[2][TERMS]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int p = 0; p < TERMS; ++p) d[u][p] = sb[((s2 * TERMS + p) * NT + 2 * tp + u) * 64 + lane];
    };
#pragma unroll
    for (int tp = 0; tp < TP; ++tp) {
        // b[tp & 1] holds this step's fragments (read in the step before)
        const bool more = tp + 1 < TP || prefetch_next_half;
        if (tp + 1 < TP) rd(s, tp + 1, b[(tp + 1) & 1]);
        else if (prefetch_next_half) rd(s + 1, 0, b[(tp + 1) & 1]);
#pragma unroll
        for (int pr = 0; pr < NP; ++pr)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    acc[rt][2 * tp + u] = mfma32_bf16(at[rt][PA[pr]], b[tp & 1][u][PB[pr]], acc[rt][2 * tp + u]);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int w = tp * WPS; w < (tp + 1) * WPS; ++w) wide_split_pair<TERMS>(xs0[rt], xs1[rt], w, an[rt]);
        if (more) wide_step_schedule<2 * TERMS, 2 * NP * RT, true>();
        else wide_step_schedule<0, 2 * NP * RT, true>();
    }
}

// One quad (four rows of a 32-row tile, four columns per lane) of the
// epilogue.  KIND 0: general, 1: beta == 0, 2: beta == 0 and alpha == 1.
// At KIND 2 the split modes scale in binary32: acc * 2^e is exact in
// binary64, so RN32 of it is one correctly rounded scaling, which is what
// v_ldexp_f32 computes (subnormal and overflowing results included).
template <int MODE, int KIND>
__device__ __forceinline__ f4v wide_out4(const f16v (&acc)[4], int r, const int (&e)[4], double alpha, double beta,
                                         const f4v &c) {
    f4v o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float a = acc[i][r];
        if constexpr (MODE == 0 && KIND == 2) {
            o[i] = a;  // RN32(a) == a
        } else if constexpr (KIND == 2) {
            o[i] = __builtin_ldexpf(a, e[i]);  // RN32(a * 2^e)
        } else {
#pragma clang fp contract(off)
            double t = (double)a;
            if constexpr (MODE != 0) t = __builtin_ldexp(t, e[i]);
            if constexpr (KIND != 2) t = alpha * t;
            if constexpr (KIND == 0) t = t + beta * (double)c[i];
            o[i] = (float)t;
        }
    }
    return o;
}

// binary64 epilogue of the wavefront's RT x NT tiles, 16-byte C vectors:
// out = RN32(RN(alpha * acc * 2^e) + RN(beta * c)) in binary64 (e: the
// column exponent of the split modes).  Two shortcuts give the same bits:
// beta == 0 never loads C, and alpha == 1 drops the multiplication.  The
// choice is made per quad, so that the compiler cannot hoist work common to
// the variants (it would keep every accumulator live as binary64).  With
// beta != 0, C is read one quad ahead.
template <int MODE, int NT, int RT>
__device__ __forceinline__ void wide_epilogue(const f16v (&acc)[RT][NT], const int (&ex)[NT / 4][4],
                                              float *__restrict__ C, int64_t m, int n, int64_t row_base,
                                              double alpha, double beta, int j, int q) {
    constexpr int NG = NT / 4;
    constexpr int NQ = RT * NG * 4;  // quads: (rt, g, r / 4)
    const int kind = beta != 0.0 ? 0 : (alpha != 1.0 ? 1 : 2);
    __amdgpu_buffer_rsrc_t rc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64(row_base + 32 * rt);
        rc[rt] = make_rsrc(C + row0 * n, tile_rows32(m, row0) * (int64_t)n * 4);
    }
    int vo = (4 * q * n + 4 * j) * 4;  // row 4q, columns 4j.. of a tile (opaque, as in wide_load_a)
    asm volatile("" : "+v"(vo));
    auto off = [&](int g, int r) { return vo + ((8 * (r / 4) + r % 4) * n + 128 * g) * 4; };
    f4v cv[2][4];
    if (kind == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            cv[0][i] = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rc[0], off(0, i), 0, 2));
    }
#pragma unroll
    for (int qd = 0; qd < NQ; ++qd) {
        const int rt = qd / (NG * 4), g = (qd / 4) % NG, r4 = qd % 4;
        const f16v(&a4)[4] = *reinterpret_cast<const f16v(*)[4]>(&acc[rt][4 * g]);
        if (kind == 0) {
            if (qd + 1 < NQ) {
                const int rt1 = (qd + 1) / (NG * 4), g1 = ((qd + 1) / 4) % NG, r41 = (qd + 1) % 4;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    cv[(qd + 1) & 1][i] = __builtin_bit_cast(
                        f4v, __builtin_amdgcn_raw_buffer_load_b128(rc[rt1], off(g1, 4 * r41 + i), 0, 2));
            }
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                __builtin_amdgcn_raw_buffer_store_b128(
                    __builtin_bit_cast(u32x4, wide_out4<MODE, 0>(a4, 4 * r4 + rr, ex[g], alpha, beta, cv[qd & 1][rr])),
                    rc[rt], off(g, 4 * r4 + rr), 0, 2);
        } else if (kind == 1) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                __builtin_amdgcn_raw_buffer_store_b128(
                    __builtin_bit_cast(u32x4, wide_out4<MODE, 1>(a4, 4 * r4 + rr, ex[g], alpha, beta, f4v{})),
                    rc[rt], off(g, 4 * r4 + rr), 0, 2);
        } else {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                __builtin_amdgcn_raw_buffer_store_b128(
                    __builtin_bit_cast(u32x4, wide_out4<MODE, 2>(a4, 4 * r4 + rr, ex[g], alpha, beta, f4v{})),
                    rc[rt], off(g, 4 * r4 + rr), 0, 2);
        }
    }
}

// MODE: 0 binary32 products, 3 or 6 split-bf16 products.  KC: packed k
// class (64, 128, 256); NT: 32-column tiles (n / 32); RT: 32-row tiles per
// wavefront; WV: wavefronts per workgroup (4 or 8: one or two per SIMD).
template <int MODE, int KC, int NT, int RT, int WV>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(WV / 4, WV / 4))) void k_wide(
    const float *__restrict__ A, const u32x4 *__restrict__ W, const int32_t *__restrict__ exps,
    float *__restrict__ C, int64_t m, int n, int k, double alpha, double beta) {
    constexpr int F = WideCfg<MODE>::F;
    constexpr int TERMS = WideCfg<MODE>::TERMS;
    constexpr int NCH = KC / 32;
    constexpr int SLAB = F * NT;
    constexpr int ROWS = WV * RT * 32;
    static_assert(NCH % 2 == 0 && SLAB % WV == 0 && NT % 4 == 0 && (WV == 4 || WV == 8), "wide kernel shape");

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

    // Pipeline.  Chunk g (g counts over the tiles of this workgroup) reads
    // slab g from LDS; slab g+1 is moved in during chunk g.
    //   binary32: A(g) is read from registers during the chunk, A(g+1)
    //   loads meanwhile; the end of the chunk waits for every load.
    //   split: the A terms of each bf16 k-step are split one half chunk
    //   ahead, in the shadow of the products; A(g+2) is loaded into the
    //   registers of A(g) as they free up (the first two vectors at the
    //   start of chunk g, the last two at its middle), so every A load has
    //   more than a chunk to arrive.  At the end of a chunk only those A
    //   loads may still be in flight: slab g+1 has landed.
    f4v x0[RT][4], x1[RT][4];
    if constexpr (MODE == 0) {
        wide_dma<SLAB, WV>(rw, 0, wave, lane, sb0);
        wide_load_a<RT, 0, 4>(A, m, k, tile * ROWS + wrow, 0, j, q, x0);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        for (;;) {
            f16v acc[RT][NT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[rt][t] = f16v{};
            const int64_t next = tile + gridDim.x;
#pragma unroll
            for (int c = 0; c < NCH; c += 2) {
                wide_dma<SLAB, WV>(rw, c + 1, wave, lane, sb1);
                wide_load_a<RT, 0, 4>(A, m, k, tile * ROWS + wrow, c + 1, j, q, x1);
                wide_chunk_f32<NT, RT>(sb0, x0, acc, lane);
                __builtin_amdgcn_s_waitcnt(0x0F70);
                __syncthreads();
                const bool last = c + 2 >= NCH;
                wide_dma<SLAB, WV>(rw, last ? 0 : c + 2, wave, lane, sb0);
                wide_load_a<RT, 0, 4>(A, m, k, (last ? next : tile) * ROWS + wrow, last ? 0 : c + 2, j, q, x0);
                wide_chunk_f32<NT, RT>(sb1, x1, acc, lane);
                __builtin_amdgcn_s_waitcnt(0x0F70);
                __syncthreads();
            }
            wide_epilogue<MODE, NT, RT>(acc, ex, C, m, n, tile * ROWS + wrow, alpha, beta, j, q);
            tile = next;
            if (tile >= ntile) break;
        }
    } else {
        constexpr int NA = RT * 4;  // A loads per chunk
        constexpr int WAIT_END = 0x0F70 | (NA & 15) | ((NA >> 4) << 14);  // vmcnt(NA)
        u32x4 atA[RT][TERMS], atB[RT][TERMS];  // A terms of the chunk's first / second k-step
        u32x4 b[2][2][TERMS];                  // B fragments, one step ahead
        wide_dma<SLAB, WV>(rw, 0, wave, lane, sb0);
        wide_load_a<RT, 0, 4>(A, m, k, tile * ROWS + wrow, 0, j, q, x0);
        wide_load_a<RT, 0, 4>(A, m, k, tile * ROWS + wrow, 1, j, q, x1);
        __builtin_amdgcn_s_waitcnt(WAIT_END);
        __syncthreads();
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int w = 0; w < 4; ++w) wide_split_pair<TERMS>(x0[rt][0], x0[rt][1], w, atA[rt]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int p = 0; p < TERMS; ++p) b[0][u][p] = sb0[(p * NT + u) * 64 + lane];
        for (;;) {
            f16v acc[RT][NT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[rt][t] = f16v{};
            const int64_t next = tile + gridDim.x;
#pragma unroll
            for (int c = 0; c < NCH; c += 2) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int cc = c + half;
                    const u32x4 *cur = half ? sb1 : sb0;
                    u32x4 *nxt = half ? sb0 : sb1;
                    f4v(&xc)[RT][4] = half ? x1 : x0;  // A(g); becomes A(g+2)
                    f4v(&xo)[RT][4] = half ? x0 : x1;  // A(g+1)
                    const int c1 = cc + 1 < NCH ? cc + 1 : cc + 1 - NCH;
                    const int c2 = cc + 2 < NCH ? cc + 2 : cc + 2 - NCH;
                    const int64_t t2 = cc + 2 < NCH ? tile : next;
                    wide_dma<SLAB, WV>(rw, c1, wave, lane, nxt);
                    wide_load_a<RT, 0, 2>(A, m, k, t2 * ROWS + wrow, c2, j, q, xc);
                    __builtin_amdgcn_sched_barrier(0);
                    f4v s0[RT], s1[RT];
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        s0[rt] = xc[rt][2];
                        s1[rt] = xc[rt][3];
                    }
                    // first k-step; split this chunk's second k-step meanwhile
                    wide_half_split<MODE, NT, RT>(cur, 0, true, atA, s0, s1, atB, b, acc, lane);
                    wide_load_a<RT, 2, 4>(A, m, k, t2 * ROWS + wrow, c2, j, q, xc);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        s0[rt] = xo[rt][0];
                        s1[rt] = xo[rt][1];
                    }
                    // second k-step; split the next chunk's first k-step
                    wide_half_split<MODE, NT, RT>(cur, 1, false, atB, s0, s1, atA, b, acc, lane);
                    __builtin_amdgcn_s_waitcnt(WAIT_END);  // this wavefront's slab g+1 has landed
                    __syncthreads();                        // ... and every wavefront's
                    // first fragments of the next chunk
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int p = 0; p < TERMS; ++p) b[0][u][p] = nxt[(p * NT + u) * 64 + lane];
                }
            }
            wide_epilogue<MODE, NT, RT>(acc, ex, C, m, n, tile * ROWS + wrow, alpha, beta, j, q);
            tile = next;
            if (tile >= ntile) break;
        }
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

template <int MODE, int KC, int NT, int RT, int WV>
hipError_t run_wide(const float *A, const void *W, const int32_t *exps, float *C, int64_t m, int64_t n, int64_t k,
                    double alpha, double beta, int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL((k_wide<MODE, KC, NT, RT, WV>), dim3((unsigned)grid), dim3(64 * WV), 0, s, A,
                       static_cast<const u32x4 *>(W), exps, C, m, (int)n, (int)k, alpha, beta);
    return hipGetLastError();
}

typedef hipError_t (*WideFn)(const float *, const void *, const int32_t *, float *, int64_t, int64_t, int64_t,
                             double, double, int64_t, hipStream_t);
struct WideEntry {
    int mode, KC, NT, RT, WV;
    WideFn fn;
};

#define TSMM_WE(M, KC, NT, RT, WV) {M, KC, NT, RT, WV, &run_wide<M, KC, NT, RT, WV>},
#define TSMM_WE_KC(M, NT, RT, WV) TSMM_WE(M, 64, NT, RT, WV) TSMM_WE(M, 128, NT, RT, WV) TSMM_WE(M, 256, NT, RT, WV)
// four 32-row tiles per wavefront only for binary32 products: the split
// modes' A terms would not fit the registers beside 256 accumulators.
// Eight wavefronts (two per SIMD) hold one row tile each.
static const WideEntry kWideTable[] = {TSMM_WE_KC(0, 8, 2, 4) TSMM_WE_KC(0, 4, 2, 4) TSMM_WE_KC(0, 4, 4, 4)
                                       TSMM_WE_KC(3, 8, 2, 4) TSMM_WE_KC(3, 4, 2, 4) TSMM_WE_KC(6, 8, 2, 4)
                                       TSMM_WE_KC(6, 4, 2, 4)
                                       TSMM_WE_KC(0, 8, 1, 8) TSMM_WE_KC(0, 4, 1, 8) TSMM_WE_KC(3, 8, 1, 8)
                                       TSMM_WE_KC(3, 4, 1, 8) TSMM_WE_KC(6, 8, 1, 8) TSMM_WE_KC(6, 4, 1, 8)};

static WideFn find_wide(int mode, int KC, int NT, int RT, int WV) {
    for (const WideEntry &e : kWideTable)
        if (e.mode == mode && e.KC == KC && e.NT == NT && e.RT == RT && e.WV == WV) return e.fn;
    return nullptr;
}

bool wide_variant_exists(int products, int KC, int NT, int RT, int waves) {
    return find_wide(products, KC, NT, RT, waves) != nullptr;
}

int64_t wide_rows_per_wg(int RT, int waves) { return (int64_t)waves * RT * 32; }

hipError_t launch_wide(int products, int KC, int NT, int RT, int waves, const void *A, const void *W,
                       const int32_t *exps, void *C, int64_t m, int64_t n, int64_t k, double alpha, double beta,
                       int64_t grid, hipStream_t s) {
    WideFn fn = find_wide(products, KC, NT, RT, waves);
    if (!fn || n != 32 * NT || k > KC || k % 8 != 0 || grid < 1) return hipErrorInvalidValue;
    return fn(static_cast<const float *>(A), W, exps, static_cast<float *>(C), m, n, k, alpha, beta, grid, s);
}

}  // namespace tsmm
