// op N with bfloat16 matrix-core products (V_MFMA_F32_16X16X32_BF16):
//   - split-bf16 modes for binary32 A and B: every binary32 element is
//     written as a sum of bfloat16 terms (hi, mid[, lo]); A is split in
//     registers as it streams in, B was split once at pack time (with a
//     power-of-two scale per column, undone in the epilogue); the products
//     of term order i + j <= 1 (3 products) or i + j <= 2 (6 products) are
//     accumulated in binary32, the leading hi*hi product in its own
//     accumulator and the correction products in a second one, and the two
//     are added in the binary64 epilogue;
//   - plain bfloat16 inputs (one term, one product), binary32 output.
// Row tiles are walked with a grid stride exactly as in the binary64 /
// binary32 streaming kernel (k_stream.h).
#pragma once

#include "k_common.h"
#include "tsmm_internal.h"

namespace tsmm {

constexpr int kBf16Block = 256;
constexpr int kBf16LdsBudget = 128 * 1024;

__device__ __forceinline__ f4v mfma_bf16(const u16x8 &a, const u16x8 &b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c,
                                                   0, 0, 0);
}

// Residual split of 8 binary32 values into TERMS bfloat16 vectors.
template <int TERMS>
__device__ __forceinline__ void split8(const float (&x)[8], u16x8 (&t)[TERMS]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        float r = x[e];
#pragma unroll
        for (int p = 0; p < TERMS; ++p) {
            const uint16_t h = float_to_bf16_bits(r);
            t[p][e] = h;
            if (p + 1 < TERMS) r = r - bf16_bits_to_float(h);
        }
    }
}

// How a kernel receives A: 0 bfloat16 values (one term), 1 binary32
// values split in registers, 2 or 3: A split ahead of time into that many
// bfloat16 planes (packed A, presplit layout of tsmm_internal.h; uint16_t
// with PROD > 1).
template <typename TA, int PROD> constexpr int a_kind() {
    return PROD == 1 ? 0 : (sizeof(TA) == 4 ? 1 : (PROD == 3 ? 2 : 3));
}
template <int KIND, int RT, int NCH> struct RawA {  // pre-split planes
    u16x8 v[RT][NCH][KIND];
};
template <int RT, int NCH> struct RawA<1, RT, NCH> {
    float v[RT][NCH][8];
};
template <int RT, int NCH> struct RawA<0, RT, NCH> {
    u16x8 v[RT][NCH];
};

// A of row tiles t .. t+RT-1: binary32 values (split modes), bf16 vectors,
// or the vectors of every plane of a pre-split A.  Vector loads go through
// one buffer resource per 16-row tile sized to the rows that exist (rows
// beyond m read 0); columns beyond k read through kOOB.
template <typename TA, int KC, int RT, int PROD, bool VEC>
__device__ __forceinline__ void bf16_load_step(const TA *__restrict__ A, int64_t m, int k, int64_t t, int j, int q,
                                               RawA<a_kind<TA, PROD>(), RT, KC / 32> &x) {
    constexpr int NCH = KC / 32;
    constexpr int KIND = a_kind<TA, PROD>();
    constexpr bool F32IN = KIND == 1;
    constexpr int SZ = F32IN ? 4 : 2;
    if constexpr (KIND >= 2) {
        static_assert(VEC, "pre-split rows are whole vectors");
        // plane p of tile row0: 16 padded rows (zeros past m), none past
        // the last tile
        const int ld = (int)presplit_ld(k);
        const int64_t pstride = presplit_rows(m) * ld;
        const int voff0 = j * ld * 2;
        constexpr int AUX = KC * 2 >= 1024 ? 0 : 2;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t row0 = uniform64((t + rt) * 16);
            const int bytes = row0 < m ? 16 * ld * 2 : 0;
#pragma unroll
            for (int p = 0; p < KIND; ++p) {
                const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + p * pstride + row0 * ld, bytes);
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const int col = 32 * c + 8 * q;
                    x.v[rt][c][p] = __builtin_bit_cast(
                        u16x8, __builtin_amdgcn_raw_buffer_load_b128(ra, col < k ? voff0 + col * 2 : kOOB, 0, AUX));
                }
            }
        }
    } else {
        // rows of 1 KiB and more: default cache policy (see stream_load_a)
        constexpr int AUX = KC * SZ >= 1024 ? 0 : 2;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t row0 = uniform64((t + rt) * 16);
            if constexpr (VEC) {
                const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + row0 * k, tile_rows(m, row0) * (int64_t)k * SZ);
                const int voff0 = j * k * SZ;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const int col = 32 * c + 8 * q;
                    if constexpr (F32IN) {
                        const f4v v0 = BufIO<float>::load_vec<AUX>(ra, col < k ? voff0 + col * SZ : kOOB);
                        const f4v v1 = BufIO<float>::load_vec<AUX>(ra, col + 4 < k ? voff0 + (col + 4) * SZ : kOOB);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            x.v[rt][c][e] = v0[e];
                            x.v[rt][c][4 + e] = v1[e];
                        }
                    } else {
                        x.v[rt][c] = __builtin_bit_cast(
                            u16x8, __builtin_amdgcn_raw_buffer_load_b128(ra, col < k ? voff0 + col * SZ : kOOB, 0, AUX));
                    }
                }
            } else {
                // one load per value through the tile's resource: values past k
                // read through kOOB (no branch around a load, so the compiler
                // need not wait for the prefetch before the products)
                const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + row0 * k, tile_rows(m, row0) * (int64_t)k * SZ);
                const int voff0 = j * k * SZ;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const int col = 32 * c + 8 * q;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int off = col + e < k ? voff0 + (col + e) * SZ : kOOB;
                        if constexpr (F32IN)
                            x.v[rt][c][e] = BufIO<float>::template load1<AUX>(ra, off);
                        else
                            x.v[rt][c][e] = __builtin_amdgcn_raw_buffer_load_b16(ra, off, 0, AUX);
                    }
                }
            }
        }
    }
}

// One row step: products of tiles t.. from x_use while tiles tnext.. load
// into x_load; C is read through a resource that is empty when beta == 0.
template <typename TA, int KC, int NT, int RT, int PROD, bool VEC, bool IL = false, bool CPRE = true>
__device__ __forceinline__ void bf16_step(const TA *__restrict__ A, const u16x8 *__restrict__ Bsrc, int bstride,
                                          const int32_t *__restrict__ exps, float *__restrict__ C, int64_t m, int n,
                                          int k, double alpha, double beta, int col0, int64_t t, int64_t tnext,
                                          int j, int q, int lane,
                                          const RawA<a_kind<TA, PROD>(), RT, KC / 32> &x_use,
                                          RawA<a_kind<TA, PROD>(), RT, KC / 32> &x_load) {
    constexpr int TERMS = PROD == 1 ? 1 : (PROD == 3 ? 2 : 3);
    constexpr int NCH = KC / 32;
    constexpr bool TWO_ACC = PROD > 1;
    constexpr int KIND = a_kind<TA, PROD>();

    __amdgpu_buffer_rsrc_t rc[RT], rl[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t row0 = uniform64((t + rt) * 16);
        const int64_t bytes = (tile_rows(m, row0) * (int64_t)n - col0) * 4;
        rc[rt] = make_rsrc(C + row0 * n + col0, bytes);
        rl[rt] = make_rsrc(C + row0 * n + col0, beta != 0.0 ? bytes : 0);
    }
    // Interleaved columns (IL, n % 4 == 0; the fragment order of
    // tsmm_internal.h): tile tt of lane j is column colp(tt) of the group, a
    // lane holds 4 adjacent columns in the 4 tiles of a group, and C moves
    // in 16-byte vectors.
    constexpr int PG = IL ? 4 : 1;
    static_assert(!IL || NT % 4 == 0, "interleave: whole groups of 4 column tiles");
    auto colp = [=](int tt) { return 16 * PG * (tt / PG) + PG * j + tt % PG; };
    auto coff = [=](int tt, int r) { return (col0 + colp(tt) < n) ? ((4 * q + r) * n + colp(tt)) * 4 : kOOB; };
    auto voff = [=](int g, int r) {
        return (col0 + colp(PG * g) < n) ? ((4 * q + r) * n + colp(PG * g)) * 4 : kOOB;
    };
    float cv[RT][NT][4];
    if constexpr (CPRE) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            if constexpr (IL) {
#pragma unroll
                for (int g = 0; g < NT / PG; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const f4v v = BufIO<float>::load_vec(rl[rt], voff(g, r));
#pragma unroll
                        for (int i = 0; i < PG; ++i) cv[rt][PG * g + i][r] = v[i];
                    }
            } else {
#pragma unroll
                for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) cv[rt][tt][r] = BufIO<float>::load1(rl[rt], coff(tt, r));
            }
        }
    }
    bf16_load_step<TA, KC, RT, PROD, VEC>(A, m, k, tnext, j, q, x_load);
    __builtin_amdgcn_sched_barrier(0);

    f4v acc[RT][NT];
    f4v acc2[TWO_ACC ? RT : 1][TWO_ACC ? NT : 1];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
            acc[rt][tt] = f4v{};
            if constexpr (TWO_ACC) acc2[rt][tt] = f4v{};
        }

    // small B may live in registers; larger B is re-read per row step
    int bofs = 0;
    if constexpr (NCH * NT * TERMS > 8) asm volatile("" : "+v"(bofs));

#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        u16x8 at[RT][TERMS];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            if constexpr (KIND == 1) {
                split8<TERMS>(x_use.v[rt][c], at[rt]);
            } else if constexpr (KIND == 0) {
                at[rt][0] = x_use.v[rt][c];
            } else {
#pragma unroll
                for (int p = 0; p < TERMS; ++p) at[rt][p] = x_use.v[rt][c][p];
            }
        }
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
            u16x8 bt[TERMS];
#pragma unroll
            for (int p = 0; p < TERMS; ++p) bt[p] = Bsrc[bofs + ((c * bstride + tt) * TERMS + p) * 64 + lane];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                acc[rt][tt] = mfma_bf16(at[rt][0], bt[0], acc[rt][tt]);
                if constexpr (PROD >= 3) {
                    acc2[rt][tt] = mfma_bf16(at[rt][0], bt[1], acc2[rt][tt]);
                    acc2[rt][tt] = mfma_bf16(at[rt][1], bt[0], acc2[rt][tt]);
                }
                if constexpr (PROD == 6) {
                    acc2[rt][tt] = mfma_bf16(at[rt][0], bt[2], acc2[rt][tt]);
                    acc2[rt][tt] = mfma_bf16(at[rt][1], bt[1], acc2[rt][tt]);
                    acc2[rt][tt] = mfma_bf16(at[rt][2], bt[0], acc2[rt][tt]);
                }
            }
        }
    }
    __builtin_amdgcn_sched_barrier(0);

    if constexpr (IL) {
        // the column exponents of the split modes, per tile of this lane
        int ecol[PROD > 1 ? NT : 1];
        if constexpr (PROD > 1) {
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
                const int col = col0 + colp(tt);
                ecol[tt] = col < n ? exps[col] : 0;
            }
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int g = 0; g < NT / PG; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if constexpr (!CPRE) {
                        const f4v v = beta != 0.0 ? BufIO<float>::load_vec(rl[rt], voff(g, r)) : f4v{};
#pragma unroll
                        for (int i = 0; i < PG; ++i) cv[rt][PG * g + i][r] = v[i];
                    }
                    f4v o;
#pragma unroll
                    for (int i = 0; i < PG; ++i) {
                        // the same arithmetic as the plain column order below
                        double sacc = (double)acc[rt][PG * g + i][r];
                        if constexpr (TWO_ACC) sacc = sacc + (double)acc2[rt][PG * g + i][r];
                        if constexpr (PROD > 1) sacc = __builtin_ldexp(sacc, ecol[PG * g + i]);
                        o[i] = (float)epilogue(alpha, sacc, beta, (double)cv[rt][PG * g + i][r]);
                    }
                    BufIO<float>::store_vec(o, rc[rt], voff(g, r));
                }
    } else {
        int ecol[PROD > 1 ? NT : 1];
        if constexpr (PROD > 1) {
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
                const int col = col0 + 16 * tt + j;
                ecol[tt] = col < n ? exps[col] : 0;
            }
        }
        // the column tiles of one row quad are stored back to back: the
        // parts of a 128-byte line of C then reach the cache together.  In
        // the split modes the stores keep the default cache policy, so the
        // cache joins the parts of a line before writing it (streaming
        // stores were measured to write 10-16% more bytes than C holds at
        // n = 32, and ran 4% slower); plain bfloat16 inputs (the batched
        // launch) stream, which measured faster there.
        constexpr int SAUX = PROD > 1 ? 0 : 2;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int tt = 0; tt < NT; ++tt) {
                    // without the C prefetch, C is read here (beta != 0 only)
                    if constexpr (!CPRE) cv[rt][tt][r] = beta != 0.0 ? BufIO<float>::load1(rl[rt], coff(tt, r)) : 0.0f;
                    double sacc = (double)acc[rt][tt][r];
                    if constexpr (TWO_ACC) sacc = sacc + (double)acc2[rt][tt][r];
                    if constexpr (PROD > 1) sacc = __builtin_ldexp(sacc, ecol[tt]);
                    BufIO<float>::template store1<SAUX>((float)epilogue(alpha, sacc, beta, (double)cv[rt][tt][r]),
                                                        rc[rt], coff(tt, r));
                }
    }
}

// PROD: 1 (plain bf16), 3 (two terms) or 6 (three terms).  NT: column tiles
// per workgroup (one column group of the nt_total tiles when nsplit > 1,
// with the workgroup -> (row block, group) map of k_stream.h).
template <typename TA, int KC, int NT, int RT, int PROD, bool VEC, bool IL>
__global__ __launch_bounds__(kBf16Block) void k_splitbf16(const TA *__restrict__ A,
                                                          const uint16_t *__restrict__ Bf,
                                                          const int32_t *__restrict__ exps,
                                                          float *__restrict__ C, int64_t m, int n, int k,
                                                          double alpha, double beta, int nt_total, int nsplit) {
    constexpr int TERMS = PROD == 1 ? 1 : (PROD == 3 ? 2 : 3);
    constexpr int NCH = KC / 32;
    constexpr int FRAGV = NCH * NT * TERMS * 64;  // 16-byte vectors per workgroup
    constexpr bool BLDS = FRAGV * 16 <= kBf16LdsBudget;

    int group = 0;
    int64_t rb = blockIdx.x, nrb = gridDim.x;
    if (nsplit > 1) {
        const int64_t slot = blockIdx.x >> 3;
        group = (int)(slot % nsplit);
        rb = (slot / nsplit) * 8 + (blockIdx.x & 7);
        nrb = gridDim.x / nsplit;
    }
    const int col0 = group * NT * 16;

    __shared__ u16x8 sB[BLDS ? FRAGV : 1];
    const u16x8 *__restrict__ Bg = reinterpret_cast<const u16x8 *>(Bf);
    if constexpr (BLDS) {
        for (int idx = threadIdx.x; idx < FRAGV; idx += blockDim.x) {
            const int c = idx / (NT * TERMS * 64), rem = idx % (NT * TERMS * 64);
            sB[idx] = Bg[(c * nt_total + group * NT) * TERMS * 64 + rem];
        }
        __syncthreads();
    }

    const int lane = threadIdx.x & 63;
    const int j = lane & 15;
    const int q = lane >> 4;
    const int64_t ntile = (m + 15) >> 4;
    const int wpb = blockDim.x >> 6;
    const int64_t gw = rb * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tstride = nrb * wpb * RT;

    const u16x8 *__restrict__ Bsrc = BLDS ? sB : Bg + group * NT * TERMS * 64;
    const int bstride = BLDS ? NT : nt_total;  // column tiles per k-chunk in Bsrc
    // Ping-pong over two register sets, steps in pairs with no branch between
    // them (a pair's second step may lie past the last tile: its loads read
    // 0 and its stores are dropped).
    RawA<a_kind<TA, PROD>(), RT, NCH> x0, x1;
    int64_t t = gw * RT;
    if (t >= ntile) return;
    bf16_load_step<TA, KC, RT, PROD, VEC>(A, m, k, t, j, q, x0);
    for (; t < ntile; t += 2 * tstride) {
        bf16_step<TA, KC, NT, RT, PROD, VEC, IL>(A, Bsrc, bstride, exps, C, m, n, k, alpha, beta, col0, t,
                                                 t + tstride, j, q, lane, x0, x1);
        bf16_step<TA, KC, NT, RT, PROD, VEC, IL>(A, Bsrc, bstride, exps, C, m, n, k, alpha, beta, col0,
                                                 t + tstride, t + 2 * tstride, j, q, lane, x1, x0);
    }
}

template <typename TA, int KC, int NT, int RT, int PROD, bool VEC, bool IL>
hipError_t run_splitbf16(const void *A, const void *Bf, const int32_t *exps, void *C, int64_t m, int64_t n,
                         int64_t k, double alpha, double beta, int64_t grid, int block, int nt_total, int nsplit,
                         hipStream_t s) {
    hipLaunchKernelGGL((k_splitbf16<TA, KC, NT, RT, PROD, VEC, IL>), dim3((unsigned)grid), dim3(block), 0, s,
                       static_cast<const TA *>(A), static_cast<const uint16_t *>(Bf), exps, static_cast<float *>(C),
                       m, (int)n, (int)k, alpha, beta, nt_total, nsplit);
    return hipGetLastError();
}

typedef hipError_t (*Bf16Fn)(const void *, const void *, const int32_t *, void *, int64_t, int64_t, int64_t,
                             double, double, int64_t, int, int, int, hipStream_t);
struct Bf16Entry {
    int KC, NT, RT, prod, vec, il;
    Bf16Fn fn;
};

}  // namespace tsmm

#define TSMM_BE(TA, KC, NT, RT, P, V) {KC, NT, RT, P, V, 0, &tsmm::run_splitbf16<TA, KC, NT, RT, P, V, false>},
#define TSMM_BE_NT(TA, KC, RT, P, V) \
    TSMM_BE(TA, KC, 1, RT, P, V) TSMM_BE(TA, KC, 2, RT, P, V) TSMM_BE(TA, KC, 4, RT, P, V) TSMM_BE(TA, KC, 8, RT, P, V) \
    TSMM_BE(TA, KC, 16, RT, P, V)
#define TSMM_BE_KC(TA, RT, P, V) \
    TSMM_BE_NT(TA, 32, RT, P, V) TSMM_BE_NT(TA, 64, RT, P, V) TSMM_BE_NT(TA, 128, RT, P, V) TSMM_BE_NT(TA, 256, RT, P, V)
// interleaved columns (NT >= 4): bfloat16 inputs (TSMM_BEI*), binary32
// split modes (TSMM_BEF*)
#define TSMM_BEF(KC, NT, RT, P, V) {KC, NT, RT, P, V, 1, &tsmm::run_splitbf16<float, KC, NT, RT, P, V, true>},
#define TSMM_BEF_NT(KC, RT, P, V) TSMM_BEF(KC, 4, RT, P, V) TSMM_BEF(KC, 8, RT, P, V) TSMM_BEF(KC, 16, RT, P, V)
#define TSMM_BEF_KC(RT, P, V) \
    TSMM_BEF_NT(32, RT, P, V) TSMM_BEF_NT(64, RT, P, V) TSMM_BEF_NT(128, RT, P, V) TSMM_BEF_NT(256, RT, P, V)
#define TSMM_BEI(KC, NT, RT, V) {KC, NT, RT, 1, V, 1, &tsmm::run_splitbf16<uint16_t, KC, NT, RT, 1, V, true>},
#define TSMM_BEI_NT(KC, RT, V) TSMM_BEI(KC, 4, RT, V) TSMM_BEI(KC, 8, RT, V) TSMM_BEI(KC, 16, RT, V)
#define TSMM_BEI_KC(RT, V) TSMM_BEI_NT(32, RT, V) TSMM_BEI_NT(64, RT, V) TSMM_BEI_NT(128, RT, V) TSMM_BEI_NT(256, RT, V)
