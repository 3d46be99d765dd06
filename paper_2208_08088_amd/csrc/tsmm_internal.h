// Internal declarations shared by the host runtime and the HIP kernels of
// libtsmm: packed-operand layout rules, plan structures and kernel
// launchers.  Not part of the public ABI (include/tsmm.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tsmm.h"

namespace tsmm {

// ---------------------------------------------------------------- layout
//
// Matrix-core fragment order of a packed B (op N).
//
// The streaming kernels use the 16x16x4 matrix-core products for binary64
// and binary32 (V_MFMA_F64_16X16X4_F64, V_MFMA_F32_16X16X4_F32).  In one
// product, lane l = 16*q + j (q = 0..3, j = 0..15) supplies
//   A-operand element (row j, k-slot q) and B-operand element (k-slot q,
//   column j),
// and receives four accumulator rows of column j: rows q + 4*r (binary64)
// or 4*q + r (binary32), r = 0..3.
// The k-slot -> column-of-A assignment is free as long as A and B agree,
// so it is chosen to make every lane's A load one contiguous 16-byte
// vector: with VW = 16 / sizeof(T) elements per vector, k-step s and slot q
// read column
//     col(s, q) = (s / VW) * 4*VW + q*VW + (s % VW)        (vector mapping)
//     col(s, q) = 4*s + q                                   (scalar mapping)
// The vector mapping is used when k % VW == 0 and KC % (4*VW) == 0 (rows
// stay 16-byte aligned and a vector never straddles the end of a row).
// When NT >= VW and n % VW == 0 the columns of B are interleaved in groups of PG = VW column tiles (otherwise PG = 1): tile t,
// lane column j holds
// column
//     colp(t, j) = 16*PG*(t / PG) + PG*j + t % PG,
// so that a lane's accumulators of the PG tiles of a group are PG adjacent
// columns of C (one 16-byte vector).  Packed B holds, for k-step s < KC/4,
// column tile t < NT and lane l,
//     frag[(s*NT + t)*64 + l] = B[col(s, q)][colp(t, j)]   (0 outside k x n).
// A plan that splits the tiles into column groups keeps whole interleave
// groups in each (NT / nsplit a multiple of PG).
//
// The split-bfloat16 kernels use V_MFMA_F32_16X16X32_BF16: lane 16*q + j
// supplies 8 consecutive k-slots 8q..8q+7 of a 32-wide k-chunk.  Packed B
// holds, per chunk c < KC/32, column tile t, plane p and lane l, 8 bfloat16
//     bfrag[(((c*NT + t)*P + p)*64 + l)*8 + u] = plane p of
//         B[32c + 8q + u][16t + j] * 2^-e_(16t+j)
// where e_j is the column's power-of-two exponent (1 <= max|B[:,j]|*2^-e_j
// < 2) and planes are the residual split hi, mid, lo.  With NT >= 4 and
// n % 4 == 0 the columns are interleaved in groups of 4 tiles as above
// (16t + j -> colp(t, j) with PG = 4), so that binary32 C moves in 16-byte
// vectors; the row-major split planes and the exponents keep the plain
// column order.
//
// The wide kernels (k_wide.hip; binary32 B with n = 128 or 256, k <= 256,
// k % 8 == 0) use the 32x32 products.  Their image holds, per 32-row chunk
// c < KC/32 of B, fragment f < F, 32-column tile t < NT = n/32 and lane
// l = 32q + j, one 16-byte vector:
//   native (F = 4, f = h):       B[32c + 8h + 4q + u][col(t, j)], u < 4
//   split  (F = 2T, f = s*T + p): plane p of
//                                B[32c + 16s + 8(e/4) + 4q + e%4][col(t, j)], e < 8
// at wfrag[((c*F + f)*NT + t)*64 + l], col(t, j) = 128(t/4) + 4j + t%4, and
// 0 outside k x n.

constexpr int kMaxKC = 256;  // largest packed k class of the fragment kernels
// The k-slab kernel (long shared dimension): k per slab of packed B, and
// the largest k it takes.
constexpr int kSlabK = 32;
constexpr int64_t kSlabMaxK = (int64_t)1 << 20;
constexpr int kMaxNT = 16;   // largest number of 16-column tiles (n <= 256)

inline int elem_bytes(tsmm_dtype d) { return d == TSMM_F64 ? 8 : (d == TSMM_F32 ? 4 : 2); }

// Column interleave group of the 16x16x4 fragments (see above).
inline int frag4_pg(tsmm_dtype d, int NT, int64_t n) {
    const int vw = 16 / elem_bytes(d);
    return (NT % vw == 0 && n % vw == 0) ? vw : 1;
}
// Column interleave group of the bfloat16 fragments (bfloat16 inputs and
// the split modes of binary32 inputs).
inline int bfrag_pg(tsmm_dtype d, int NT, int64_t n) {
    (void)d;
    return (NT % 4 == 0 && n % 4 == 0) ? 4 : 1;
}

// Smallest k class >= k for the 16x16x4 kernels (0 if k > kMaxKC).
inline int kclass4(int64_t k) {
    for (int c = 4; c <= kMaxKC; c *= 2)
        if (k <= c) return c;
    return 0;
}
// Smallest k class >= k for the bf16 16x16x32 kernels (0 if k > kMaxKC).
inline int kclass32(int64_t k) {
    for (int c = 32; c <= kMaxKC; c *= 2)
        if (k <= c) return c;
    return 0;
}
// Number of 16-column tiles as a power of two class (0 if n > 256).
inline int ntclass(int64_t n) {
    for (int c = 1; c <= kMaxNT; c *= 2)
        if (n <= 16 * c) return c;
    return 0;
}
// Packed A of the split-bf16 modes: rows padded to a multiple of 8
// bfloat16 values (whole 16-byte vectors), the row count to a multiple of
// the 16-row tile, padding holding zeros; plane p starts at
// p * presplit_rows(m) * presplit_ld(k) elements.
__host__ __device__ inline int64_t presplit_ld(int64_t k) { return (k + 7) & ~(int64_t)7; }
__host__ __device__ inline int64_t presplit_rows(int64_t m) { return (m + 15) & ~(int64_t)15; }
inline bool vec_mapping(tsmm_dtype d, int64_t k, int KC) {
    int vw = 16 / elem_bytes(d);
    return (k % vw) == 0 && (KC % (4 * vw)) == 0;
}

// ---------------------------------------------------------------- packed

struct PackedLayout {
    int KC = 0, NT = 0;         // fragment class (0: no fragment copy)
    bool vec = false;           // vector k-slot mapping (16x16x4 kernels)
    int pg = 1;                 // column interleave group (16x16x4 kernels)
    int terms = 0;              // split planes (0: not a split mode)
    size_t off_rowmajor = 0;    // k*n elements of the input type
    size_t off_frag = 0;        // 16x16x4 fragments, or bf16 fragments
    size_t off_planes = 0;      // split: terms*k*n uint16, row-major
    size_t off_exps = 0;        // split: n int32
    int wide_KC = 0, wide_NT = 0;  // wide-kernel image (0: none)
    size_t off_wide = 0;
    // packed A of the split modes with k % 8 == 0: RN32(alpha*A), dense
    // row-major m x k binary32, after the planes (for the wide kernels)
    bool has_a32 = false;
    size_t off_a32 = 0;
    size_t bytes = 0;
};

}  // namespace tsmm

struct tsmm_packed_s {
    int64_t k = 0, n = 0;
    tsmm_layout layout = TSMM_OP_N;
    tsmm_dtype dtype = TSMM_F64;
    tsmm_mode mode = TSMM_MODE_NATIVE;
    int device = 0;
    tsmm::PackedLayout L;
    void *dev = nullptr;        // one device allocation holding every section
    const void *ref = nullptr;  // op T: the caller's B (nothing is copied)
    // packed A (tsmm_pack_a): m x k, alpha folded in; n stays 0.  Native
    // modes: dense row-major alpha*A; split modes: L.terms planes
    // (presplit_ld / presplit_rows).
    bool is_a = false;
    int64_t m = 0;
    double alpha = 1.0;
};

namespace tsmm {

// ------------------------------------------------------------------ plan

struct BatchedInstance {  // host copy of one batched instance
    int64_t m, n, k;
};

// Device descriptor of one batched instance (bound operands).
struct alignas(16) BatchDesc {
    const void *A;
    const void *Bfrag;  // packed fragments of B
    void *C;
    double alpha, beta;
    int64_t m;
    int32_t k, n;
    int32_t KC, NT;
    int32_t vec, il;  // vector k-slot mapping; interleaved columns (16-byte C vectors)
    int32_t chunk_rows;  // rows of this instance per work item
    int32_t pad_;
};

// Rows of one batched chunk (the unit of the dynamic schedule) when the
// tile table has no batched entry, the allowed range (powers of two; a
// multiple of the 16-row tile), and wavefronts per workgroup of the
// batched kernel.
constexpr int kBatchChunkDefault = 4096;
constexpr int kBatchChunkMin = 256, kBatchChunkMax = 65536;
// Rows of one work item of an instance: chunk_rows is the size for rows
// of 256 bytes (a row of A plus a row of C); an instance scales it by
// 256 / its row bytes, to the power of two at or below, within the
// allowed range, so that every work item moves about the same bytes and
// the workgroups finish together.
inline int batch_instance_chunk(int chunk_rows, int64_t k, int64_t n, int a_bytes) {
    const int64_t row_bytes = k * a_bytes + n * 4;
    int64_t c = (int64_t)chunk_rows * 256 / (row_bytes > 0 ? row_bytes : 1);
    int64_t p2 = kBatchChunkMin;
    while (p2 * 2 <= c && p2 < kBatchChunkMax) p2 *= 2;
    return (int)p2;
}
constexpr int kBatchWaves = 8;

}  // namespace tsmm

struct tsmm_plan_s {
    int64_t m = 0, n = 0, k = 0;
    tsmm_layout layout = TSMM_OP_N;
    tsmm_dtype dtype = TSMM_F64;
    tsmm_mode mode = TSMM_MODE_NATIVE;
    tsmm_device_caps caps{};
    int device = 0;
    tsmm_tile tile{};
    int tile_from_table = 0;  // tile source: 0 built-in default or the caller's, 1 tile table, 2 runtime evaluator
    int last_kernel = 0;      // kernel family the last execute ran (0: none yet); differs from tile.kernel when
                              // operand alignment or strides sent it to the any-shape kernel
    // derived launch geometry
    int KC = 0, NT = 0;
    bool vec = false;
    int64_t grid = 0;
    int block = 0;
    int64_t grid_y = 1;
    size_t workspace_bytes = 0;
    hipStream_t stream = nullptr;
    void *workspace = nullptr;
    size_t workspace_size = 0;
    bool owns_workspace = false;
    // batched: instances in execution order (longest first)
    bool batched = false;
    std::vector<tsmm::BatchedInstance> inst;  // caller order
    std::vector<int64_t> order;               // execution position -> caller index
    int64_t n_work = 0;                       // chunks over all instances
    void *d_desc = nullptr;                   // device BatchDesc[count] (execution order)
    void *h_desc = nullptr;                   // pinned staging BatchDesc[count]
    void *d_inst_start = nullptr;             // device int64[count + 1]: first chunk
    void *d_ctr = nullptr;                    // device int32[2]: work counter, finished workgroups
    size_t batch_lds = 0;                     // dynamic LDS of the batched launch
    int graphs = 0;                           // live graphs captured from this plan
    bool bound = false;
    std::vector<tsmm::BatchDesc> bound_desc;
};

struct tsmm_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    tsmm_plan_s *plan = nullptr;  // the batched plan it was captured from
};

namespace tsmm {

// ------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.  All are asynchronous.

// Pack B (k x n row-major) into the 16x16x4 fragment order.
// bcol: B is column-major (element (l, j) at l + j*k) instead of row-major.
// Static device scratch of tsmm_execute_noalloc (k_scratch.hip): bytes, and
// its device address on a device (looked up once per device).
constexpr size_t kScratchBytes = TSMM_NOALLOC_SCRATCH_BYTES;
hipError_t scratch_device_ptr(int device, void **out);

hipError_t launch_pack_frag4(tsmm_dtype dt, bool bcol, const void *B, void *frag, int64_t k, int64_t n,
                             int KC, int NT, bool vec, int pg, hipStream_t s);
// Split-bf16 pack: column exponents, row-major planes and fragments.
// For TSMM_BF16 inputs (terms == 1) B is bf16 and no scaling is applied.
// pg: column interleave group of the fragments (4 or 1; bfloat16 inputs).
hipError_t launch_pack_bf16(tsmm_dtype dt, const void *B, void *frag, void *planes, int32_t *exps,
                            int64_t k, int64_t n, int KC, int NT, int terms, int pg, hipStream_t s);
// Unpack a split handle: B_out[i][j] = (sum of planes) * 2^e_j (binary32).
hipError_t launch_unpack_split(const void *planes, const int32_t *exps, void *B_out, int64_t k,
                               int64_t n, int terms, hipStream_t s);

// Wide kernels (op N binary32 A and C, n = 32*NT with NT 4 or 8, k <= KC,
// k % 8 == 0).  products: 0 (binary32 products), 3 or 6 (split modes).
size_t wide_image_bytes(int KC, int NT, int terms);
hipError_t launch_pack_wide(const void *Bf32, const void *planes, void *W, int64_t k, int64_t n, int KC, int NT,
                            int terms, hipStream_t s);
// waves: wavefronts per workgroup (4 with RT 2 or 4, 8 with RT 1).
bool wide_variant_exists(int products, int KC, int NT, int RT, int waves);
int64_t wide_rows_per_wg(int RT, int waves);
hipError_t launch_wide(int products, int KC, int NT, int RT, int waves, const void *A, const void *W,
                       const int32_t *exps, void *C, int64_t m, int64_t n, int64_t k, double alpha, double beta,
                       int64_t grid, hipStream_t s);

// C = beta*C (alpha == 0 or k == 0 paths).
hipError_t launch_scale(tsmm_dtype out_dt, void *C, int64_t count, double beta, hipStream_t s);

// op N, any shape: one thread per output element, reads the row-major B.
// Any shape with row strides (op N: A(i, l) at i*lda + l; trans: A(l, i) at
// l*lda + i; B(l, j) at l*ldb + j; C(i, j) at i*ldc + j).
hipError_t launch_simple_ld(tsmm_dtype dt, bool trans, const void *A, int64_t lda, const void *B, int64_t ldb,
                            void *C, int64_t ldc, int64_t m, int64_t n, int64_t k, double alpha, double beta,
                            hipStream_t s);
hipError_t launch_simple_n(tsmm_dtype dt, const void *A, const void *B, void *C, int64_t m,
                           int64_t n, int64_t k, double alpha, double beta, hipStream_t s);
// op T, any shape: one thread per output element.
hipError_t launch_simple_t(tsmm_dtype dt, const void *A, const void *B, void *C, int64_t m,
                           int64_t n, int64_t k, double alpha, double beta, hipStream_t s);

// op N streaming, binary64 / binary32 16x16x4 fragments.
// NT: column tiles per workgroup; nt_total = NT * nsplit column tiles of
// the packed B.  With nsplit > 1, grid must be a multiple of 8 * nsplit.
// cm: how C moves: 0 element by element; 1 the fragments interleave
// columns (pg > 1), 16-byte vectors; 2 lane pairs (binary64, NT = 1, n
// even), 16-byte vectors; 5, 6: modes 1, 2 with default-policy C stores
// (binary64, beta == 0).
// lda, ldc: row strides of A and C in elements (>= k, >= n); vector
// k-slot mapping needs lda a multiple of the vector width, C vectors (cm 1
// and 2) a 16-byte aligned C and ldc a multiple of it.
hipError_t launch_stream(tsmm_dtype dt, int KC, int NT, int RT, bool vec, int cm, const void *A,
                         const void *Bfrag, void *C, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldc,
                         double alpha, double beta, int64_t grid, int block, int nt_total, int nsplit,
                         hipStream_t s);
bool stream_variant_exists(tsmm_dtype dt, int KC, int NT, int RT, bool vec, int cm);

// op N, split-bf16 (terms 2 or 3 of binary32 A and B; products 3 or 6) or
// plain bf16 inputs (terms == 1).
hipError_t launch_splitbf16(tsmm_dtype dt, int KC, int NT, int RT, int products, bool il, const void *A,
                            const void *Bfrag, const int32_t *exps, void *C, int64_t m, int64_t n,
                            int64_t k, double alpha, double beta, int64_t grid, int block, int nt_total,
                            int nsplit, hipStream_t s);
bool splitbf16_variant_exists(tsmm_dtype dt, int KC, int NT, int RT, int products, bool il);

// Packed A: alpha*A into `out` (terms 0: dense row-major of the input type;
// terms 2 / 3: bfloat16 planes of RN32(alpha*A), presplit layout).
hipError_t launch_pack_a(tsmm_dtype dt, int terms, const void *A, int64_t lda, void *out, int64_t m, int64_t k,
                         double alpha, hipStream_t s);
// The split-bf16 kernel on a pre-split A (products 3 or 6; alpha folded in
// at pack time, so the epilogue takes alpha = 1).
hipError_t launch_splitbf16_presplit(int products, int KC, int NT, int RT, bool il, const void *planes,
                                     const void *Bfrag,
                                     const int32_t *exps, void *C, int64_t m, int64_t n, int64_t k, double beta,
                                     int64_t grid, int block, int nt_total, int nsplit, hipStream_t s);
bool splitbf16_presplit_exists(int products, int KC, int NT, int RT, bool il);

// op N binary64 on the vector ALU: NB columns per wavefront (16, 32),
// B row-major; requires n % NB == 0 and k % 8 == 0.  grid = 64-row tiles
// walked by each column-group block.
hipError_t launch_valu64(int NB, const double *A, const double *B, double *C, int64_t m, int64_t n, int64_t k,
                         double alpha, double beta, int64_t grid, hipStream_t s);
bool valu64_variant_exists(int NB);

// op T, split-k: pass 1 writes P partial m x n sums, pass 2 reduces them in
// ascending order and applies the epilogue.
hipError_t launch_splitk(int MT, int NT, int RG, const double *A, const double *B, double *W,
                         double *C, int64_t K, int64_t m, int64_t n, int P, double alpha,
                         double beta, int block, hipStream_t s);
bool splitk_variant_exists(int MT, int NT, int RG);

// op N, long k: packed B (16x16x4 fragment order over KCimg = a multiple of
// kSlabK) streamed through LDS in k-slabs, splitk parts of the k range
// (W: splitk * ceil(m/16) * NT * 64 * 4 binary64 partials when splitk > 1,
// then an ordered second pass).
hipError_t launch_slab(tsmm_dtype dt, int NT, int RT, bool vec, bool il, const void *A, const void *Bf, void *C,
                       double *W, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldc, int KCimg, double alpha,
                       double beta, int splitk, int64_t grid, hipStream_t s);
bool slab_variant_exists(tsmm_dtype dt, int NT, int RT, bool vec, bool il);
int slab_rows(int RT);  // rows of one work item (four wavefronts of RT 16-row tiles)

// Column-major operands: packed B (scalar k-slot mapping, plain column
// order, nt_total column tiles) times column-major A into column-major C;
// m a multiple of the vector width, A and C 16-byte aligned.
// NT column tiles per wavefront, NG column groups inside a workgroup.
// lda, ldc: column strides of A and C (>= m, multiples of the vector width).
hipError_t launch_colmajor(tsmm_dtype dt, int KC, int NT, int NG, const void *A, const void *Bf, void *C, int64_t m,
                           int64_t n, int64_t k, int64_t lda, int64_t ldc, double alpha, double beta, int64_t grid,
                           int nt_total, int nsplit, hipStream_t s);
bool colmajor_variant_exists(tsmm_dtype dt, int KC, int NT, int NG);

// Batched persistent launch: workgroup w runs work tiles
// [wg_begin[w], wg_begin[w+1]) of the instance sequence described by
// inst_start (prefix counts of work tiles).  lds_bytes: the largest packed
// B of the batch (batched_lds_bytes); prepare_batched must have been called
// with at least that size.  block must be 256.
size_t batched_lds_bytes(tsmm_dtype dt, int KC, int NT);
hipError_t prepare_batched(tsmm_dtype dt, size_t lds_bytes);
// chunk_start: device int64[count + 1], first chunk of each instance (in
// descriptor order); chunk_rows: rows per chunk (a multiple of 16); ctr:
// device int32[2], zero before the first launch (every launch leaves it
// zero again).
hipError_t launch_batched(tsmm_dtype dt, const BatchDesc *desc, const int64_t *chunk_start, int64_t nchunks,
                          int chunk_rows, int32_t *ctr, int64_t grid, int block, size_t lds_bytes,
                          hipStream_t s);

}  // namespace tsmm
