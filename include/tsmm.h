/*
 * tsmm.h -- pre-packed tall-and-skinny matrix multiply on MI355X (gfx950).
 *
 * The operation is the GEMM contract of AutoTSMM (Sec. I, Eq. (1)):
 *
 *     C = alpha * op(A) * B + beta * C
 *
 * for the tall-and-skinny case, where one dimension of an operand is far
 * smaller than the other (Sec. I).  The library follows the paper's split
 * of the problem (Algorithm 1, Sec. III):
 *
 *   tsmm_pack     packs the small operand once into a reusable handle
 *                 (the PACKB step of Algorithm 1; the pre-pack module of
 *                 Sec. IV-A.3);
 *   tsmm_plan     builds an execution plan for a shape from the tile table
 *                 written by the install-time autotuner (the runtime stage
 *                 of Sec. III: cache-blocked designer, multi-thread
 *                 optimizer, performance evaluator; Eqs. (2)-(3));
 *   tsmm_execute  runs the multiply (the COMPUTE step of Algorithm 1);
 *   tsmm_pack_a / tsmm_execute_packed_a  pack a big operand that is reused
 *                 across calls (the PACKA step, alpha folded in) and
 *                 multiply with it.
 *
 * Conventions shared by every entry point:
 *   - Matrices are dense and row-major (TSMM_COLMAJOR: column-major);
 *     tsmm_execute_ld takes leading dimensions of A and C, every other
 *     entry point the natural ones.
 *   - op N:  A is m x k, B is k x n, C is m x n:      C = a*A*B   + b*C.
 *     op T:  A is k x m, B is k x n, C is m x n:      C = a*A^T*B + b*C,
 *            the reduction shape over a long shared dimension k.
 *   - Every matrix pointer passed to tsmm_pack / tsmm_execute* is a DEVICE
 *     pointer owned by the caller; size and shape arrays passed to the plan
 *     calls are HOST pointers.  C must not alias A or B.
 *   - alpha and beta are binary64.  The epilogue is evaluated in binary64 as
 *     RN(RN(alpha*acc) + RN(beta*c)), with no fused multiply-add, and rounded
 *     once more to C's type.  beta == 0 never reads C (NaN in C is safe);
 *     alpha == 0 never reads A or the packed operand; k == 0 gives
 *     C = beta*C; m == 0 or n == 0 launches nothing.
 *   - Element types: TSMM_F64 inputs give a binary64 C; TSMM_F32 inputs give
 *     a binary32 C; TSMM_BF16 inputs give a binary32 C.
 *   - Every call returns a tsmm_status and never aborts.  Arguments are
 *     validated on the host before any HIP call, so invalid arguments are
 *     reported the same way on hosts without a GPU.  tsmm_last_error()
 *     returns a thread-local text with the detail of the last failure.
 *   - tsmm_pack and tsmm_execute* are asynchronous on the HIP stream given
 *     (NULL = the null stream); device faults surface at the caller's next
 *     synchronisation.
 *   - Handles are opaque host objects; the destroy calls accept NULL.
 *     Plans and packed handles are immutable once built, except for the
 *     stream / workspace / tile setters, which a caller must not race with
 *     an execute on the same plan.
 */
#ifndef TSMM_H
#define TSMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tsmm_status {
    TSMM_SUCCESS = 0,
    TSMM_ERROR_INVALID_VALUE = 1,  /* bad pointer, negative size, bad enum */
    TSMM_ERROR_SHAPE_MISMATCH = 2, /* plan and packed operand disagree      */
    TSMM_ERROR_NOT_SUPPORTED = 3,  /* shape/type/mode outside the library   */
    TSMM_ERROR_TABLE = 4,          /* tile table unreadable (strict mode)   */
    TSMM_ERROR_OUT_OF_MEMORY = 5,  /* device or host allocation failed      */
    TSMM_ERROR_NO_DEVICE = 6,      /* no usable gfx950 device               */
    TSMM_ERROR_HIP = 7             /* a HIP runtime call failed             */
} tsmm_status;

typedef enum tsmm_dtype {
    TSMM_F64 = 0,  /* binary64 in, binary64 out                       */
    TSMM_F32 = 1,  /* binary32 in, binary32 out                       */
    TSMM_BF16 = 2  /* bfloat16 in, binary32 accumulation and output   */
} tsmm_dtype;

typedef enum tsmm_layout {
    TSMM_OP_N = 0,     /* C = alpha*A*B + beta*C,   A m x k, all row-major */
    TSMM_OP_T = 1,     /* C = alpha*A^T*B + beta*C, A k x m, all row-major */
    TSMM_COLMAJOR = 2  /* C = alpha*A*B + beta*C with A (m x k), B (k x n)
                          and C (m x n) column-major (element (i, j) at
                          i + j * rows), the layout of the paper's analysis
                          (Sec. IV-A); binary64 / binary32, NATIVE mode.
                          Also the row-major small-A times wide-B
                          orientation: row-major C = A B is column-major
                          C^T = B^T A^T on the same memory, i.e. this
                          layout with (m, n, k) = (n, m, k), the wide B as
                          A, the small A packed as B (k x m)         */
} tsmm_layout;

/* Arithmetic used for TSMM_F32 inputs (other types accept NATIVE only).
 *   NATIVE  binary32 matrix-core products, binary32 accumulation.
 *   BF16X3  two-term bfloat16 split of both operands (x = hi + mid + r),
 *           products hi*hi + hi*mid + mid*hi, binary32 accumulation.
 *   BF16X6  three-term split (x = hi + mid + lo, exact for normal binary32),
 *           the six products with term order i + j <= 2, binary32
 *           accumulation.  The packed operand carries a power-of-two scale
 *           per column of B that the binary64 epilogue undoes. */
typedef enum tsmm_mode {
    TSMM_MODE_NATIVE = 0,
    TSMM_MODE_BF16X3 = 1,
    TSMM_MODE_BF16X6 = 2
} tsmm_mode;

/* Kernel families a tile can name (tsmm_tile.kernel). */
typedef enum tsmm_kernel {
    TSMM_KERNEL_AUTO = 0,     /* let the plan choose                          */
    TSMM_KERNEL_SIMPLE = 1,   /* any shape: one thread per output, no packing
                                 assumptions; the conservative fallback        */
    TSMM_KERNEL_STREAM = 2,   /* op N streaming: packed B fragments, A rows
                                 streamed through registers, matrix cores     */
    TSMM_KERNEL_SPLITK = 3,   /* op T: split-k partials + ordered reduce      */
    TSMM_KERNEL_SPLITBF16 = 4, /* op N, TSMM_F32 in BF16X3 / BF16X6 mode and
                                  TSMM_BF16 inputs: bf16 matrix cores          */
    TSMM_KERNEL_VALU64 = 5,    /* op N binary64 on the vector ALU: one row per
                                  lane, k % 8 == 0, n a multiple of the
                                  column block                               */
    TSMM_KERNEL_WIDE = 6,      /* op N TSMM_F32 (native, BF16X3, BF16X6) with
                                  n = 128 or 256, k <= 256, k % 8 == 0: a
                                  wavefront owns whole rows of C in 32x32
                                  matrix-core accumulators, packed B streams
                                  through LDS in 32-row slabs; A and C 16-byte
                                  aligned                                    */
    TSMM_KERNEL_BATCHED = 7,   /* batched plans only: the persistent launch
                                  over chunks of instance rows               */
    TSMM_KERNEL_SLAB = 8,      /* op N TSMM_F64 / TSMM_F32 (native) with a long
                                  k (beyond 256, up to 2^20; also any k class
                                  of 32 and more), n <= 256: a wavefront keeps
                                  its rows' accumulators for all n columns,
                                  packed B streams through LDS in 32-k slabs;
                                  splitk cuts the k range (binary64 partials,
                                  ordered second pass)                       */
    TSMM_KERNEL_COLMAJOR = 9   /* TSMM_COLMAJOR, TSMM_F64 / TSMM_F32, k and
                                  n <= 256, m a multiple of the 16-byte vector
                                  width: packed B as the matrix-core product's
                                  first operand, A columns streamed as the
                                  second; A and C 16-byte aligned          */
} tsmm_kernel;

/* One entry of the tile table: the register/LDS blocking and launch shape
 * of a plan (the analogue of the paper's m_t / m_c / k_c / n_c blocking and
 * thread split, Sec. IV-A.1 and IV-A.2).  Zero in a field means "default". */
typedef struct tsmm_tile {
    int32_t kernel;        /* tsmm_kernel                                   */
    int32_t rows_per_wave; /* 16-row tiles a wavefront owns at a time: 1,2,4,
                              8 (TSMM_KERNEL_VALU64: C columns per
                              wavefront, 16 or 32; TSMM_KERNEL_WIDE:
                              32-row tiles, 2, or 4 for native mode at
                              n = 128, with 4 wavefronts; 1 with 8;
                              TSMM_KERNEL_COLMAJOR: column groups
                              inside a workgroup, 1 or 2)               */
    int32_t waves_per_wg;  /* wavefronts per workgroup: 1, 2 or 4
                              (TSMM_KERNEL_WIDE: 4, one per SIMD, or 8,
                              two per SIMD)                             */
    int32_t wg_per_cu;     /* resident workgroups per compute unit (grid =
                              CUs * wg_per_cu, capped by the work): 1..32   */
    int32_t splitk;        /* op T: number of partial sums P (1..65536);
                              TSMM_KERNEL_SLAB: parts of the k range        */
    int32_t nsplit;        /* op N: column groups sharing one row block     */
    int32_t chunk_rows;    /* batched plans: rows per work item for an
                              instance whose rows (of A plus of C) take 256
                              bytes, a power of two in 256..65536 (0 =
                              default); each instance scales it by 256 / its
                              row bytes (power of two at or below, within
                              256..65536), so that work items move about the
                              same bytes; 0 elsewhere                       */
} tsmm_tile;

/* Device properties the planner uses; tsmm_plan reads them from the current
 * HIP device.  tsmm_plan_with_caps takes them from the caller instead, so
 * that plan arithmetic can be checked without a GPU. */
typedef struct tsmm_device_caps {
    int32_t compute_units;    /* 256 on MI355X                      */
    int32_t lds_bytes_per_cu; /* 163840 on gfx950                   */
    int32_t gcn_arch;         /* 950 for gfx950                     */
} tsmm_device_caps;

typedef struct tsmm_packed_s *tsmm_packed_t;
typedef struct tsmm_plan_s *tsmm_plan_t;
typedef struct tsmm_graph_s *tsmm_graph_t;

/* ------------------------------------------------------------------ errors */

/* Static text for a status code; never NULL. */
const char *tsmm_status_string(tsmm_status status);

/* Thread-local detail of the last failing call on this thread ("" if none).
 * The pointer stays valid until the next tsmm_* call on the same thread. */
const char *tsmm_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t tsmm_version(void);

/* The key lines a tile table must carry to be used (the install-time stage
 * of Sec. III: the table records timings taken on one device, runtime and
 * library, and is only valid there).  Writes three lines,
 *     key arch gfx<N>\nkey hip <hipRuntimeGetVersion()>\nkey libtsmm <tsmm_version()>\n
 * into buf (at most len bytes including the terminating NUL) for
 * architecture gcn_arch (950 for gfx950), or for the current HIP device
 * when gcn_arch is 0.  tsmm_plan ignores a table whose key lines are
 * missing or name another runtime or library version (and applies its
 * entries only to plans for the keyed architecture); it then uses built-in
 * tiles, or fails with TSMM_ERROR_TABLE when the environment variable
 * TSMM_STRICT_TABLE is set.
 * Errors: INVALID_VALUE (NULL buf, len too small, negative gcn_arch),
 * NO_DEVICE (gcn_arch 0 without a usable device). */
tsmm_status tsmm_table_key(int32_t gcn_arch, char *buf, size_t len);

/* -------------------------------------------------------------------- pack */

/* Pack the small operand B once, for reuse by any number of executes
 * (Algorithm 1, PACKB with unit scale; Sec. II-C and IV-A.3: packing is
 * done apart from, and before, the computation so that its cost is paid
 * once).
 *   B       device pointer, row-major k x n of `dtype` (bfloat16 as raw
 *           16-bit patterns).  Read asynchronously on `stream`; the caller
 *           keeps it alive until the stream has passed the pack.
 *   k, n    B's shape, k >= 0, n >= 0.
 *   layout  TSMM_OP_N: B is the small operand and is rearranged into the
 *           matrix-core fragment order of the execute kernels (and, for the
 *           BF16X3 / BF16X6 modes, split into bfloat16 planes with a
 *           power-of-two scale per column).  TSMM_OP_T: both operands are
 *           tall and nothing is copied: the handle refers to B itself, which
 *           the caller keeps alive and unchanged while the handle is used.
 *           TSMM_COLMAJOR: B is column-major k x n (binary64 / binary32,
 *           NATIVE), packed into the same fragment order.
 *   mode    tsmm_mode; only TSMM_F32 accepts a mode other than NATIVE.
 *   stream  hipStream_t or NULL.
 *   out     receives the handle (host object owning device memory that the
 *           library allocates); free it with tsmm_packed_destroy after the
 *           last execute that uses it has completed.
 * Errors: INVALID_VALUE (NULL out, NULL B with k*n > 0, negative sizes, bad
 * enum), NOT_SUPPORTED (mode not valid for dtype), OUT_OF_MEMORY, HIP. */
tsmm_status tsmm_pack(const void *B, int64_t k, int64_t n, tsmm_layout layout,
                      tsmm_dtype dtype, tsmm_mode mode, void *stream,
                      tsmm_packed_t *out);

/* Bytes of device memory held by a packed handle. */
tsmm_status tsmm_packed_bytes(tsmm_packed_t packed, size_t *bytes);

/* Write B back from a packed handle (row-major k x n, the packed type; for
 * the split modes the binary32 value (sum of the planes) * 2^e_j).  Used to
 * check that packing loses nothing.  B_out is a device pointer of k*n
 * elements.  Asynchronous on `stream`. */
tsmm_status tsmm_unpack(tsmm_packed_t packed, void *B_out, void *stream);

/* Copy the bfloat16 planes and column exponents of a split-mode handle:
 * planes_out receives terms*k*n uint16 values, plane t of element (i, j) at
 * t*k*n + i*n + j (the split of B[i][j] * 2^-e_j); exps_out receives n
 * int32 values e_j.  Device pointers; asynchronous on `stream`.
 * NOT_SUPPORTED for a handle that is not in a split mode. */
tsmm_status tsmm_packed_split_planes(tsmm_packed_t packed, void *planes_out,
                                     void *exps_out, void *stream);

void tsmm_packed_destroy(tsmm_packed_t packed);

/* Pack the big operand A once, for a caller that multiplies the same A by
 * many B (Algorithm 1, PACKA: A is scaled by alpha as it is packed; the
 * reused-operand case of Sec. II-C, e.g. weights against im2col panels).
 *   A       device pointer, row-major m x k with row stride lda (>= k), of
 *           `dtype` (binary64 or binary32).  Read asynchronously on `stream`.
 *   mode    NATIVE: the handle holds RN(alpha*a) in the input type (product
 *           in binary64), dense row-major; executes read it as a fresh A
 *           with alpha = 1, so nothing changes per call but the scaling.
 *           BF16X3 / BF16X6 (binary32, k <= 256): the handle holds
 *           RN32(alpha*a) already split into its 2 / 3 bfloat16 terms (the
 *           residual split of those modes), one plane per term, rows padded
 *           to a multiple of 8 and the row count to a multiple of 16 with
 *           zeros: executes on the split-bf16 kernel load the terms instead
 *           of splitting A on every call (2 bytes of traffic per term and
 *           element instead of 4).  When k % 8 == 0 it also holds
 *           RN32(alpha*a) itself (m x k binary32), which executes of plans
 *           that run the wide kernels read instead: those split in the
 *           shadow of their products, into the same terms.
 *   alpha   folded into the handle; alpha = 0 makes executes compute
 *           beta*C without reading A or B (reference-BLAS convention).
 *   out     receives the handle (owns device memory; free it with
 *           tsmm_packed_destroy after the last execute that uses it).
 *           tsmm_packed_bytes reports its size; it cannot be unpacked and is
 *           refused where a packed B is expected.
 * Errors: INVALID_VALUE (NULL out, NULL A with m*k > 0, negative sizes,
 * lda < k, bad enum), NOT_SUPPORTED (bfloat16 A, split mode with a type
 * other than binary32 or k > 256), OUT_OF_MEMORY, HIP. */
tsmm_status tsmm_pack_a(const void *A, int64_t m, int64_t k, int64_t lda, tsmm_dtype dtype,
                        tsmm_mode mode, double alpha, void *stream, tsmm_packed_t *out);

/* -------------------------------------------------------------------- plan */

/* Build an execution plan for one shape (the runtime stage of Sec. III):
 * the tile comes from the tile table (TSMM_TILE_TABLE, else tile_table.txt
 * beside the library) keyed by layout, dtype, mode and size classes, else
 * from built-in defaults; it is then checked against the device's limits
 * (LDS capacity per compute unit, the analogue of Eq. (2); register budget,
 * the analogue of Eq. (3)) and the launch geometry is derived.
 *   m, n, k  op N: A m x k, B k x n.  op T: A k x m, B k x n.  All >= 0.
 * The plan starts in TSMM_MODE_NATIVE on the null stream with no
 * workspace.  Host only: no device memory is touched.
 * Errors: INVALID_VALUE, NOT_SUPPORTED, NO_DEVICE (tsmm_plan only). */
tsmm_status tsmm_plan(int64_t m, int64_t n, int64_t k, tsmm_layout layout,
                      tsmm_dtype dtype, tsmm_plan_t *out);

tsmm_status tsmm_plan_with_caps(int64_t m, int64_t n, int64_t k,
                                tsmm_layout layout, tsmm_dtype dtype,
                                const tsmm_device_caps *caps,
                                tsmm_plan_t *out);

/* Select the arithmetic (tsmm_mode) and re-derive the tile for it. */
tsmm_status tsmm_plan_set_mode(tsmm_plan_t plan, tsmm_mode mode);

/* Replace the tile (autotuner and tests).  The tile is validated against
 * the shape and the device limits; INVALID_VALUE / NOT_SUPPORTED if it
 * cannot run.  A batched plan takes kernel TSMM_KERNEL_BATCHED (or AUTO)
 * and only chunk_rows and wg_per_cu may differ from its defaults
 * (wg_per_cu 1, 2 or 4 resident workgroups per compute unit, as far as the
 * LDS holds that many copies of the largest packed B, else INVALID_VALUE;
 * 0 keeps the plan's count, or takes the table's when chunk_rows is 0
 * too); the chunk list is rebuilt on the device (synchronously), so the
 * plan must be idle, and a plan from which a graph was made refuses it
 * (INVALID_VALUE) while the graph exists. */
tsmm_status tsmm_plan_set_tile(tsmm_plan_t plan, const tsmm_tile *tile);
tsmm_status tsmm_plan_get_tile(tsmm_plan_t plan, tsmm_tile *tile);

/* Stream (hipStream_t, NULL = null stream) on which executes are queued. */
tsmm_status tsmm_plan_set_stream(tsmm_plan_t plan, void *stream);

/* Device scratch an execute needs (the op T partial sums: splitk * m * n
 * binary64 values); 0 when none. */
tsmm_status tsmm_plan_workspace_bytes(tsmm_plan_t plan, size_t *bytes);

/* Attach caller-owned device scratch of at least tsmm_plan_workspace_bytes
 * bytes.  Without it, the first execute that needs scratch allocates it
 * and the plan owns it.  Two executes sharing one workspace must not run
 * concurrently. */
tsmm_status tsmm_plan_set_workspace(tsmm_plan_t plan, void *workspace,
                                    size_t bytes);

/* A one-line text description of the plan (kernel, tile, grid; table=0
 * built-in or caller's tile, 1 tile table, 2 runtime evaluator; ran=the
 * kernel family the latest execute ran, "-" before the first: it names the
 * any-shape kernel when operand alignment or strides kept the plan's
 * kernel from running, which TSMM_LOG=1 also reports on stderr); writes at
 * most len bytes including the terminating NUL. */
tsmm_status tsmm_plan_describe(tsmm_plan_t plan, char *buf, size_t len);

/* Runtime stage of the paper's performance evaluator (Sec. III: when the
 * install-time stage has no answer for a shape, candidate strategies are
 * timed at run time and the fastest is kept).  Times each candidate tile of
 * the plan's kernel family (and the wide kernels where they apply) on the
 * caller's operands: one warm-up and `reps` (1..1000) executes with
 * alpha = 1, beta = 0, HIP events on the plan's stream, median.  The
 * fastest tile is set in the plan and remembered for the plan's shape
 * class (the tile-table key) in this process: later tsmm_plan calls of the
 * class start from it (describe: table=2).  C is overwritten (its contents
 * afterwards are A*B); A and C follow tsmm_execute's rules.  The plan may
 * allocate a larger workspace for a candidate.  Synchronous; best_ms
 * (optional) receives the winner's median milliseconds (0 when nothing
 * runs: m, n or k is 0).
 * Errors: INVALID_VALUE (NULL arguments, batched plan, reps), NO_DEVICE
 * (plan built for explicit caps), NOT_SUPPORTED, SHAPE_MISMATCH, HIP; on
 * error the plan keeps its tile. */
tsmm_status tsmm_plan_tune(tsmm_plan_t plan, const void *A, tsmm_packed_t packed, void *C, int reps,
                           double *best_ms);

/* Forget every tile tsmm_plan_tune remembered in this process. */
void tsmm_tune_cache_clear(void);

void tsmm_plan_destroy(tsmm_plan_t plan);

/* ----------------------------------------------------------------- execute */

/* C = alpha * op(A) * B + beta * C with B taken from `packed` (Algorithm 1,
 * COMPUTE; the output line of Algorithm 1).
 *   plan    from tsmm_plan for (m, n, k, layout, dtype); its mode must match
 *           the packed handle's, and the handle's k, n, layout and dtype must
 *           match the plan (SHAPE_MISMATCH otherwise).
 *   A       device pointer, op N: m x k; op T: k x m; row-major.
 *   C       device pointer, m x n row-major, read (if beta != 0) and written.
 * Any alignment of the element type is accepted; the vectorised kernels
 * need 16-byte aligned A (and C, where they store 16-byte vectors) and the
 * plan then runs the any-shape kernel instead (split-bf16 modes report
 * INVALID_VALUE).
 * Asynchronous on the plan's stream.  An execute may be captured in a HIP
 * graph (it launches kernels only: no allocation, copy or memset) once the
 * plan's workspace, if it needs one, is attached or was allocated by an
 * earlier execute; every replay then gives the eager result.
 * Errors: INVALID_VALUE, SHAPE_MISMATCH, OUT_OF_MEMORY (lazy workspace),
 * HIP (launch failure; text in tsmm_last_error). */
tsmm_status tsmm_execute(tsmm_plan_t plan, const void *A, tsmm_packed_t packed,
                         void *C, double alpha, double beta);

/* tsmm_execute for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, natural strides, same kernels and the same results, bit
 * for bit, as tsmm_execute with the same plan.  Split-k plans (op T; k-slab
 * plans with parts of the k range) keep their partial sums in the
 * library's static device scratch instead of a workspace: 32 MiB per
 * device (TSMM_NOALLOC_SCRATCH_BYTES), alive until the process ends, its
 * device address looked up on the first call on each device.  This call
 * never allocates (no hipMalloc, no library allocation); the plan's own
 * workspace is neither used nor created.  Every call on one device shares
 * that scratch and leaves its last contents there (every partial is written
 * before it is read, so nothing needs clearing): calls that overlap in time
 * on one device -- concurrent streams, or host threads -- race and must be
 * ordered by the caller.
 * Errors: as tsmm_execute; NOT_SUPPORTED when the plan needs more scratch
 * than TSMM_NOALLOC_SCRATCH_BYTES (plan with fewer split-k parts, or use
 * tsmm_execute with a workspace); INVALID_VALUE for a batched plan. */
#define TSMM_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
tsmm_status tsmm_execute_noalloc(tsmm_plan_t plan, const void *A, tsmm_packed_t packed, void *C,
                                 double alpha, double beta);

/* tsmm_execute with leading dimensions (strided operands, as in BLAS):
 *   lda  TSMM_OP_N: row stride of A (>= k); TSMM_OP_T: row stride of the
 *        k x m A (>= m); TSMM_COLMAJOR: column stride of A (>= m).
 *   ldc  TSMM_OP_N / TSMM_OP_T: row stride of C (>= n); TSMM_COLMAJOR:
 *        column stride of C (>= m).
 * In elements.  tsmm_execute is this call with the natural strides.  The
 * streaming, k-slab and column-major kernels take strides (vector accesses
 * need the stride to be a multiple of the 16-byte vector width, else the
 * any-shape kernel runs); the other kernels run the any-shape kernel when
 * a stride is not the natural one, and the split-bf16 modes refuse it.
 * Errors: as tsmm_execute; INVALID_VALUE for strides below the natural
 * ones or, in the split-bf16 modes, other than them. */
tsmm_status tsmm_execute_ld(tsmm_plan_t plan, const void *A, int64_t lda, tsmm_packed_t packed,
                            void *C, int64_t ldc, double alpha, double beta);

/* C = A_packed * B + beta*C with A from tsmm_pack_a (alpha was folded in
 * there): the COMPUTE step of Algorithm 1 on two packed operands.  The plan
 * is an op N plan of the same m, k, dtype and mode as packed_a; packed is
 * B packed for that plan; C is row-major m x n (natural stride).
 * NATIVE plans run their own kernel on the packed copy of A.  Split-bf16
 * plans that run a wide kernel (TSMM_KERNEL_WIDE; n = 128 or 256) run it on
 * the handle's RN32(alpha*A) when it holds one (k % 8 == 0); other
 * split-bf16 plans run the split-bf16 kernel on the pre-split terms (the
 * plan's tile when the plan uses that kernel, else its default tile, with
 * fewer rows per wavefront or more column groups where a variant needs
 * them).  For alpha = 1 the result is bitwise that of tsmm_execute with
 * the same kernel and geometry, since the terms are the same values.
 * Asynchronous on the plan's stream.
 * Errors: INVALID_VALUE (NULL argument, packed_a not from tsmm_pack_a,
 * packed not a packed B, C not 4-byte aligned, or in the split modes not
 * 16-byte aligned where C moves in 16-byte vectors: n % 4 == 0 and
 * n > 48), SHAPE_MISMATCH (plan and
 * handles disagree), NOT_SUPPORTED (not an op N plan), HIP. */
tsmm_status tsmm_execute_packed_a(tsmm_plan_t plan, tsmm_packed_t packed_a, tsmm_packed_t packed,
                                  void *C, double beta);

/* ----------------------------------------------------------------- batched */

/* Plan `count` independent op N multiplies that run in ONE persistent
 * launch: instance b is m[b] x k[b] times k[b] x n[b].  Host arrays.  The
 * plan cuts the instances into chunks of rows (sized from chunk_rows, from
 * the tile table's batched entry for the dtype, else 4096; instances of one kernel
 * variant together, longest first) that the launch's workgroups (the
 * table entry's workgroups per compute unit, else one) take from
 * a device counter; the plan owns that counter, which every launch leaves
 * at zero, so the launches (or graph replays) of one plan must not overlap
 * in time.  Results do not depend on which workgroup takes which chunk.
 * dtype: TSMM_F32 (binary32 in/out) or TSMM_BF16 (bfloat16 in, binary32
 * out), NATIVE mode; 1 <= k[b], n[b] <= 128.
 * Errors: INVALID_VALUE, NOT_SUPPORTED, NO_DEVICE, OUT_OF_MEMORY, HIP. */
tsmm_status tsmm_plan_batched(int64_t count, const int64_t *m, const int64_t *n,
                              const int64_t *k, tsmm_dtype dtype,
                              tsmm_plan_t *out);

/* Bind the operands of a batched plan: host arrays of `count` device
 * pointers / handles / scalars.  The descriptor table is copied to the
 * device on the plan's stream from pinned staging memory, so a bind can be
 * captured in a graph.  Every packed[b] must match (k[b], n[b], dtype).
 * A[b] must be 16-byte aligned when k[b] allows vector loads (binary32: k
 * a multiple of 4; bfloat16: of 8) and C[b] when C is stored in 16-byte
 * vectors (n a multiple of 4 and n > 32); INVALID_VALUE otherwise. */
tsmm_status tsmm_batched_bind(tsmm_plan_t plan, const void *const *A,
                              const tsmm_packed_t *packed, void *const *C,
                              const double *alpha, const double *beta);

/* Run every instance of the bound batched plan in one launch on the plan's
 * stream.  If A is not NULL the operands are bound first (as
 * tsmm_batched_bind) when they differ from the bound ones. */
tsmm_status tsmm_execute_batched(tsmm_plan_t plan, const void *const *A,
                                 const tsmm_packed_t *packed, void *const *C,
                                 const double *alpha, const double *beta);

/* Capture the batched launch of a bound plan into a HIP graph once (on a
 * capture stream of its own, after the plan's stream has drained) and
 * instantiate it; launch it any number of times with tsmm_graph_launch on
 * any stream.  The graph reads the plan's descriptor table and work
 * counter when it runs: a later tsmm_batched_bind changes the operands it
 * uses (order the bind and the launches on one stream), and its launches
 * must not overlap those of the plan.  The plan must outlive the graph. */
tsmm_status tsmm_graph_create_batched(tsmm_plan_t plan, tsmm_graph_t *out);
tsmm_status tsmm_graph_launch(tsmm_graph_t graph, void *stream);
void tsmm_graph_destroy(tsmm_graph_t graph);

#ifdef __cplusplus
}
#endif

#endif /* TSMM_H */
