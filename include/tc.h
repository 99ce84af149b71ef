/*
 * tc.h -- C ABI of the transpose-free tensor contraction library (libtc.so)
 * for AMD MI355X (gfx950).
 *
 * The operation (Sec. 4, eq. gen-contraction, with the alpha/beta update of the
 * element-wise matrix product in Sec. 3):
 *
 *     C[idx_C] := alpha * sum_{P} A[idx_A] * B[idx_B] + beta * C[idx_C]
 *
 * Every label appears in exactly two of the three tensors: labels shared by A
 * and C form the bundle I, by B and C the bundle J, by A and B the contracted
 * bundle P.  The contraction is computed as an (m = prod I) x (n = prod J) x
 * (k = prod P) matrix product whose operands are addressed in place through
 * scatter-offset vectors and block strides (Sec. 6.1-6.2, the block-scatter-
 * matrix layout); no transposed copy of any tensor is formed.
 *
 * Conventions shared by every entry point
 *   - Tensor descriptors: ndim in [0, TC_MAX_NDIM]; lens[d] >= 0; strides[d]
 *     are in ELEMENTS (not bytes) and must be > 0 on every dimension of
 *     length > 1 (a stride on a length-0/1 dimension is ignored); idx is an
 *     array of ndim one-byte labels (not necessarily NUL-terminated), unique
 *     within a tensor.  Descriptor arrays are host memory, read during the
 *     call and not retained.
 *   - A, B, C are DEVICE pointers owned by the caller.  A and B are read only;
 *     C must not overlap itself (checked: sorted by stride, each stride must
 *     be >= the previous stride times the previous length) nor overlap A or B
 *     (checked by address ranges).  Outside graph capture every data pointer
 *     the call will read or write is also checked to be memory of the
 *     current device whose allocation holds the tensor's whole element span
 *     (TC_ERR_ARG otherwise, e.g. for a host pointer), so that such a mistake
 *     is reported instead of reaching a kernel.
 *   - beta == 0: C is write-only (NaN/Inf in C are not propagated).
 *     alpha == 0: A and B are not read; C := beta * C.
 *     A length-0 free index makes the call a no-op; a length-0 contracted
 *     index gives C := beta * C.
 *   - dtype: TC_F64 or TC_F32; A, B and C all have that storage type.
 *     mode: TC_NATIVE (multiply-add in the storage type; FP64 accumulates in
 *     FP64, FP32 in FP32) or TC_SPLIT_BF16X3 (TC_F32 only: each operand is
 *     split into bf16 hi + lo, three products hi*hi + hi*lo + lo*hi on bf16
 *     matrix cores, FP32 accumulation).  One split tile configuration (the
 *     "packed split tile", reported with "layout": 4 by tc_plan_describe)
 *     first splits each operand once into hi/lo panels in a device workspace
 *     of (ceil(m/144) + ceil(n/144)) * ceil(k/32) * 18432 bytes, which the
 *     plan owns ("workspace_bytes"): one per (device, stream) the plan runs
 *     on, allocated by the first call on that stream outside graph capture
 *     (TC_ERR_CAPTURE under capture without it; TC_ERR_NOMEM if it cannot be
 *     allocated), freed by tc_plan_destroy.  Calls on one stream are ordered
 *     by the stream; calls on different streams use different workspaces.
 *     A graph captured on a stream uses that stream's workspace, so its
 *     replays must not overlap eager calls of the plan on that stream.  The
 *     tile choice leaves the packed split tile out when its workspace would
 *     exceed 8 GiB (tc_plan_set_tile may still select it).
 *   - stream is a hipStream_t (NULL = the null stream).  Calls are
 *     asynchronous on it; device faults surface at the caller's next
 *     synchronisation.  The results of one plan and one tile configuration
 *     are deterministic (fixed summation order, no atomics on C).
 *   - Return value: TC_OK (0) or a negative TC_ERR_* status.  Entry points
 *     never abort and never throw; tc_last_error() gives a thread-local
 *     message for the last failure on the calling thread.
 */
#ifndef TC_H
#define TC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TC_MAX_NDIM 16

enum {
    TC_OK = 0,
    TC_ERR_NULL = -1,    /* a required pointer is NULL */
    TC_ERR_NDIM = -2,    /* ndim outside [0, TC_MAX_NDIM] */
    TC_ERR_LABEL = -3,   /* label repeated in one tensor, or not in exactly two tensors */
    TC_ERR_EXTENT = -4,  /* negative length, or one label with different lengths */
    TC_ERR_STRIDE = -5,  /* stride <= 0 on a dimension of length > 1 */
    TC_ERR_ALIAS = -6,   /* C overlaps itself, A or B */
    TC_ERR_DTYPE = -7,   /* unknown dtype, or mode not available for dtype */
    TC_ERR_HIP = -8,     /* a HIP runtime call failed (message in tc_last_error) */
    TC_ERR_NOMEM = -9,   /* host or device allocation failed */
    TC_ERR_ARG = -10,    /* other invalid argument (bad tile id, bad count, ...) */
    TC_ERR_CAPTURE = -11 /* work that cannot be recorded in a graph was asked for during capture */
};

enum { TC_F64 = 0, TC_F32 = 1 };
enum { TC_NATIVE = 0, TC_SPLIT_BF16X3 = 1 };

typedef struct tc_plan tc_plan;
typedef struct tc_batch tc_batch;

/*
 * One-shot contraction (Sec. 4 eq. gen-contraction; Sec. 6.2 BSMTC).
 * Builds (or fetches from a process-wide, mutex-guarded cache keyed by the
 * descriptors, dtype and mode) a plan and executes it on `stream`.  The first
 * call for a descriptor set on a device uploads the plan's offset vectors with
 * a synchronous copy, so a first call must not happen under graph capture
 * (TC_ERR_CAPTURE); use tc_plan_create + tc_plan_upload beforehand instead.
 * Cached plans live until the process ends, with their device vectors and,
 * for the packed split tile, their split panels (one set per stream used).
 */
int tc_contract(double alpha,
                const void* A, int ndim_A, const int64_t* lens_A, const int64_t* strides_A, const char* idx_A,
                const void* B, int ndim_B, const int64_t* lens_B, const int64_t* strides_B, const char* idx_B,
                double beta,
                void* C, int ndim_C, const int64_t* lens_C, const int64_t* strides_C, const char* idx_C,
                int dtype, int mode, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * contraction as tc_contract, with the same arguments, meaning and errors,
 * but it allocates nothing on the device and copies nothing from the host.
 * The plan is built on the host (and kept in a host-side cache), and its
 * offset and block-stride vectors are written by a small kernel on `stream`
 * into a static device array of TC_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends; the contraction kernel then
 * reads them from there.  A problem whose vectors need more than that
 * (about 2 (m + n + k) offsets of 4 bytes, 8 with 64-bit offsets, each vector
 * rounded up to 256 bytes) is refused with TC_ERR_ARG before any launch.
 * Every call on a GPU reuses that GPU's array and it keeps the last call's
 * contents: calls that may overlap in time on one GPU (other streams, other
 * threads) race and must be serialised by the caller; calls on one stream
 * are ordered.  Where tc_contract would run the packed split tile, which
 * needs a workspace, this entry point runs the split tile of the same sizes
 * that splits in its own producer waves (the same bits, slower).
 */
#define TC_NOALLOC_SCRATCH_BYTES (8u << 20)
int tc_contract_noalloc(double alpha,
                        const void* A, int ndim_A, const int64_t* lens_A, const int64_t* strides_A, const char* idx_A,
                        const void* B, int ndim_B, const int64_t* lens_B, const int64_t* strides_B, const char* idx_B,
                        double beta,
                        void* C, int ndim_C, const int64_t* lens_C, const int64_t* strides_C, const char* idx_C,
                        int dtype, int mode, void* stream);

/*
 * Plan creation (host only; no GPU call).  Validates the descriptors (the
 * rules above), groups the labels into I, J, P (Sec. 4), orders them with the
 * reordering heuristic of Sec. 7.3 (drop length-1 dimensions; sort I and J by
 * C stride; swap the operands when C's unit stride lies in J; order P by the
 * stride of the operand whose unit-stride index lies in P, ties to A; fold
 * dimensions contiguous in every tensor holding them), builds the six scatter
 * vectors and the block-stride vectors at the tile sizes of the chosen tile
 * configuration (Sec. 6.1-6.3).  On success *plan owns host memory and, after
 * the first upload, one device buffer per device; free it with
 * tc_plan_destroy.  On failure *plan is set to NULL.
 */
int tc_plan_create(tc_plan** plan,
                   int ndim_A, const int64_t* lens_A, const int64_t* strides_A, const char* idx_A,
                   int ndim_B, const int64_t* lens_B, const int64_t* strides_B, const char* idx_B,
                   int ndim_C, const int64_t* lens_C, const int64_t* strides_C, const char* idx_C,
                   int dtype, int mode);

/* Copy the plan's offset and block-stride vectors to the current device
 * (synchronous; not allowed under graph capture).  Idempotent per device. */
int tc_plan_upload(tc_plan* plan);

/* Execute a plan on device data (Sec. 6.2 BSMTC as one kernel launch: gather
 * of A and B slivers into LDS through the offset vectors, matrix-core
 * micro-kernel, alpha/beta scatter-store of C tiles; the packed split tile
 * adds a split-and-pack launch before it, Sec. 6.1's packing done once for
 * the whole operand).  Safe to record into a hipGraph once the plan has been
 * uploaded to the capturing device (and, for the packed split tile, has run
 * once on the capturing stream). */
int tc_plan_execute(const tc_plan* plan, double alpha, const void* A, const void* B, double beta, void* C,
                    void* stream);

/*
 * The pack and store stages of tc_plan_execute run alone, so that their
 * memory traffic can be measured (the paper's scatter packing, Sec. 6.1, with
 * the block strides of Sec. 6.2, and the scatter of the C tiles):
 *  - tc_plan_pack gathers operand `operand` (0: the plan's A, 1: its B) from
 *    `src` (laid out as that operand's descriptor says) with the
 *    contraction's own gather code and writes it to `dst` as a tile-panel
 *    matrix: with R the tile edge along the operand's free bundle (MT for the
 *    rows m of the operand that plays X, NT for the columns n of the other),
 *    KT the tile's k depth, r the free index (m or n) and p the contracted
 *    index (k) in the plan's order,
 *        dst[((r / R) * ceil(k / KT) + p / KT) * KT * R + (p % KT) * R + r % R]
 *          = operand[element (r, p)],
 *    and 0 in the padding past the last r and p.  tc_plan_pack_elements
 *    gives the number of elements dst must hold (0 when k or a free extent is
 *    0).  In TC_SPLIT_BF16X3 plans the FP32 elements are gathered unsplit.
 *  - tc_plan_store writes an m x n column-major matrix `src` (src[i + m j],
 *    i over the plan's I order, j over its J order) into C with the
 *    contraction's tile store: C[rscat_C[i] + cscat_C[j]] = alpha src[i + m j]
 *    + beta C[...] (C not read when beta = 0).
 * Both are asynchronous on `stream`, allocate nothing once the plan's vectors
 * are on the device, and check their data pointers as tc_plan_execute does
 * (dst must not overlap src, C not src: TC_ERR_ALIAS).
 */
int tc_plan_pack_elements(const tc_plan* plan, int operand, int64_t* elems);
int tc_plan_pack(const tc_plan* plan, int operand, const void* src, void* dst, void* stream);
int tc_plan_store(const tc_plan* plan, double alpha, const void* src, double beta, void* C, void* stream);

/* Free a plan and its device buffers (NULL is accepted).  The caller must
 * make sure no launch using the plan is still running. */
int tc_plan_destroy(tc_plan* plan);

/*
 * JSON description of a plan, for inspection and tests (host only): bundles
 * in planned order with lengths and strides, whether A and B were swapped,
 * m, n, k, tile configuration (with its "layout" and the device workspace it
 * needs, "workspace_bytes"), the lane-fast dimension of each operand,
 * counts of constant-stride blocks, and (for problems with at most
 * `TC_DESCRIBE_MAX_VECTOR` entries per vector) the scatter and block-stride
 * vectors.  Writes at most len bytes including the NUL; returns the full
 * length needed (excluding NUL), or a negative status.
 */
#define TC_DESCRIBE_MAX_VECTOR 4096
int tc_plan_describe(const tc_plan* plan, char* buf, size_t len);

/* Number of compiled tile configurations for (dtype, mode), and their shapes.
 * tile id -> MT x NT x KT and number of waves per workgroup. */
int tc_tile_count(int dtype, int mode);
int tc_tile_info(int dtype, int mode, int tile, int* MT, int* NT, int* KT, int* waves);

/* Force a tile configuration on a plan (rebuilds its block-stride vectors;
 * drops its device copies, so upload again before capture). */
int tc_plan_set_tile(tc_plan* plan, int tile);
int tc_plan_get_tile(const tc_plan* plan);

/*
 * Autotuner: time every compiled tile configuration of the plan on the
 * caller's data (reps launches each after one warm-up, hipEvent timing on
 * `stream`) and keep the fastest in the plan and in a process-wide cache keyed
 * by the plan's shape signature (bundle lengths, strides, dtype, mode); plans
 * created later with the same signature start from the cached choice.  C is
 * overwritten with alpha=1, beta=0 results: pass a scratch tensor laid out
 * like C.  Synchronises `stream`.  *best_ms receives the best time (may be NULL).
 */
int tc_plan_autotune(tc_plan* plan, const void* A, const void* B, void* C_scratch, int reps, void* stream,
                     double* best_ms);

/*
 * Batched contractions in persistent kernel launches (many independent
 * contractions of uneven sizes and index permutations).  tc_batch_create
 * plans every problem (all with the same dtype and mode), uploads one
 * descriptor table plus all offset vectors to the current device
 * (synchronous), and binds the given device pointers and scalars: problem i
 * is C_i := alpha[i] * A_i . B_i + beta[i] * C_i with plans[i].  The plans
 * are only read during the call.  tc_batch_execute then issues one persistent
 * launch per tile class present (see tc_batch_info) whose workgroups walk a
 * flattened list of (problem, tile) work items; it makes no allocation and no
 * host-device copy, so it may be recorded in a hipGraph and replayed.  All
 * problems run inside the same launches, so no C_i may overlap another C_j
 * or an operand A_j, B_j that problem j reads (checked at creation by
 * address ranges: TC_ERR_ALIAS).
 */
int tc_batch_create(tc_batch** batch, int count, const tc_plan* const* plans, const double* alpha,
                    const void* const* A, const void* const* B, const double* beta, void* const* C);
int tc_batch_execute(const tc_batch* batch, void* stream);
int tc_batch_destroy(tc_batch* batch);

/* One problem of tc_contract_batched: the arguments of tc_contract, with the
 * same meaning, layout and ownership. */
typedef struct tc_problem {
    double alpha;
    const void* A;
    int ndim_A;
    const int64_t* lens_A;
    const int64_t* strides_A;
    const char* idx_A;
    const void* B;
    int ndim_B;
    const int64_t* lens_B;
    const int64_t* strides_B;
    const char* idx_B;
    double beta;
    void* C;
    int ndim_C;
    const int64_t* lens_C;
    const int64_t* strides_C;
    const char* idx_C;
} tc_problem;

/* One-shot batched contraction (the definition of Sec. 4 for each problem):
 * plans every problem through the same plan cache as tc_contract, builds a
 * batch of them (as tc_batch_create), runs it on `stream` (as
 * tc_batch_execute), waits for the stream and frees the batch.  Synchronous,
 * and it allocates and uploads the batch tables on every call: for repeated
 * batches or graph capture, build a batch once with tc_batch_create and
 * replay tc_batch_execute.  count = 0 does nothing; TC_ERR_NULL for a NULL
 * problem array with count > 0, TC_ERR_ARG for count < 0 or a stream under
 * graph capture; otherwise the
 * checks and errors of tc_contract and tc_batch_create (mixed dtypes cannot
 * occur: dtype and mode apply to every problem). */
int tc_contract_batched(int count, const tc_problem* problems, int dtype, int mode, void* stream);
/* Work-item count, the tile configuration (-1: per-problem classes) and the
 * largest persistent grid of the batch.  By default every problem runs with
 * the tile configuration the planner's cost model picks for it alone among
 * the regular and regular-grid specialised-wave layouts (0 and 3);
 * problems of one class share one persistent launch (so a batch issues at
 * most one launch per configuration, the class with the most work first),
 * and each of its workgroups runs a fixed list of (problem, tile) work items
 * built on the host longest-processing-time-first (the cost of a tile is its
 * k plus three stages).  The regular layouts and the regular-grid
 * specialised-wave layout of a dtype share KT and sum every output element
 * in the same order as tc_plan_execute with any of them (bitwise equal); the
 * specialised-wave pinwheel (layout 2) sums its centre fragment in another
 * order. */
int tc_batch_info(const tc_batch* batch, int64_t* work_items, int* tile, int* grid);
/* The tile configuration problem `problem` (its index in tc_batch_create's
 * arrays) runs with under the batch's current setting, or -1 when the problem
 * launches no work (an empty free extent).  TC_ERR_ARG for an index out of
 * range. */
int tc_batch_problem_tile(const tc_batch* batch, int problem, int* tile);
/* Set one tile configuration for the whole batch (any layout but the
 * all-compute pinwheel, layout 1), or -1 for per-problem classes; re-uploads
 * the work table (synchronous, not during capture). */
int tc_batch_set_tile(tc_batch* batch, int tile);
/* Autotuner for batches: times the whole batch (reps runs after one warm-up,
 * hipEvent timing on `stream`) with per-problem classes and under every
 * single tile configuration a batch runs, and keeps the fastest.  Runs the batch
 * (1 + reps) times per candidate, so outputs with beta != 0 are updated
 * repeatedly: tune on scratch outputs.  Synchronises `stream`.  *best_ms may
 * be NULL. */
int tc_batch_autotune(tc_batch* batch, int reps, void* stream, double* best_ms);

/*
 * Building blocks of the block-scatter-matrix layout, exported for tests and
 * for inspection (host only, Sec. 6.1-6.2):
 *  - tc_scatter_vector: out[x] = sum_d x_d * strides[d] for every linear
 *    index x of the bundle (lens, in the given order, first index fastest);
 *    out has prod(lens) entries.
 *  - tc_block_strides: out[i] (ceil(len/b) entries) = s > 0 when
 *    scat[j] - scat[j-1] == s for every j of block i (i*b < j < min(len,(i+1)b)),
 *    else 0; a block of one entry has stride 1.
 */
int tc_scatter_vector(int ndim, const int64_t* lens, const int64_t* strides, int64_t* out);
int tc_block_strides(const int64_t* scat, int64_t len, int64_t b, int64_t* out);

/*
 * Strided permute-copy, the explicit transposition of the
 * transpose-transpose-GEMM-transpose method (Sec. 5, fig. TTGT) that the contraction
 * above avoids; it lets that method be timed on the same device.
 * dst[x . dst_strides] = src[x . src_strides] for every multi-index x over
 * lens (ndim dimensions, ndim in [0, TC_MAX_NDIM]; strides in elements, > 0 on
 * dimensions of length > 1).  src and dst are device pointers owned by the
 * caller, of the storage type `dtype` (TC_F64 or TC_F32); element bits are
 * copied unchanged.  dst must not overlap src, and distinct x must reach
 * distinct dst elements; neither is checked (as with memcpy).  Outside graph
 * capture both pointers are checked to be memory of the current device
 * holding the whole element span.  Asynchronous on `stream`; an empty index
 * space is a no-op.  Errors: TC_ERR_NDIM, TC_ERR_NULL, TC_ERR_DTYPE,
 * TC_ERR_EXTENT (negative length), TC_ERR_STRIDE, TC_ERR_ARG (not device
 * memory of the current device), TC_ERR_HIP (launch failure).
 */
int tc_permute(const void* src, void* dst, int ndim, const int64_t* lens, const int64_t* src_strides,
               const int64_t* dst_strides, int dtype, void* stream);

const char* tc_status_string(int status);
const char* tc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
