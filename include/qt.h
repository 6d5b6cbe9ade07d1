/*
 * qt.h -- quadtree block-sparse matrix multiply on AMD MI355X (gfx950).
 *
 * C ABI of libqt.so. Every entry point returns a qt_status, never aborts and
 * never lets a C++ exception cross this boundary; on failure the output
 * handle is left NULL, nothing leaks, and qt_last_error() describes the
 * failure (thread-local string).
 *
 * The operation (Rubensson & Rudberg, arXiv:1501.07800):
 *   - A matrix is a sparse quadtree (Sec. 3.1): each internal node has four
 *     children, any of which may be NIL (a zero submatrix that is neither
 *     stored nor addressed); the dimension halves at every level; the lowest
 *     level holds block-sparse leaves (Sec. 4.1): a leaf is an lb x lb grid
 *     of b x b blocks where only nonzero blocks are stored.
 *   - C = A*B follows Algorithm 1 (Sec. 3): NIL times anything is NIL, leaves
 *     are multiplied block by block, and C_mn = A_m1 B_1n + A_m2 B_2n at every
 *     level above (Algorithm 2 gives the sum's structure: a block of C exists
 *     iff at least one product contributes to it).
 *   - Handles are immutable once created, like registered chunks (Sec. 2):
 *     several threads may use one handle as an input at the same time.
 *
 * Conventions shared by all calls:
 *   - `stream` is a hipStream_t (NULL = the default stream). Work is queued
 *     on it; calls return before it completes except where a call says it
 *     synchronizes. Device memory of a handle is allocated stream-ordered on
 *     the stream that created it and released on that stream by qt_free.
 *   - Blocks are row-major inside a block (entry (r, c) at r*b + c).
 *   - Device pointers are HIP device pointers on the current device.
 */
#ifndef QT_H
#define QT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qt_matrix qt_matrix;   /* opaque, immutable after creation */
typedef struct qt_plan qt_plan;       /* opaque batched-multiply plan */

typedef enum {
    QT_OK = 0,
    QT_ERR_ARG = 1,          /* bad pointer, negative size, index out of range */
    QT_ERR_SHAPE = 2,        /* dimensions / block size / leaf size do not fit */
    QT_ERR_DUPLICATE = 3,    /* the same (I, J) block given twice */
    QT_ERR_OOM = 4,          /* a device or host allocation failed */
    QT_ERR_DEVICE = 5,       /* a HIP call or a kernel reported an error */
    QT_ERR_UNSUPPORTED = 6   /* a size or mode the library does not handle */
} qt_status;

typedef enum {
    QT_F64 = 0,              /* fp64 inputs, fp64 MFMA, fp64 C */
    QT_F32 = 1,              /* inputs rounded to fp32 (RNE), fp32 MFMA, fp32 C */
    QT_BF16X3 = 2            /* inputs split into bf16 hi + lo; hi*hi + hi*lo + lo*hi
                                per block product in fp32 MFMA, summed in fp64; fp64 C */
} qt_prec;

typedef enum { QT_MEM_HOST = 0, QT_MEM_DEVICE = 1 } qt_mem;

/*
 * Device allocator of the library (the paper's chunks hold their data in
 * memory the runtime manages, Sec. 2; here the caller may manage it).
 *
 * Every device buffer the library creates -- a handle's values, tree and
 * derived operand forms, a multiply's scratch, a plan's work list -- is then
 * obtained with alloc(bytes, stream, ctx) and returned with
 * free_(p, stream, ctx):
 *   alloc:  returns at least `bytes` of device memory on the current device,
 *           aligned to 256 bytes, that work queued on `stream` from now on may
 *           use; NULL when it cannot (the library call then fails with
 *           QT_ERR_OOM and releases whatever it had obtained).
 *   free_:  gives p back. All use of p by the library is queued on `stream`
 *           before this point, or on other streams that `stream` already
 *           waits for; the allocator may hand p to later work on `stream`,
 *           and to other streams once they have waited for this point.
 * Both callbacks may be called from any thread that calls the library, and
 * from several at once. Buffers made before a change are still returned to
 * the allocator that made them, so ctx must stay valid while any of them
 * lives. alloc == free_ == NULL restores the default: HIP's stream-ordered
 * pool (hipMallocAsync / hipFreeAsync on the device's default pool). A few
 * bytes per device that the library keeps until the process ends (a lift
 * table, pinned read-back slots) never go through the allocator.
 * Errors: ARG (exactly one of alloc, free_ is NULL).
 */
qt_status qt_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                           void (*free_)(void* p, void* stream, void* ctx), void* ctx);

/*
 * Build a matrix from a list of nonzero blocks (Sec. 3.1 and 4.1).
 *
 * n_rows, n_cols: scalar dimensions; both multiples of block_size.
 * block_size:     b, the side of a block. The library runs b in {16, 32, 64}.
 * leaf_size:      side of a leaf; leaf_size / b must be a power of two <= 8.
 * nblocks:        number of blocks listed (0 gives an all-NIL matrix).
 * I, J:           block row / column of each block, 0 <= I < n_rows/b,
 *                 0 <= J < n_cols/b; any order; no (I, J) twice.
 * values:         nblocks * b * b fp64 values, block t at values + t*b*b.
 * where:          whether I, J, values are host or device memory.
 * The arrays are copied; the caller keeps ownership. Synchronizes `stream`
 * (validation reads back an error flag). The matrix is padded to a square of
 * side leaf_size * 2^L, the smallest that covers both dimensions.
 * Errors: ARG (NULL pointer, negative size, I/J out of range), SHAPE (b or
 * leaf rejected, dimension not a multiple of b), DUPLICATE, OOM, DEVICE.
 */
qt_status qt_build(int64_t n_rows, int64_t n_cols, int32_t block_size, int32_t leaf_size,
                   int64_t nblocks, const int32_t* I, const int32_t* J, const double* values,
                   qt_mem where, void* stream, qt_matrix** out);

/*
 * C = A * B (Algorithm 1). A and B may be the same handle.
 *
 * Both operands must have the same b and leaf size, and A's column count must
 * equal B's row count (else SHAPE). The symbolic phase walks both quadtrees
 * level by level from the roots, skipping every pair with a NIL operand, and
 * lists the block products of every C block in ascending inner index k; the
 * numeric phase runs one MFMA block GEMM per C block, accumulating in
 * registers, and stores each C block once. The result's value type follows
 * `prec` (F64 and BF16X3 give fp64 C, F32 gives fp32 C).
 * The symbolic phase runs on a stream of the library (one per device, default
 * priority), since it reads only the operands' structure; the host waits for
 * it once, to read the number of C blocks before C's values are allocated,
 * but does not wait for work already queued on `stream`. The numeric kernel
 * is queued on `stream` behind an event of that phase, and the call returns
 * without waiting for it: C is ready in stream order on `stream`.
 * Errors: ARG, SHAPE, OOM, DEVICE, UNSUPPORTED (more than 2^31 - 1 products).
 */
qt_status qt_multiply(const qt_matrix* A, const qt_matrix* B, qt_prec prec,
                      void* stream, qt_matrix** C);

/*
 * C = op(A) op(B) with op(X) = X or X^T (Sec. 3.2: the transposed multiply
 * task types C = A^T B, A B^T, A^T B^T), optionally forming only the blocks
 * of C on or above the block diagonal. op_flags is a combination of:
 *   QT_OP_TRANS_A  use A^T;   QT_OP_TRANS_B  use B^T;
 *   QT_OP_UPPER    C(I, J) only for I <= J (C must be square); the traversal
 *                  drops every quadrant strictly below the diagonal.
 * A transposed operand is read from its stored blocks as they are: the
 * product lists mark its blocks, and the numeric kernel loads each marked
 * block transposed; no copy of any operand is made. Otherwise as qt_multiply.
 * Errors: ARG (unknown flag), SHAPE, OOM, DEVICE, UNSUPPORTED.
 */
#define QT_OP_TRANS_A 1
#define QT_OP_TRANS_B 2
#define QT_OP_UPPER 4
qt_status qt_multiply_ex(const qt_matrix* A, const qt_matrix* B, int32_t op_flags, qt_prec prec, void* stream,
                         qt_matrix** C);

/*
 * C = A * B without the negligible products: the product with a norm
 * threshold that storing each submatrix's Frobenius norm in the quadtree
 * makes possible (the paper's conclusions, Sec. 7, after Bock and
 * Challacombe). Every node and block of A and B gets its squared Frobenius
 * norm (made once per handle, as qt_norms); the traversal drops every pair
 * (A node, B node) with ||A node||_F ||B node||_F < tau at any level, and the
 * leaf step every block product with ||A(I,K)||_F ||B(K,J)||_F < tau. A
 * node's norm bounds those of the blocks below it, so C(I,J) is the sum over
 * the K with ||A(I,K)|| ||B(K,J)|| >= tau, present iff one such K exists, and
 * ||C - A B||_F is at most the sum of ||A(I,K)|| ||B(K,J)|| over the dropped
 * products. tau = 0 gives the exact product (as qt_multiply). Comparisons are
 * made on squares in fp64; a product whose norm lies within rounding of tau
 * may go either way. The norms are made on `stream` from the operands'
 * values, and the traversal waits for them there; otherwise as qt_multiply
 * (qt_stats counts the pairs and products actually formed).
 * Errors: ARG (NULL argument, tau negative, NaN or above 1e150), SHAPE, OOM,
 * DEVICE, UNSUPPORTED (a structure-only operand, as made for qt_sysq).
 */
qt_status qt_multiply_tau(const qt_matrix* A, const qt_matrix* B, double tau, qt_prec prec, void* stream,
                          qt_matrix** C);

/*
 * Squared Frobenius norms (the per-submatrix norms of the paper's
 * conclusions, Sec. 7): block_norm2 (may be NULL) receives ||M(I,J)||_F^2 of
 * every stored block in (I, J) row-major order, as qt_to_blocks lists them;
 * total_norm2 (may be NULL) receives ||M||_F^2 (the quadtree root's, summed
 * up the tree). Both arrays are host or device memory as `where` says. The
 * norms of every node are made once per handle (on `stream`) and kept with
 * it. Synchronizes `stream` when `where` is QT_MEM_HOST.
 * Errors: ARG, OOM, DEVICE, UNSUPPORTED (a structure-only matrix).
 */
qt_status qt_norms(const qt_matrix* M, double* block_norm2, double* total_norm2, qt_mem where, void* stream);

/*
 * C = A + B (Algorithm 2, Sec. 3): the union of the two block patterns; a
 * block present in both is the sum of the two (fp64), a block present in one
 * is copied. A and B must agree in dimensions, block size and leaf size.
 * Synchronizes `stream`. Errors: ARG, SHAPE, OOM, DEVICE, UNSUPPORTED.
 */
qt_status qt_add(const qt_matrix* A, const qt_matrix* B, void* stream, qt_matrix** C);

/*
 * Value truncation: T holds M without its smallest blocks, removed in order
 * of increasing Frobenius norm for as long as the Frobenius norm of all
 * removed blocks together stays below eps (the error matrix E = M - T has
 * ||E||_F < eps; Sec. 6.2 truncates its overlap matrix this way). Kept blocks
 * are copied unchanged. *removed / *removed_norm2 (may be NULL) receive the
 * number of removed blocks and ||E||_F^2. Synchronizes `stream`.
 * Errors: ARG (eps negative or NaN), OOM, DEVICE.
 */
qt_status qt_truncate(const qt_matrix* M, double eps, void* stream, qt_matrix** T, int64_t* removed,
                      double* removed_norm2);

/*
 * Symmetric matrix square (Sec. 3.3): A holds the upper block triangle
 * (blocks with I <= J; diagonal blocks stored whole) of a symmetric S; C
 * holds the upper block triangle of S*S. The quadtree of S is formed once
 * from A's block pattern and kept with A: structure only (keys, tree, and
 * for each block of S the block of A that holds it, the mirrored ones marked
 * as transposed), about 12 bytes per block and no values. The product reads
 * A's values through it and skips every C quadrant below the diagonal, about
 * half the block products of S*S. A may hold fp64 or fp32 values.
 * Errors: ARG (a block below the diagonal), SHAPE (not square), OOM, DEVICE.
 */
qt_status qt_sysq(const qt_matrix* A, qt_prec prec, void* stream, qt_matrix** C);

/*
 * Describe a matrix (its shape as a quadtree over uniform blocks, Sec. 3.1).
 * Any output pointer may be NULL; value_type is QT_F64 or QT_F32.
 * Errors: ARG (NULL matrix).
 */
qt_status qt_info(const qt_matrix* M, int64_t* n_rows, int64_t* n_cols, int32_t* block_size,
                  int32_t* leaf_size, qt_prec* value_type);

/*
 * The number of stored (nonzero) blocks of M; zero submatrices are not
 * stored (Sec. 3.1). Known on the host for every handle the library returns
 * (a multiply reads its count back before it returns), so this never
 * synchronizes. Errors: ARG (NULL matrix or output).
 */
qt_status qt_nblocks(const qt_matrix* M, int64_t* nblocks);

/*
 * Copy a matrix out as a block list sorted by (I, J), row-major: the nonzero
 * blocks of the uniform block partition, zero blocks being absent (Sec. 3.1),
 * the form qt_build takes them in. I, J: nblocks int32 each; values: nblocks*b*b entries of out_type
 * (QT_F64 -> double, QT_F32 -> float; rounding to nearest even when the
 * stored type is wider). `where` says whether the three arrays are host or
 * device memory. values may be NULL to copy out the block pattern only.
 * Synchronizes `stream` when `where` is QT_MEM_HOST.
 * Errors: ARG, UNSUPPORTED (out_type QT_BF16X3), OOM, DEVICE.
 */
qt_status qt_to_blocks(const qt_matrix* M, int32_t* I, int32_t* J, void* values,
                       qt_prec out_type, qt_mem where, void* stream);

/*
 * qt_to_blocks for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same copy-out into device arrays I, J, values (values may be NULL),
 * bitwise the same result, but every buffer it needs beyond the caller's
 * arrays is a fixed scratch array of the library, 12 MiB per device, held
 * until the process ends. It calls no allocator (neither HIP's nor one set
 * with qt_set_allocator) and does not synchronize; the copy is queued on
 * `stream`. All calls on one device share that scratch and its contents
 * stay from call to call: calls on one device that overlap in time (on two
 * streams, or from two threads without ordering) race and give wrong
 * results; order them on one stream. The matrix must live on the current
 * device. Errors: ARG (NULL matrix or array, matrix on another device),
 * UNSUPPORTED (out_type QT_BF16X3, more than QT_NOALLOC_MAX_BLOCKS blocks),
 * DEVICE.
 */
#define QT_NOALLOC_MAX_BLOCKS (1 << 20)
qt_status qt_to_blocks_noalloc(const qt_matrix* M, int32_t* I, int32_t* J, void* values, qt_prec out_type,
                               void* stream);

/*
 * Fetch chosen blocks (a zero block is NIL and not stored, Sec. 3.1): for
 * t < count, block (I[t], J[t]) is looked up by
 * binary search over the matrix's Morton-ordered block keys and copied to
 * values + t*b*b (as out_type, like qt_to_blocks); found[t] is 1, or 0 with
 * a zero block when the block is not stored (a NIL block). I, J, values and
 * found are host or device memory as `where` says; out-of-range (I, J) give
 * found = 0. Synchronizes `stream` when `where` is QT_MEM_HOST.
 * Errors: ARG, UNSUPPORTED (out_type QT_BF16X3), OOM, DEVICE.
 */
qt_status qt_get_blocks(const qt_matrix* M, int64_t count, const int32_t* I, const int32_t* J, void* values,
                        int32_t* found, qt_prec out_type, qt_mem where, void* stream);

/*
 * Counters of the multiply that produced C (Sec. 5): pairs[l] is the number
 * of (A node, B node) pairs with both present at quadtree level l
 * (0 = root .. depth = leaf level, the levels qt_levels counts), i.e. the
 * multiply tasks of Algorithm 1 at that level; *products (may be NULL) is the
 * number of block products. At most max_levels entries are written; entries
 * past the leaf level are not touched. For a matrix from qt_build all
 * counters are zero. Errors: ARG.
 */
qt_status qt_stats(const qt_matrix* C, int64_t* pairs, int32_t max_levels, int64_t* products);

/*
 * Nodes of the quadtree per level (Sec. 3.1): nodes[l] is the number of
 * non-NIL nodes at level l (0 = root .. n_levels-1 = leaf level). A zero
 * submatrix is NIL at every level, so a multiply result keeps exactly the
 * nodes with at least one stored block below them (a leaf pair with no block
 * product, and a node over only such leaves, are NIL). At most max_levels
 * entries are written; *n_levels (may be NULL) receives the depth + 1.
 * Errors: ARG (NULL matrix, negative max_levels, NULL nodes with
 * max_levels > 0).
 */
qt_status qt_levels(const qt_matrix* M, int64_t* nodes, int32_t max_levels, int32_t* n_levels);

/*
 * Prepare the operand forms a multiply at `prec` reads (fp32 copy, bf16
 * hi/lo split; the leaf products run in single or double precision as in
 * Sec. 6.1) so that a later timed multiply does not build them. Optional:
 * qt_multiply builds them on first use. Thread-safe. Errors: OOM, DEVICE.
 */
qt_status qt_prepare(const qt_matrix* M, qt_prec prec, void* stream);

/* Release a handle (NULL is ignored): a matrix, like a registered chunk
 * (Sec. 2), belongs to the library from its creation until it is released.
 * Its device memory is released in order on the stream that created it. */
void qt_free(qt_matrix* M);

/*
 * Batched multiplies (many independent C_i = A_i * B_i, one block size).
 *
 * qt_plan_create runs the symbolic phase (the quadtree traversal of
 * Algorithm 1, Sec. 3) of every problem now -- it synchronizes `stream` and
 * allocates every C_i -- and lays the numeric work of all problems out as one
 * work list: problems by decreasing block products, C blocks of a problem in
 * its launch order (see QT_PLAN_ORDER_MORTON below).
 *   count:  number of problems (>= 1); A[i], B[i] as for qt_multiply (same
 *           block size across the batch; leaf sizes may differ per problem).
 * Errors: ARG, SHAPE, OOM, DEVICE, UNSUPPORTED.
 *
 * qt_plan_execute computes every C_i: one kernel launch (plus a one-thread
 * counter reset for the dynamic schedules, a kernel, not a memset) on
 * `stream`, which allocates nothing and does not synchronize, so a caller may
 * capture it into a HIP graph of its own. qt_plan_replay computes the same:
 * its first call captures that launch sequence into a HIP graph the plan
 * keeps, and every call replays the graph on `stream` (one launch from the
 * host). Executions on one plan, by either call, must not overlap (they share
 * the plan's work counter and the C_i). Errors: ARG (NULL plan), DEVICE.
 *
 * A plan runs in one of QT_PLAN_CONFIGS configurations, a schedule (0 .. 3)
 * plus option bits:
 *   schedule 0  flat grid: one workgroup per work item, the hardware
 *               dispatcher balancing the uneven problems;
 *   schedule 1  persistent, balanced: as many workgroups as fit on the GPU
 *               at once, each taking a contiguous run of work items that
 *               holds an equal share of the work (block products plus one per
 *               C block, summed when the plan is created; no counter);
 *   schedule 2  persistent, dynamic per XCD: each workgroup takes 2 items at
 *               a time from a counter of its XCD, over the flat grid's runs
 *               of neighbouring items per XCD;
 *   schedule 3  persistent, dynamic: 16 items at a time from a counter;
 *   QT_PLAN_ORDER_MORTON  every problem's C blocks in Morton order (without
 *               it a problem whose C blocks average under two block products
 *               is launched grouped by inner index, as qt_multiply does);
 *   QT_PLAN_TILE_WAVE     at b = 64, one wave per 32 x 32 tile instead of one
 *               four-wave workgroup per C block sharing its operands through
 *               LDS (no effect at other block sizes).
 * Every configuration gives bitwise the same C_i (and the same as
 * qt_multiply). A new plan starts in configuration 0.
 *
 * qt_plan_tune times every configuration that differs on this plan, `reps`
 * runs each, keeps the fastest and reports it in *schedule; ms (may be NULL)
 * receives QT_PLAN_CONFIGS mean times, -1 for configurations not tried. It
 * computes the C_i as a side effect and synchronizes `stream`.
 *
 * qt_plan_set_schedule picks a configuration directly (e.g. one tuned
 * earlier); ARG unless 0 <= schedule < QT_PLAN_CONFIGS.
 *
 * qt_plan_result returns C_i, owned by the plan: valid until
 * qt_plan_destroy, and qt_free on it does nothing. qt_plan_info reports the
 * number of work items, block products and the configuration.
 * qt_plan_destroy waits for the plan's last execution and releases all of it.
 */
#define QT_PLAN_SCHEDULES 4
#define QT_PLAN_ORDER_MORTON 4
#define QT_PLAN_TILE_WAVE 8
#define QT_PLAN_CONFIGS 16
qt_status qt_plan_create(int32_t count, const qt_matrix* const* A, const qt_matrix* const* B, qt_prec prec,
                         void* stream, qt_plan** plan);
qt_status qt_plan_execute(qt_plan* plan, void* stream);
qt_status qt_plan_replay(qt_plan* plan, void* stream);
qt_status qt_plan_tune(qt_plan* plan, void* stream, int reps, int32_t* schedule, float* ms);
qt_status qt_plan_set_schedule(qt_plan* plan, int32_t schedule);   /* a configuration, 0 .. QT_PLAN_CONFIGS-1 */
qt_status qt_plan_result(const qt_plan* plan, int32_t i, qt_matrix** C);
qt_status qt_plan_info(const qt_plan* plan, int64_t* work_items, int64_t* products, int32_t* schedule);
void qt_plan_destroy(qt_plan* plan);

/*
 * Leaf-size tuner. Rebuilds A and B at every leaf size b, 2b, 4b, 8b and
 * times the full qt_multiply (`reps` runs each) at precision `prec`; returns
 * the fastest leaf size in *best_leaf. The leaf size only changes the
 * symbolic phase (how many quadtree levels are walked before the block-sparse
 * leaves, Sec. 4.1 and Sec. 5): the products and the result are the same at
 * every leaf size. leaves / ms (may be NULL) receive up to max_out tried
 * sizes and their mean times; *n_tried how many were tried. Synchronizes.
 * Errors: ARG, SHAPE, OOM, DEVICE.
 */
qt_status qt_tune_leaf(const qt_matrix* A, const qt_matrix* B, qt_prec prec, void* stream, int reps,
                       int32_t* best_leaf, int32_t* leaves, float* ms, int32_t max_out, int32_t* n_tried);

/*
 * Tuning cache (the leaf size trades the quadtree's overhead against the
 * leaf multiplies', Sec. 5): the choices of the tuners kept in a text file (one line per
 * choice, "key<TAB>value") and reused instead of timing again. The key is
 * the GPU architecture (e.g. gfx950), the block size, the precision, the
 * tuner and a class the caller names: for qt_tune_leaf_cached a pattern class
 * (e.g. "random n2^11 fill2^-6": the leaf size that suits a problem depends on
 * its pattern, size and fill), for qt_plan_tune_cached the batch (its
 * configuration depends on the mix of problems).
 * qt_tune_cache(path) sets the file and reads what it holds (a missing file
 * is made on the first new choice; NULL stops using a file). Every new choice
 * rewrites the file (to path.tmp, then renamed over path). The tuners
 * otherwise behave as qt_tune_leaf and qt_plan_tune; *cached (may be NULL) is
 * 1 when the choice came from the file (nothing was timed, and the plan was
 * only set to it), else 0. Without a file they always time.
 * Errors: ARG (NULL argument, unknown precision, the file cannot be written),
 * and those of the tuner.
 */
qt_status qt_tune_cache(const char* path);
qt_status qt_tune_leaf_cached(const qt_matrix* A, const qt_matrix* B, qt_prec prec, void* stream, int reps,
                              const char* pattern_class, int32_t* best_leaf, int32_t* cached);
qt_status qt_plan_tune_cached(qt_plan* plan, void* stream, int reps, const char* batch_class, int32_t* schedule,
                              int32_t* cached);

/* Per-phase GPU timing of qt_multiply (the two phases of Algorithm 1's
 * multiply: the quadtree traversal, Sec. 3.2, and the leaf products, Sec. 4.1),
 * from HIP events recorded on the multiply's stream. qt_profile(1) starts recording (and clears totals),
 * qt_profile(0) stops. qt_profile_read synchronizes on the recorded events
 * and returns the summed milliseconds of the symbolic phase (traversal and
 * product lists) and of the numeric kernel, the number of multiplies timed,
 * and the summed block products and C blocks of those multiplies.
 * Any output pointer may be NULL. */
qt_status qt_profile(int enable);
qt_status qt_profile_read(double* symbolic_ms, double* numeric_ms, int64_t* calls,
                          int64_t* products, int64_t* c_blocks);

/* Attainable MFMA rate: times a register-only loop of the MFMA instruction
 * the numeric kernels of `prec` issue (fp64 16x16x4, fp32 16x16x4, bf16
 * 16x16x32; eight independent accumulator chains per wave, eight waves per
 * SIMD, no memory traffic in the loop) and returns its rate in TFLOP/s
 * (2*M*N*K flops per instruction) in *tflops. A diagnostic beside the
 * published peak, not part of the multiply (the paper measures its own
 * "practical peak" of the batched leaf GEMM the same way, Sec. 6.1, Table 2).
 * Synchronizes `stream`. Errors: ARG (NULL output, unknown precision), DEVICE. */
qt_status qt_probe_mfma(qt_prec prec, void* stream, double* tflops);

/* Practical peak of the batched block GEMM (Sec. 6.1, Table 2, which times
 * 64000 products C_i = A B of b x b blocks, A and B the same for all): runs
 * `count` such products through the multiply's own numeric kernels (one C
 * block per product, the operands one block of A and one of B read by every
 * product), ten launches after one warm-up, and returns 2 b^3 count / time
 * in TFLOP/s in *tflops. count is at most 2^24; the C blocks (count b^2
 * values) are allocated for the call. Synchronizes `stream`.
 * Errors: ARG (NULL output, count out of range, unknown precision), SHAPE (b
 * not 16, 32 or 64), UNSUPPORTED (BF16X3 at b = 16), OOM, DEVICE. */
qt_status qt_probe_batched(qt_prec prec, int32_t block_size, int64_t count, void* stream, double* tflops);

/* Text of the last error on this thread ("" if none). A library utility, no
 * operation of the paper. */
const char* qt_last_error(void);

/* Library version string. A library utility, no operation of the paper. */
const char* qt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QT_H */
