/*
 * bsmm -- block-sparse matrix multiply for AMD MI355X (gfx950).
 *
 * C-ABI of the node-local multiply of the DBCSR method (Bethune et al.,
 * "Porting of the DBCSR library for Sparse Matrix-Matrix Multiplications to
 * Intel Xeon Phi systems", 2017, Section 2): blocked-CSR matrices made of
 * small dense blocks, C = alpha*A*B + beta*C built from pairwise block
 * products, with the on-the-fly norm filter.
 *
 * Conventions for every entry point:
 *   - No exception or abort crosses this boundary; every call returns a
 *     bsmm_status and, on failure, bsmm_last_error() describes it.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it in order.  Calls that must report sizes to the
 *     host synchronise that stream and say so below.
 *   - Handles are not thread-safe; do not use one handle from two threads at
 *     once.  Distinct handles may be used concurrently on distinct streams.
 *   - Block values are FP64, each block stored row-major, blocks contiguous
 *     in CSR order (block b of row i has row_sizes[i] x col_sizes[col_idx[b]]
 *     values).  Block sizes are >= 1.
 *   - The library owns all device memory behind a handle and frees it in
 *     bsmm_destroy().  Buffers passed in are only read during the call
 *     (create) or only written (norms, export); the caller keeps ownership.
 */
#ifndef BSMM_H
#define BSMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsmm_matrix* bsmm_mat;
typedef struct bsmm_graph_s* bsmm_graph;

typedef enum {
  BSMM_OK = 0,
  BSMM_E_ARG = 1,          /* NULL handle/pointer, bad size, non-finite scalar, unknown enum */
  BSMM_E_SHAPE = 2,        /* block sizes of the operands do not conform */
  BSMM_E_PATTERN = 3,      /* row_ptr not monotone / wrong ends, column out of range,
                              columns not strictly increasing in a row */
  BSMM_E_ALIAS = 4,        /* output handle is also an input operand (A or B) */
  BSMM_E_NOMEM = 5,        /* device or host allocation failed */
  BSMM_E_CAPACITY = 6,     /* a result exceeds int32 block indexing or a reserved capacity */
  BSMM_E_HIP = 7,          /* a HIP runtime call failed */
  BSMM_E_UNSUPPORTED = 8   /* valid input outside what this build handles (message says why) */
} bsmm_status;

/* Arithmetic of the block products.  Norms, filter decisions, the symbolic
 * phase and the C accumulation are FP64 in every mode. */
typedef enum {
  BSMM_FP64 = 0,          /* FP64 products and accumulation */
  BSMM_SPLIT_F32X2 = 1,   /* two FP32 terms per value: not built (BSMM_E_UNSUPPORTED) */
  BSMM_SPLIT_BF16X3 = 2,  /* three BF16 terms per value, the six term products of combined
                             order <= 2 on BF16 matrix cores with FP32 accumulation, each
                             block product added in FP64; 23x23 blocks only
                             (BSMM_E_UNSUPPORTED otherwise).  Per C element the error is
                             below 2^-15 * |alpha| * sum_k |A(i,k)| |B(k,j)| plus FP64
                             rounding. */
  BSMM_SLICE_INT8X7 = 3   /* exact slices (Ozaki-style splitting of the block products of
                             Section 2): every value is scaled by a power of two per row of
                             its block row (A) or per column of its block column (B) and cut
                             into seven signed 7-bit digits; the digit products of combined
                             order <= 8 run on INT8 matrix cores with exact INT32 sums over
                             all products of a C block, combined in FP64 at its end.  23x23
                             blocks only (BSMM_E_UNSUPPORTED otherwise); values must be
                             finite.  Per element (r,q) of C(i,j) the error is below
                             2^-39 * |alpha| * n_ij * MA(i,r) * MB(j,q) plus FP64 rounding of
                             the alpha/beta update, with n_ij the performed block products,
                             MA(i,r) the largest |A| in row r of block row i and MB(j,q) the
                             largest |B| in column q of block column j.  Its digit buffers
                             are allocated on first use, also for a reserved C_out. */
} bsmm_prec;

enum { BSMM_PTR_HOST = 0, BSMM_PTR_DEVICE = 1 };

/* Kernel path that computed the block products of a multiply. */
enum {
  BSMM_PATH_GENERIC = 0, /* any other block sizes, FP64, in 32x32 sub-tiles and K chunks of 32 */
  BSMM_PATH_TILE23 = 1,  /* uniform 23x23 blocks, FP64 */
  BSMM_PATH_SMALL = 2,   /* every block edge <= 16, FP64, one launch over all shape classes */
  BSMM_PATH_SPLIT23 = 3, /* uniform 23x23 blocks, BSMM_SPLIT_BF16X3 */
  BSMM_PATH_SLICE23 = 4  /* uniform 23x23 blocks, BSMM_SLICE_INT8X7 */
};

/* Number of compiled pipeline variants of the small-block path. */
#define BSMM_SMALL_VARIANTS 8

/* Number of variants of the generic path (bsmm_tune_mid). */
#define BSMM_MID_VARIANTS 8

/* Counters of the last multiply that wrote a handle. */
typedef struct {
  int64_t candidates;  /* block products with both blocks present (before the filter) */
  int64_t products;    /* block products kept by the filter and computed */
  int64_t nnzb;        /* blocks in the result */
  int64_t nvals;       /* values in the result */
  double useful_flops; /* sum over kept products of 2*m*n*k */
  int32_t path;        /* BSMM_PATH_* */
  int32_t variants[4]; /* small-block variant used per shape class 8x8, 8x16, 16x8, 16x16;
                          on the generic path {variant, -1, -1, -1} (bsmm_tune_mid);
                          -1 on the 23x23 paths */
  int32_t panels;      /* stack panels the products were built and consumed in (1: whole stack) */
} bsmm_mult_stats;

/*
 * Create a matrix from blocked CSR (Section 2, storage format).
 *   nbrows, nbcols      : block rows / block columns (>= 0)
 *   row_sizes[nbrows]   : rows of each block row (>= 1); always host memory
 *   col_sizes[nbcols]   : columns of each block column (>= 1); always host memory
 *   nnzb                : stored blocks
 *   row_ptr[nbrows+1]   : row_ptr[0] = 0, non-decreasing, row_ptr[nbrows] = nnzb
 *   col_idx[nnzb]       : block columns, strictly increasing within a row
 *   values              : all block values (see conventions); NULL = all zero
 *   ptr_kind            : BSMM_PTR_HOST or BSMM_PTR_DEVICE for row_ptr/col_idx/values
 * The inputs are copied and validated (device inputs are copied to the host
 * for validation, which synchronises `stream`).  On error *out is untouched.
 */
bsmm_status bsmm_create(bsmm_mat* out, int32_t nbrows, int32_t nbcols, const int32_t* row_sizes,
                        const int32_t* col_sizes, int32_t nnzb, const int32_t* row_ptr,
                        const int32_t* col_idx, const double* values, int ptr_kind, void* stream);

/* Release a handle and its device memory (synchronises the device first). NULL is a no-op. */
bsmm_status bsmm_destroy(bsmm_mat m);

/*
 * C_out = alpha * A * B + beta * C_in, with the on-the-fly filter
 * (Section 2): the product of blocks A(i,k) and B(k,j) is performed only if
 * filter_eps <= 0 or fl(|A(i,k)|_F * |B(k,j)|_F) > filter_eps.
 *   - The result pattern is every (i,j) with at least one performed product,
 *     plus the pattern of C_in when beta != 0.  Blocks are kept even if zero.
 *   - C_in may be NULL (no old values), may be C_out (in-place update) and
 *     may be A or B.  With beta == 0 it is never read.
 *   - C_out must not be A or B (BSMM_E_ALIAS).  Its previous pattern and
 *     values are replaced.  A.col_sizes must equal B.row_sizes, and C_out
 *     (and C_in when read) must have A's row sizes and B's column sizes
 *     (BSMM_E_SHAPE).
 *   - alpha, beta and filter_eps must be finite (BSMM_E_ARG).
 *   - Synchronises `stream` once, after the symbolic phase, to size C_out,
 *     unless C_out is reserved (bsmm_reserve): then it never synchronises
 *     (twice when the stack is built in panels, see bsmm_set_stack_limit).
 *   - Symbolic pass limits: at most 2048 stored blocks in a block row of A
 *     and 2048 blocks in a block row of the result (BSMM_E_UNSUPPORTED).
 * Errors: a call rejected by its checks (arguments, shapes, aliasing, the
 * symbolic pass limits, capacity, an unsupported precision/size pair) leaves
 * C_out as it was, values, pattern and product stack included.  If device
 * allocation (BSMM_E_NOMEM) or a HIP call (BSMM_E_HIP) fails after C_out began
 * to be rewritten, C_out is left a valid empty matrix (no blocks, no product
 * stack) and the message says so.
 */
bsmm_status bsmm_multiply(double alpha, bsmm_mat A, bsmm_mat B, double beta, bsmm_mat C_in,
                          bsmm_mat C_out, double filter_eps, int prec, void* stream);
/* (prec is a bsmm_prec; an unknown value is BSMM_E_ARG.) */

/*
 * Drop every block whose Frobenius norm is not above eps (eps <= 0 keeps
 * all blocks); compacts the pattern and values in place (Section 2: the
 * filter increases sparsity).  Synchronises `stream` to read the new size,
 * except for a reserved matrix (see bsmm_reserve), where it stays on the
 * device.
 */
bsmm_status bsmm_filter(bsmm_mat m, double eps, void* stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): bsmm_filter with the same
 * result bits, that allocates nothing.  Its temporaries (block norms, keep
 * flags, the two scans) live in one fixed scratch array of the library, 6 MiB
 * on every GPU it runs on, held until the process ends; the compacted matrix
 * goes to the matrix's second storage, which must already hold the matrix's
 * size (bsmm_reserve provides it; so does one earlier bsmm_filter or in-place
 * multiply of at least this size).
 *   - At most 131072 blocks (the reserved block capacity for a reserved
 *     matrix), else BSMM_E_CAPACITY; BSMM_E_CAPACITY too if the second
 *     storage is smaller than the matrix.  Nothing is changed on error.
 *   - Reads the new size back like bsmm_filter (synchronises `stream`) except
 *     for a reserved matrix.
 *   - Every call on one GPU uses that GPU's one scratch array: calls that
 *     overlap in time on one GPU (other streams, other threads) race.
 */
bsmm_status bsmm_filter_noalloc(bsmm_mat m, double eps, void* stream);

/*
 * Frobenius norm of every stored block, in CSR order, into out[nnzb]
 * (device memory owned by the caller; for a device-sized matrix it must hold
 * the reserved block capacity).  The sum of squares runs in a fixed
 * order (64 interleaved partial sums with fused multiply-add, then a pairwise
 * tree, then a correctly rounded square root), so the values are bitwise
 * reproducible.
 */
bsmm_status bsmm_norms(bsmm_mat m, double* out, void* stream);

/* Sizes of a matrix (any pointer may be NULL).  Host-side metadata; if the
 * matrix was last written by a reserved (device-sized) multiply or filter,
 * this first waits for the device and reads the sizes back, and reports a
 * reserved operation that overflowed (BSMM_E_CAPACITY; the matrix is then
 * empty). */
bsmm_status bsmm_info(bsmm_mat m, int32_t* nbrows, int32_t* nbcols, int32_t* nnzb, int64_t* nvals);

/*
 * Copy the pattern and values out: row_ptr[nbrows+1], col_idx[nnzb],
 * values[nvals] (any pointer may be NULL), host or device memory per
 * ptr_kind.  Synchronises `stream` (and reads device-resident sizes back,
 * see bsmm_info).
 */
bsmm_status bsmm_export(bsmm_mat m, int32_t* row_ptr, int32_t* col_idx, double* values, int ptr_kind,
                        void* stream);

/*
 * Product stack of the last multiply that wrote C: one entry per performed
 * block product, (C block, A block, B block) indices in CSR order, sorted by
 * C block and then by the inner block index k.  *nprod receives the count;
 * the arrays (any may be NULL) must hold that many entries.  Synchronises.
 * BSMM_E_UNSUPPORTED if that multiply built its stack in panels (see
 * bsmm_set_stack_limit): panels are consumed and not kept.
 */
bsmm_status bsmm_export_stack(bsmm_mat C, int32_t* st_c, int32_t* st_a, int32_t* st_b, int64_t* nprod,
                              int ptr_kind, void* stream);

/* Counters of the last multiply that wrote C (zeros if none).  Waits for the
 * device like bsmm_info when C is device-sized. */
bsmm_status bsmm_stats(bsmm_mat C, bsmm_mult_stats* out);

/*
 * Autotuner of the small-block path (Section 2: the batched multiply is tuned
 * for each set of block dimensions).  The path pads each block to a shape
 * class, 8 or 16 rows by 8 or 16 columns; a variant fixes, per class, the
 * form of the block product (FP64 vector units or FP64 matrix cores) and the
 * number of block products in flight per wave (bsmm_small_variant).  The
 * tuning table maps a tuning key (the block edges present in A's rows, A's
 * columns and B's columns) to one variant per class; classes of a multiply
 * whose key has no entry use variant 1.  Classes that share a variant run in
 * one launch.
 *
 * bsmm_tune_small computes C_out = alpha*A*B + beta*C_in exactly as
 * bsmm_multiply with BSMM_FP64 does, then, if the small-block path served it,
 * times the products of each class alone with every variant (`reps` launches
 * each, HIP events on `stream`), enters for each class the variant with the
 * least time into the table and leaves C_out as those variants compute it
 * (variants of the same form give identical values; the forms add in
 * different orders, all within FP64 rounding of the exact sum).
 * Arguments as bsmm_multiply, plus:
 *   reps         : launches per variant and class, 1 ..  1000
 *   variants_out : host array [4]: chosen variant per class, or all -1 when
 *                  another path serves these sizes (then nothing is timed and
 *                  the table is unchanged)
 *   ms_out       : NULL, or host array [BSMM_SMALL_VARIANTS * 4] receiving
 *                  the milliseconds of variant v, class c at [4*v + c],
 *                  summed over the reps (0 for a variant that does not serve
 *                  these block edges)
 * C_in must not be C_out (BSMM_E_ARG), and C_out must not be reserved.
 * Synchronises `stream`.
 */
bsmm_status bsmm_tune_small(double alpha, bsmm_mat A, bsmm_mat B, double beta, bsmm_mat C_in, bsmm_mat C_out,
                            double filter_eps, int32_t reps, int32_t* variants_out, double* ms_out, void* stream);

/* Form and depth of variant v in the classes 8x8, 8x16, 16x8 and 16x16 (rows
 * x columns) into depths[4].  On the vector units: the products kept in
 * flight per wave, where 1 means several products of one C block per step
 * (four for 8x8, one per 16-lane group; two for 8x16 and 16x8, one per
 * 32-lane group) and 8 two such steps of the 8x8 class, which only serves
 * block edges of at most 8 (multiplies with larger edges use variant 1 for
 * that class instead).  16 + d: the FP64 matrix-core form
 * (v_mfma_f64_4x4x4_4b, the block padded to 4x4 tiles and the inner index to
 * a multiple of 8) with d products in flight.  BSMM_E_ARG if v is out of
 * range. */
bsmm_status bsmm_small_variant(int32_t v, int32_t* depths);

/* Tuning key of the product A*B: bits e-1, 16+e-1 and 32+e-1 are set for each
 * block edge e in A's row sizes, A's column sizes and B's column sizes.
 * BSMM_E_UNSUPPORTED if an edge exceeds 16 (the small-block path does not
 * serve such sizes). */
bsmm_status bsmm_tune_key(bsmm_mat A, bsmm_mat B, uint64_t* key);

/* Table entry of `key`: bsmm_tune_set enters variants[4] (one per class, each
 * 0 .. BSMM_SMALL_VARIANTS-1) or removes the entry (variants NULL);
 * bsmm_tune_get writes the entry into variants[4], all -1 if there is none.
 * The table is process-wide and guarded by a lock. */
bsmm_status bsmm_tune_set(uint64_t key, const int32_t* variants);
bsmm_status bsmm_tune_get(uint64_t key, int32_t* variants);

/* Copy up to `cap` table entries (ascending key) into keys[cap] and
 * variants[4*cap] (host arrays); *n receives the number of entries in the
 * table. */
bsmm_status bsmm_tune_entries(uint64_t* keys, int32_t* variants, int32_t cap, int32_t* n);

/*
 * Autotuner of the generic path (blocks that are neither all <= 16 nor all
 * 23x23; Section 2: the batched multiply is tuned for each set of block
 * dimensions).  The path cuts every C block into square sub-tiles and
 * accumulates one sub-tile per wave over K chunks of 32.  A variant fixes the
 * tile shape and the form:
 *   bit 0 (tile policy): 0 = 32x32 sub-tiles for every C block; 1 = one
 *          16x16 sub-tile, on the vector units, for each C block with both
 *          edges <= 16 (a 9x9 block beside 22- and 32-edge blocks pads to
 *          16x16 instead of 32x32);
 *   bit 1 (form): the FP64 matrix cores (v_mfma_f64_4x4x4_4b) for 32x32
 *          sub-tiles of C blocks with both edges >= 16; only allowed when
 *          every inner block edge is >= 16, and dropped otherwise;
 *   bit 2 (C_in prefetch): a sub-tile's C_in values are loaded before its
 *          last K chunk is multiplied (pays where C blocks have few
 *          products; the kernel without it keeps fewer registers live).
 * The table maps the block edges present (A's rows, A's columns, B's
 * columns, each as a mask with bit e-1 set for edge e and bit 31 for every
 * edge >= 32) to a variant; a multiply whose masks have no entry uses 2 when
 * every inner edge is >= 16, else 0.  The vector form gives the same bits
 * with either tile policy and with or without the prefetch; the matrix-core form adds in another order, within
 * FP64 rounding of the exact sum.
 *
 * bsmm_tune_mid computes C_out = alpha*A*B + beta*C_in exactly as
 * bsmm_multiply with BSMM_FP64 does, then, if the generic path served it,
 * times the numeric phase with every allowed variant (`reps` launches each,
 * HIP events on `stream`), enters the fastest into the table and leaves C_out
 * as that variant computes it.  Arguments as bsmm_tune_small, except:
 *   variant_out : host int32: the chosen variant, or -1 when another path
 *                 serves these sizes (nothing is timed, the table unchanged)
 *   ms_out      : NULL, or host array [BSMM_MID_VARIANTS]: milliseconds of
 *                 each variant summed over the reps (0 if not allowed)
 * Synchronises `stream`.
 */
bsmm_status bsmm_tune_mid(double alpha, bsmm_mat A, bsmm_mat B, double beta, bsmm_mat C_in, bsmm_mat C_out,
                          double filter_eps, int32_t reps, int32_t* variant_out, double* ms_out, void* stream);

/* Key of the product A*B in the generic path's table: masks[3] (host) =
 * {A's row edges, A's column edges, B's column edges}, as described above. */
bsmm_status bsmm_mid_key(bsmm_mat A, bsmm_mat B, uint32_t* masks);

/* Table entry of masks[3]: bsmm_mid_set enters `variant`
 * (0 .. BSMM_MID_VARIANTS-1) or removes the entry (variant -1); bsmm_mid_get
 * writes the entry into *variant, -1 if there is none.  Process-wide, guarded
 * by the same lock as the small-block table. */
bsmm_status bsmm_mid_set(const uint32_t* masks, int32_t variant);
bsmm_status bsmm_mid_get(const uint32_t* masks, int32_t* variant);

/* Copy up to `cap` entries of the generic path's table into masks[3*cap] and
 * variants[cap] (host arrays); *n receives the number of entries. */
bsmm_status bsmm_mid_entries(uint32_t* masks, int32_t* variants, int32_t cap, int32_t* n);

/*
 * Graph-capturable mode.  Reserve device capacity in m for the results of the
 * multiplies and filters that will write it: at most max_nnzb blocks,
 * max_nvals values and max_products block products per multiply.  From then
 * on, bsmm_multiply(..., C = m, ...) and bsmm_filter(m, ...) neither allocate
 * nor synchronise: the result sizes stay on the device, kernels read them
 * there, and the host learns them at the next synchronising call (info,
 * export, export_stack, stats).  A result that does not fit is not written;
 * the overflow is recorded on the device and reported by that call as
 * BSMM_E_CAPACITY (or BSMM_E_UNSUPPORTED for a row beyond the symbolic
 * limits), after which m is empty.  The current contents of m are kept.
 * Inputs of such a multiply must not hold more blocks than the capacity of
 * the output (the norm scratch of the filter is sized by it).  The operand
 * buffers of split and exact-slice precision are not reserved: the first
 * multiply into m in such a precision allocates them (run it once before
 * capturing).  Synchronises `stream` once.  Capacities must be >= 1, the
 * block capacity below 2^31, and the product capacity too unless m has
 * uniform 23x23 blocks (stack panels, see bsmm_set_stack_limit).
 */
bsmm_status bsmm_reserve(bsmm_mat m, int64_t max_nnzb, int64_t max_nvals, int64_t max_products, void* stream);

/*
 * Stack limit of m (Section 2: the local multiply fills stacks of block
 * products and processes each when it is full): the block products one
 * stack panel of a multiply into m may hold, 2 .. 2^31-1, default 2^30 (8 GB
 * of indices).  A multiply of uniform 23x23 blocks (any precision) with more
 * products than the limit builds and consumes its stack in panels of
 * consecutive C block rows, each holding at most the limit: with R the most
 * products of one block row, a panel starts at every multiple of
 * max(limit - R, limit/2) products, so panels are nearly full, and a block
 * row may hold at most half the limit (BSMM_E_CAPACITY otherwise).  Results
 * are bit-identical to the whole-stack multiply; the multiply's stats count
 * the panels that hold a row.  Other block sizes build the whole stack (at most
 * 2^31-1 products) whatever the limit.  For a reserved output the limit sizes
 * the stack: bsmm_reserve allocates min(max_products, limit) entries and the
 * multiplies run ceil(max_products / (limit/2)) + 1 panels (at most 4096;
 * empty panels cost a few launches), so max_products may exceed 2^31-1 for
 * 23x23 blocks.  Set it before bsmm_reserve (BSMM_E_ARG after).
 */
bsmm_status bsmm_set_stack_limit(bsmm_mat m, int64_t max_products);

/*
 * ||m||_F of all stored values into out[0] (device memory owned by the
 * caller), in FP64 with a fixed summation order (256 contiguous slices, each
 * summed by 256 interleaved fused multiply-add partials and a pairwise tree;
 * the slice sums by a pairwise tree; a correctly rounded square root).
 * Asynchronous; works on device-sized matrices (the Newton-Schulz residual).
 */
bsmm_status bsmm_frobenius(bsmm_mat m, double* out, void* stream);

/*
 * HIP graph capture of a sequence of calls on one created (non-default)
 * stream: bsmm_capture_begin, then reserved multiplies / filters /
 * frobenius on that stream, then bsmm_capture_end, which instantiates the
 * graph.  bsmm_graph_launch replays it on any stream; each replay re-runs the
 * captured calls on the same buffers.  Calls that would allocate or
 * synchronise must not be captured (they fail the capture); run the sequence
 * once before capturing so every scratch buffer has its final size.
 */
bsmm_status bsmm_capture_begin(void* stream);
bsmm_status bsmm_capture_end(void* stream, bsmm_graph* out);
bsmm_status bsmm_graph_launch(bsmm_graph g, void* stream);
bsmm_status bsmm_graph_destroy(bsmm_graph g);

/* Phases timed by bsmm_timing / bsmm_phase_times. */
enum {
  BSMM_PHASE_NORMS = 0,    /* block norms of A and B (only when filter_eps > 0) */
  BSMM_PHASE_COUNT = 1,    /* symbolic count pass and row scans */
  BSMM_PHASE_SIZING = 2,   /* read-back of the result size and output allocation */
  BSMM_PHASE_FILL = 3,     /* symbolic fill pass: pattern and product stack */
  BSMM_PHASE_NUMERIC = 4,  /* batched block products and alpha/beta finalisation */
  BSMM_PHASE_TOTAL = 5,    /* whole multiply, first to last enqueued operation */
  BSMM_NPHASES = 6
};

/*
 * Start (enable != 0) or stop recording HIP events around the phases of every
 * multiply that writes C, on the multiply's own stream.  Starting clears
 * earlier records.  Recording adds no synchronisation.
 */
bsmm_status bsmm_timing(bsmm_mat C, int enable);

/*
 * Sum of each phase's duration in milliseconds over the multiplies recorded
 * since bsmm_timing(C, 1): ms[BSMM_NPHASES]; *count receives the number of
 * recorded multiplies.  Synchronises on the recorded events.
 */
bsmm_status bsmm_phase_times(bsmm_mat C, double* ms, int64_t* count);

/* Message for the last failing call on this thread ("" if none). */
const char* bsmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BSMM_H */
