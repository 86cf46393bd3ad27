// Internal declarations shared by the host planner (api.cpp) and the HIP
// kernels of libbsmm.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsmm {

// Read-only device view of a blocked-CSR matrix, passed to kernels by value.
struct MatView {
  int32_t nbrows;
  int32_t nbcols;
  int32_t nnzb;
  const int32_t* row_sizes;  // [nbrows]
  const int32_t* col_sizes;  // [nbcols]
  const int32_t* row_ptr;    // [nbrows+1]
  const int32_t* col_idx;    // [nnzb]
  const int64_t* blk_off;    // [nnzb+1] value offset of each block
  const double* values;
};

// Symbolic row-pass limits (LDS-resident hash of one C block row).  The
// ordinary forms take rows of up to kLargeRowA stored A blocks and
// kLargeRowBlocks result blocks; longer rows go to the huge forms (one
// workgroup per CU), which take up to kMaxRowA and kMaxRowBlocks.
constexpr int kSymThreads = 256;
constexpr int kHashSlots = 2048;       // open-addressing table over block columns (ordinary forms)
constexpr int kLargeRowBlocks = 1024;  // result blocks per C block row, ordinary forms
constexpr int kLargeRowA = 1024;       // stored A blocks per block row, ordinary forms
constexpr int kMaxRowBlocks = 2048;    // result blocks per C block row
constexpr int kMaxRowA = 2048;         // stored A blocks per block row

// Device-side flags raised by kernels (bit mask in a uint32 word).
enum : uint32_t {
  kFlagRowTooManyA = 1u,      // an A block row has more than kMaxRowA blocks
  kFlagRowTooManyC = 2u,      // a C block row has more than kMaxRowBlocks blocks
};
// Error bits of a matrix's size record (dsz[2]); the row flags above too.
constexpr int64_t kErrCapacity = 4;  // a result did not fit the reserved capacity

// Slots of the per-multiply totals array (device int64).
enum : int {
  kTotNnzc = 0,      // result blocks
  kTotNprod = 1,     // kept block products
  kTotNvals = 2,     // result values
  kTotCand = 3,      // candidate products before the filter
  kTotFlags = 4,     // symbolic-pass flags
  kTotFlopHalf = 5,  // sum over kept products of m*n*k
  kTotAbort = 6,     // nonzero: the result does not fit; later kernels do nothing
  kTotPanelMax = 7,  // most products of any stack panel (panelled multiplies)
  kTotPanelUsed = 8, // stack panels that hold a block row (panelled multiplies)
  kTotWide = 9,      // block rows the count pass left to the workgroup forms
  kTotHuge = 10,     // block rows left to the huge forms
  kTotForms = 11,    // kForm* bits: fill forms beyond the tiny one that some row needs
  kTotCount = 12
};

// Row limits of the two smallest workgroup forms of the fill pass (stored A
// blocks, result blocks); rows beyond the small form's take the large form.
constexpr int kTinyRowA = 128, kTinyRowC = 256;
constexpr int kSmallRowA = 256, kSmallRowC = 512;
enum : uint32_t {
  kFormSmall = 1u,  // some row exceeds the tiny form and fits the small one
  kFormLarge = 2u,  // some row exceeds the small form (and is no huge row)
};
// Fill launches (launch_sym_fill): an eager multiply launches only the forms
// the count pass found rows for (and the thin form whenever the stack is built
// in panels: it writes each panel's end offset); a reserved one (graph)
// launches all.
enum : uint32_t {
  kFillThin = 1u, kFillTiny = 2u, kFillSmall = 4u, kFillLarge = 8u, kFillHuge = 16u, kFillAll = 31u,
};

// Doubles of zero slack kept after the last value of every matrix: the
// small-block kernel reads up to 256 values from the start of any block.
constexpr int kValueSlackDoubles = 256;

// Result blocks of the multiply whose totals these are (0 once aborted).
__device__ __forceinline__ int32_t live_nnzc(const int64_t* totals) {
  return totals[kTotAbort] ? 0 : (int32_t)totals[kTotNnzc];
}

// Inputs of the symbolic phase.
struct SymArgs {
  MatView A, B, Cin;
  int use_old;        // beta != 0 and C_in given
  int use_eps;        // filter_eps > 0
  double eps;
  const double* normA;  // [A.nnzb] (only if use_eps)
  const double* normB;  // [B.nnzb] (only if use_eps)
  // Kept prefixes (only if sorted_mode, which needs use_eps): each B block row
  // in descending norm order, bord[row_ptr[k] + r] the B block of rank r and
  // bnrm its norm (rows of more than kSortRow blocks stay unsorted,
  // bsorted[k] = 0).  The products an A entry keeps on a sorted B row are
  // then the first akeep[A entry] of that order (the norm product is
  // monotone in the B norm, so the filter's test selects a prefix): the row
  // passes enumerate only those, the count pass writing akeep for the fill.
  int sorted_mode;
  const int32_t* bord;    // [B.nnzb]
  const double* bnrm;     // [B.nnzb]
  const uint8_t* bsorted; // [B.nbrows]
  int32_t* akeep;         // [A.nnzb]
  const int32_t* c_row_sizes;
  const int32_t* c_col_sizes;
  int32_t c_col_uniform;  // common size of every block column of C, or 0 (then c_col_sizes is read)
  // count pass outputs (length nbrows+1; entry i+1 written for row i)
  int64_t* row_nc;
  int64_t* row_np;
  int64_t* row_nv;
  int64_t* row_ncand;
  int64_t* row_nf;     // m_i * sum over kept products of n_j * k
  uint32_t* flags;
  // rows the one-thread (thin) path leaves to the workgroup forms, listed by
  // the count pass in any order; *n_wide must be zero when the count pass starts
  int32_t* wide;       // [nbrows]
  int32_t* n_wide;
  // rows the ordinary forms leave to the huge forms (listed the same way)
  int32_t* huge;       // [nbrows]
  int32_t* n_huge;
  uint32_t* forms;     // kForm* bits raised by the count pass (zero when it starts)
  // fill pass: only rows [panel[0], panel[1]) are filled, and their products
  // are written from stack position row_pstart[panel[0]] on at index 0 (the
  // stack holds one panel of rows); nullptr = every row, one stack
  const int32_t* panel;
  // fill pass inputs/outputs (exclusive prefixes of the counts, length nbrows+1)
  const int32_t* c_row_ptr;
  const int64_t* row_pstart;
  const int64_t* row_vstart;
  int32_t* c_col_idx;
  int64_t* c_blk_off;
  int64_t* prod_ptr;    // [nnzc+1] start of each C block's products
  int32_t* c_old_idx;   // [nnzc] block of C_in or -1
  int2* prod;           // [nprod] {A block, B block} of every product
  const int64_t* totals;  // per-multiply totals (the fill does nothing once aborted)
};

struct NumArgs {
  MatView A, B, Cin;
  int use_old;
  double alpha, beta;
  int64_t nnzc_bound;      // host bound on the result blocks (exact, or the reserved capacity)
  const int64_t* totals;   // device totals: the result block count, abort flag
  const int32_t* c_row_sizes;
  const int32_t* c_col_sizes;
  const int32_t* c_col_idx;
  const int64_t* c_blk_off;
  const int64_t* prod_ptr;
  const int32_t* c_old_idx;
  const int2* prod;
  double* c_values;
  int wide_inner;          // every inner block edge >= 16: the generic path may use the matrix-core form
  int mid_t16;             // generic path: one 16x16 sub-tile for C blocks with both edges <= 16
  int mid_cpre;            // generic path: load a sub-tile's C_in before its last chunk's multiply
  int uniform;             // common edge of every block of A and B, or 0
  // 23x23 paths: only the C blocks of rows [panel[0], panel[1]) are computed,
  // and prod holds that panel's products from index 0; nullptr = all
  const int32_t* panel;
  const int32_t* c_row_ptr;
};

// Launchers (all enqueue on `s`; they return the launch status).
// Norms of the first *d_nnzb blocks; bound >= *d_nnzb sizes the launch;
// max_block bounds the values of one block (selects the launch shape).
hipError_t launch_block_norms(const int64_t* blk_off, const double* values, const int64_t* d_nnzb, int64_t bound,
                              int64_t max_block, double* out, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
// Zero the value slack after the result and write its size record
// dsz = {nnzb, nvals, error bits}.
hipError_t launch_finish_multiply(const int64_t* totals, double* values, int64_t* dsz, hipStream_t s);
// Reserved multiply: abort (totals[kTotAbort]) if the counted result exceeds
// the capacities or a row limit was met; with big_stack the products may
// exceed 2^31-1 (the stack is built in panels).
hipError_t launch_check_capacity(int64_t* totals, int64_t cap_nnzb, int64_t cap_nvals, int64_t cap_nprod,
                                 int big_stack, hipStream_t s);
// Stacks in panels of rows (23x23 paths): panels[0..np] row bounds from the
// per-row product prefix np_pre, each panel starting at a multiple of
// max(cap - R, half) products (R: the most products of one row), so that no
// panel exceeds cap while R <= cap - half; the largest panel's products go to
// totals[kTotPanelMax] (the multiply is aborted if they exceed cap), the count
// of panels that hold a row to totals[kTotPanelUsed].  Panels past the last
// row are empty.  np <= kMaxPanels.
constexpr int32_t kMaxPanels = 4096;
hipError_t launch_panel_rows(const int64_t* np_pre, int32_t nbrows, int64_t half, int32_t np, int64_t cap,
                             int32_t* panels, int64_t* totals, hipStream_t s);
// Frobenius norm of the first *d_nvals values into out[0] (device); partial
// needs frobenius_tmp_elems() doubles.
int64_t frobenius_tmp_elems();
hipError_t launch_frobenius(const double* values, const int64_t* d_nvals, double* partial, double* out,
                            hipStream_t s);

// Device-wide exclusive scan of n int64 values into out[0..n] (out[n] = total).
// tmp must hold scan_tmp_elems(n) entries; in and out must not overlap.
int64_t scan_tmp_elems(int64_t n);
hipError_t scan_exclusive(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s);
// The same for narr (<= 8) arrays at once (per-row counts).
hipError_t scan_rows(const int64_t* const* in, int64_t* const* out, int narr, int64_t n, int64_t* tmp,
                     hipStream_t s);

// Rank the entries of every B block row by descending norm (ties by block
// index): bord/bnrm/bsorted as described in SymArgs.  B rows of more than
// kSortRow blocks are left unsorted.
constexpr int kSortRow = 2048;
hipError_t launch_sort_row_norms(const MatView& B, const double* normB, int32_t* bord, double* bnrm,
                                 uint8_t* bsorted, hipStream_t s);
hipError_t launch_sym_count(const SymArgs& a, hipStream_t s);
hipError_t launch_sym_fill(const SymArgs& a, uint32_t launch_mask, hipStream_t s);
hipError_t launch_finish_rows(int32_t nbrows, const int64_t* nc_pre, const int64_t* np_pre, const int64_t* nv_pre,
                              int32_t* c_row_ptr, int64_t* prod_ptr, int64_t* c_blk_off, const int64_t* totals,
                              hipStream_t s);
hipError_t launch_gather_totals(int32_t n, const int64_t* nc_pre, const int64_t* np_pre, const int64_t* nv_pre,
                                const int64_t* cand_pre, const int64_t* nf_pre, const uint32_t* flags,
                                int64_t* totals, hipStream_t s);
// `work` holds numeric_work_elems() entries (the 23x23 kernels' schedule).
int64_t numeric_work_elems();
// Schedule of the 23x23 kernels (FP64, split, exact slices): the C blocks of
// the panel (rows [panel[0], panel[1]) of c_row_ptr; all if panel is
// nullptr) in kSliceParts parts of equal product counts, each cut into ns
// slices, written to `work` (see k_product_slices); returns ns.  The kernels
// run on tile23_workgroups() workgroups of four waves.
constexpr int kSliceParts = 8;  // one per XCD
int32_t launch_product_slices(const int64_t* prod_ptr, const int64_t* totals, const int32_t* c_row_ptr,
                              const int32_t* panel, int32_t* work, hipStream_t s);
// Stack position that index 0 of prod holds, stored after the
// slice bounds by k_product_slices.
__device__ __forceinline__ int64_t slices_pbase(const int32_t* bounds, int32_t ns) {
  return *reinterpret_cast<const int64_t*>(bounds + kSliceParts * (ns + 1));
}
int32_t tile23_workgroups();
hipError_t launch_numeric(const NumArgs& a, int uniform_size, int32_t* work, hipStream_t s);

// Small-block path (every block edge <= kSmallEdge): C blocks are partitioned
// by padded shape class, then one persistent launch multiplies all classes.
constexpr int kSmallEdge = 16;
int64_t class_list_tmp_elems(int64_t nnzc_bound);  // entries of cnt and cnt_pre
// list holds two int4 per C block: {m | n << 8, first product, product count, 0}
// and {C value offset, C_in value offset or -1} (int64 pairs).  cnp and qstart
// hold class_entries(bound) (+1) int64: product counts in list order and their
// exclusive scan; desc receives the operand descriptors {A value offset |
// k << 56, B value offset} of every product in list order.
int64_t class_entries(int64_t nnzc_bound);
hipError_t launch_class_lists(const NumArgs& a, int64_t* cnt, int64_t* cnt_pre, int64_t* tmp, int4* list,
                              int32_t* cls_start, int64_t* cnp, int64_t* qstart, int4* desc, hipStream_t s);
// Variants of the small-block kernel: variant v runs class c in form and
// depth small_variant_depths(v)[c]: on the vector units, 1 means the form
// with several products per step (four for 8x8, two for 8x16, 16x8), 8 two
// steps of the 8x8 class for block edges of at most 8, other values the
// products in flight of the one-product form; 16 + d the FP64 matrix-core
// form with d products in flight.  `mask` selects the classes to run (bit c
// = class c).  kSmallDefault is the untuned choice.
constexpr int32_t kSmallVariants = 8;
constexpr int32_t kSmallDefault = 1;  // 8x8 class four products per step, 2 in flight for the others
constexpr int32_t kSmallAllClasses = 15;
void small_variant_depths(int32_t v, int32_t* depths);
// Largest block edge variant v serves (8 for the variant that keeps two steps
// of four 8x8 products in flight; multiplies with larger edges use the default).
int32_t small_variant_max_edge(int32_t v);
hipError_t launch_numeric_small(const NumArgs& a, const int4* list, const int32_t* cls_start, const int64_t* qstart,
                                const int4* desc, int32_t variant, int32_t mask, hipStream_t s);

// Split precision (23x23 blocks): FP64 values -> three BF16 terms per value,
// split_elems(nblocks) uint16 per matrix; transpose = 1 stores each block
// transposed (the B operand).  The numeric kernel multiplies the terms on
// BF16 matrix cores and accumulates each block product into FP64.
int64_t split_elems(int64_t nblocks);
hipError_t launch_split_bf16x3(const double* values, const int64_t* d_nnzb, int64_t bound, int transpose,
                               uint16_t* out, hipStream_t s);
hipError_t launch_numeric_split23(const NumArgs& a, const uint16_t* As, const uint16_t* Bs, int32_t* work,
                                  hipStream_t s);

// Exact-slice precision (23x23 blocks): seven INT8 digits per value under a
// power-of-two scale per row of each block row of A (transpose = 0, scale
// groups = block rows, rowof: scratch of `bound` entries) or per column of
// each block column of B (transpose = 1, groups = block columns);
// slice_bytes(nblocks) bytes of digits, exps[ngroups*23] exponents.
int64_t slice_bytes(int64_t nblocks);
hipError_t launch_slice_int8x7(const double* values, const int64_t* d_nnzb, int64_t bound, int transpose,
                               const int32_t* row_ptr, int32_t nbrows, const int32_t* col_idx, int32_t ngroups,
                               int32_t* rowof, int32_t* exps, uint8_t* out, hipStream_t s);
hipError_t launch_numeric_slice23(const NumArgs& a, const int32_t* c_row_ptr, int32_t nbrows, const uint8_t* As,
                                  const uint8_t* Bs, const int32_t* ea, const int32_t* eb, int32_t* work,
                                  hipStream_t s);

// filter(M, eps) over the first dsz[0] blocks (bound >= dsz[0] sizes the
// launches; keep/vsz/keep_pos/voff are scratch of bound (+1) entries).  The
// new sizes replace dsz[0..1].
hipError_t launch_filter(const int32_t* row_ptr, const int32_t* col_idx, const int64_t* blk_off,
                         const double* values, int32_t nbrows, int64_t* dsz, int64_t bound, const double* norms,
                         double eps, int64_t* keep, int64_t* vsz, int64_t* keep_pos, int64_t* voff, int64_t* tmp,
                         int32_t* out_row_ptr, int32_t* out_col_idx, int64_t* out_blk_off,
                         double* out_values, hipStream_t s);

}  // namespace bsmm
