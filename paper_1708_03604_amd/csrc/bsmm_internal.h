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

// Symbolic row-pass limits (LDS-resident hash of one C block row).
constexpr int kSymThreads = 256;
constexpr int kHashSlots = 2048;   // open-addressing table over block columns
constexpr int kMaxRowBlocks = 1024; // result blocks per C block row
constexpr int kMaxRowA = 1024;      // stored A blocks per block row

// Device-side flags raised by kernels (bit mask in a uint32 word).
enum : uint32_t {
  kFlagRowTooManyA = 1u,      // an A block row has more than kMaxRowA blocks
  kFlagRowTooManyC = 2u,      // a C block row has more than kMaxRowBlocks blocks
};

// Inputs of the symbolic phase.
struct SymArgs {
  MatView A, B, Cin;
  int use_old;        // beta != 0 and C_in given
  int use_eps;        // filter_eps > 0
  double eps;
  const double* normA;  // [A.nnzb] (only if use_eps)
  const double* normB;  // [B.nnzb] (only if use_eps)
  const int32_t* c_row_sizes;
  const int32_t* c_col_sizes;
  // count pass outputs (length nbrows+1; entry i+1 written for row i)
  int64_t* row_nc;
  int64_t* row_np;
  int64_t* row_nv;
  int64_t* row_ncand;
  int64_t* row_nf;     // m_i * sum over kept products of n_j * k
  uint32_t* flags;
  // fill pass inputs/outputs (exclusive prefixes of the counts, length nbrows+1)
  const int32_t* c_row_ptr;
  const int64_t* row_pstart;
  const int64_t* row_vstart;
  int32_t* c_col_idx;
  int64_t* c_blk_off;
  int64_t* prod_ptr;    // [nnzc+1] start of each C block's products
  int32_t* c_old_idx;   // [nnzc] block of C_in or -1
  int32_t* prod_a;      // [nprod]
  int32_t* prod_b;      // [nprod]
};

struct NumArgs {
  MatView A, B, Cin;
  int use_old;
  double alpha, beta;
  int32_t nnzc;
  const int32_t* c_row_sizes;
  const int32_t* c_col_sizes;
  const int32_t* c_col_idx;
  const int64_t* c_blk_off;
  const int64_t* prod_ptr;
  const int32_t* c_old_idx;
  const int32_t* prod_a;
  const int32_t* prod_b;
  double* c_values;
};

// Launchers (all enqueue on `s`; they return the launch status).
hipError_t launch_block_norms(const int64_t* blk_off, const double* values, int32_t nnzb, double* out,
                              hipStream_t s);

// Device-wide exclusive scan of n int64 values into out[0..n] (out[n] = total).
// tmp must hold scan_tmp_elems(n) entries; in and out must not overlap.
int64_t scan_tmp_elems(int64_t n);
hipError_t scan_exclusive(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s);
// The same for narr (<= 8) arrays at once (per-row counts).
hipError_t scan_rows(const int64_t* const* in, int64_t* const* out, int narr, int64_t n, int64_t* tmp,
                     hipStream_t s);

hipError_t launch_sym_count(const SymArgs& a, hipStream_t s);
hipError_t launch_sym_fill(const SymArgs& a, hipStream_t s);
hipError_t launch_finish_rows(int32_t nbrows, const int64_t* nc_pre, const int64_t* np_pre, const int64_t* nv_pre,
                              int32_t* c_row_ptr, int64_t* prod_ptr, int64_t* c_blk_off, hipStream_t s);
hipError_t launch_gather_totals(int32_t n, const int64_t* nc_pre, const int64_t* np_pre, const int64_t* nv_pre,
                                const int64_t* cand_pre, const int64_t* nf_pre, const uint32_t* flags,
                                int64_t* totals, hipStream_t s);
hipError_t launch_numeric(const NumArgs& a, int uniform_size, int32_t* work, hipStream_t s);

// filter(M, eps): keep/vsz/keep_pos/voff are scratch of nnzb (+1) entries.
hipError_t launch_filter(const int32_t* row_ptr, const int32_t* col_idx, const int64_t* blk_off,
                         const double* values, int32_t nbrows, int32_t nnzb, const double* norms, double eps,
                         int64_t* keep, int64_t* vsz, int64_t* keep_pos, int64_t* voff, int64_t* tmp,
                         int32_t* out_row_ptr, int32_t* out_col_idx, int64_t* out_blk_off,
                         double* out_values, hipStream_t s);

}  // namespace bsmm
