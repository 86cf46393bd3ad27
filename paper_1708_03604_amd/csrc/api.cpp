// C-ABI of libbsmm: validation, device storage, and the multiply pipeline
//   norms -> symbolic count -> scans -> (one sync to size C) -> symbolic fill
//   -> numeric (with the alpha/beta finalisation fused in).
// The operations follow Section 2 of the paper (blocked CSR, pairwise block
// products, on-the-fly norm filter); see include/bsmm.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bsmm.h"
#include "bsmm_internal.h"

using namespace bsmm;

namespace {

thread_local std::string g_err;

bsmm_status fail(bsmm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(BSMM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// HIP_TRY for the part of a multiply that already rewrites the result matrix C.
#define HIP_W(expr)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return empty_result(C, s, BSMM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Growable device buffer.
template <typename T>
struct DBuf {
  T* p = nullptr;
  int64_t cap = 0;  // elements
  hipError_t ensure(int64_t n) {
    if (n <= cap && p) return hipSuccess;
    int64_t want = std::max<int64_t>(n + n / 4, 16);
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      cap = 0;
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), sizeof(T) * (size_t)want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// Pattern + values of one matrix.  Values carry kValueSlack doubles of slack so that
// kernels may read a little past the last block (never used in results).
struct Storage {
  DBuf<int32_t> row_ptr;
  DBuf<int32_t> col_idx;
  DBuf<int64_t> blk_off;
  DBuf<double> values;
  void release() {
    row_ptr.release();
    col_idx.release();
    blk_off.release();
    values.release();
  }
};

constexpr int64_t kValueSlack = kValueSlackDoubles;
constexpr int kPinned = 32;
// Default stack limit: 2^30 products (8 GB of stack indices); a 23x23
// multiply with more products builds and consumes its stack in panels.
constexpr int64_t kDefaultStackLimit = int64_t(1) << 30;
// B blocks per B block row from which a filtered multiply enumerates kept
// prefixes (molecule rows of ~26 blocks stay below it; semi-empirical rows of
// ~84 and the sign chain's rows of hundreds to 2048 blocks are above it).
constexpr int64_t kSortedRowAvg = 48;

// Panels for `products` block products under a stack limit (half the limit
// per panel start, plus one: see launch_panel_rows).
int64_t panels_for(int64_t products, int64_t limit) {
  const int64_t half = std::max<int64_t>(limit / 2, 1);
  return (products + half - 1) / half + 1;
}

}  // namespace

struct bsmm_matrix {
  int32_t nbrows = 0, nbcols = 0;
  std::vector<int32_t> row_sizes, col_sizes;
  DBuf<int32_t> d_row_sizes, d_col_sizes;
  int32_t nnzb = 0;
  int64_t nvals = 0;
  int uniform = 0;  // common block edge if every row and column size is equal, else 0
  int col_uniform = 0;  // common block edge of the columns, else 0
  int max_edge = 0; // largest row or column block size
  uint32_t row_edges = 0, col_edges = 0;  // bit e-1 set for each block edge e (edges above 32 set bit 31)
  Storage cur, spare;
  // product stack of the last multiply that wrote this matrix
  DBuf<int64_t> prod_ptr;
  DBuf<int2> prod;  // {A block, B block} of every product, in stack order
  DBuf<int32_t> old_idx;
  int64_t nprod = 0;
  bool has_stack = false;
  bsmm_mult_stats stats{};
  // Size record on the device: {nnzb, nvals, error bits, 0}, kept current by
  // every operation that writes the matrix.  A reserved matrix is written
  // without host synchronisation (possibly by graph replays the host does not
  // see), so its host-side sizes and counters are re-read from the device at
  // every synchronising call.
  DBuf<int64_t> dsz;
  int64_t cap_nnzb = 0, cap_nvals = 0, cap_nprod = 0;  // reserved capacity (0: not reserved)
  DBuf<double> frob_tmp;
  // scratch
  DBuf<double> norm_a, norm_b, norm_self;
  DBuf<int32_t> bord, akeep;   // B rows in norm order, kept prefixes of A entries (filtered multiplies)
  DBuf<double> bnrm;           // the norms in that order
  DBuf<uint8_t> bsorted;       // B rows that have an order
  DBuf<int64_t> rows[5], pre[5], scan_tmp, totals, fkeep, fvsz, fpos, fvoff;
  DBuf<uint32_t> flags;
  DBuf<int32_t> work;
  DBuf<int32_t> wide;   // rows for the workgroup forms of the symbolic pass (count in flags[1])
  DBuf<int32_t> huge;   // rows for the huge forms of the symbolic pass (count in flags[2])
  DBuf<int32_t> panels; // row bounds of the stack panels (23x23 paths)
  int64_t stack_limit = kDefaultStackLimit;  // products one stack panel may hold (23x23 paths)
  int64_t cap_stack = 0;        // reserved: stack entries allocated
  int32_t res_panels = 1;       // reserved: stack panels per multiply on the 23x23 paths
  bool stack_panelled = false;  // the last multiply built its stack in panels (not kept)
  DBuf<int4> class_list;          // C blocks by padded shape class (small-block path), 2 per block
  DBuf<int4> prod_desc;           // per product operand offsets (small-block path)
  DBuf<uint16_t> split_a, split_b; // BF16 terms of the operands (split precision)
  DBuf<uint8_t> slice_a, slice_b;  // INT8 digits of the operands (exact-slice precision)
  DBuf<int32_t> slice_ea, slice_eb, slice_rowof;  // their scale exponents; block rows of A's blocks
  DBuf<int64_t> class_cnt, class_pre, class_np, class_q;
  DBuf<int32_t> class_start;
  NumArgs small_args{};  // arguments of the last small-block launch (re-launched by the tuner)
  NumArgs mid_args{};    // arguments of the last generic-path launch (re-launched by the tuner)
  int64_t* h_totals = nullptr;  // pinned, kPinned entries
  // phase timing: 7 events per recorded multiply
  bool timing = false;
  std::vector<hipEvent_t> events;
};

namespace {

MatView view(const bsmm_matrix* m) {
  MatView v;
  v.nbrows = m->nbrows;
  v.nbcols = m->nbcols;
  v.nnzb = m->nnzb;
  v.row_sizes = m->d_row_sizes.p;
  v.col_sizes = m->d_col_sizes.p;
  v.row_ptr = m->cur.row_ptr.p;
  v.col_idx = m->cur.col_idx.p;
  v.blk_off = m->cur.blk_off.p;
  v.values = m->cur.values.p;
  return v;
}

bool is_finite(double x) { return std::isfinite(x); }

bsmm_status check_pattern(int32_t nbrows, int32_t nbcols, int32_t nnzb, const int32_t* rp, const int32_t* ci) {
  if (rp[0] != 0) return fail(BSMM_E_PATTERN, "row_ptr[0] must be 0");
  if (rp[nbrows] != nnzb) return fail(BSMM_E_PATTERN, "row_ptr[nbrows] must equal nnzb");
  for (int32_t i = 0; i < nbrows; ++i) {
    if (rp[i + 1] < rp[i]) return fail(BSMM_E_PATTERN, "row_ptr is not non-decreasing at row " + std::to_string(i));
    for (int32_t b = rp[i]; b < rp[i + 1]; ++b) {
      if (ci[b] < 0 || ci[b] >= nbcols)
        return fail(BSMM_E_PATTERN, "column index out of range at block " + std::to_string(b));
      if (b > rp[i] && ci[b] <= ci[b - 1])
        return fail(BSMM_E_PATTERN, "columns not strictly increasing in row " + std::to_string(i));
    }
  }
  return BSMM_OK;
}

hipError_t ensure_storage(Storage& st, int32_t nbrows, int64_t nnzb, int64_t nvals) {
  hipError_t e;
  if ((e = st.row_ptr.ensure(nbrows + 1)) != hipSuccess) return e;
  if ((e = st.col_idx.ensure(std::max<int64_t>(nnzb, 1))) != hipSuccess) return e;
  if ((e = st.blk_off.ensure(nnzb + 1)) != hipSuccess) return e;
  if ((e = st.values.ensure(nvals + kValueSlack)) != hipSuccess) return e;
  return hipSuccess;
}

bsmm_status ensure_pinned(bsmm_matrix* m) {
  if (!m->h_totals) {
    if (hipHostMalloc(reinterpret_cast<void**>(&m->h_totals), kPinned * sizeof(int64_t), 0) != hipSuccess) {
      m->h_totals = nullptr;
      return fail(BSMM_E_NOMEM, "pinned host allocation failed");
    }
  }
  return BSMM_OK;
}

bool same_sizes(const std::vector<int32_t>& a, const std::vector<int32_t>& b) { return a == b; }

constexpr int kEventsPerMultiply = 7;

void drop_events(bsmm_matrix* m) {
  for (hipEvent_t e : m->events) (void)hipEventDestroy(e);
  m->events.clear();
}

// Event slot `k` of the multiply being recorded (nullptr when not timing).
hipEvent_t* mark(bsmm_matrix* m, size_t base, int k, hipStream_t s) {
  if (!m->timing) return nullptr;
  (void)hipEventRecord(m->events[base + k], s);
  return &m->events[base + k];
}

// Upper bound on the stored blocks / values (exact unless device-sized).
int64_t blocks_bound(const bsmm_matrix* m) { return m->cap_nnzb > 0 ? m->cap_nnzb : m->nnzb; }

// Values of the largest possible block of m.
int64_t max_block(const bsmm_matrix* m) { return (int64_t)m->max_edge * m->max_edge; }

// Bring the host copy of a device-sized matrix's sizes (and of the counters of
// its last multiply) up to date; synchronises `s`.  A reserved operation that
// overflowed leaves the matrix empty and is reported here.
bsmm_status sync_sizes(bsmm_matrix* m, hipStream_t s) {
  if (m->cap_nnzb == 0) return BSMM_OK;
  bsmm_status st = ensure_pinned(m);
  if (st != BSMM_OK) return st;
  // the record may have been written on any stream: with no stream given,
  // wait for the whole device
  if (!s) HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpyAsync(m->h_totals, m->dsz.p, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(m->h_totals + 4, m->totals.p, kTotCount * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t err = m->h_totals[2];
  if (err) {
    m->nnzb = 0;
    m->nvals = 0;
    m->nprod = 0;
    m->has_stack = false;
    m->stack_panelled = false;
    m->stats = bsmm_mult_stats{};
    std::fill(m->stats.variants, m->stats.variants + 4, -1);
    const int64_t zero[3] = {0, 0, 0};
    HIP_TRY(hipMemsetAsync(m->cur.row_ptr.p, 0, sizeof(int32_t) * (m->nbrows + 1), s));
    HIP_TRY(hipMemsetAsync(m->cur.blk_off.p, 0, sizeof(int64_t), s));
    HIP_TRY(hipMemcpyAsync(m->dsz.p, zero, sizeof(zero), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(m->totals.p, 0, kTotCount * sizeof(int64_t), s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err & (kFlagRowTooManyA | kFlagRowTooManyC))
      return fail(BSMM_E_UNSUPPORTED, "a reserved multiply met a block row beyond the symbolic pass limits "
                                      "(A rows <= " + std::to_string(kMaxRowA) + ", C rows <= " +
                                      std::to_string(kMaxRowBlocks) + " blocks); the matrix was emptied");
    return fail(BSMM_E_CAPACITY, "a reserved multiply exceeded the reserved capacity; the matrix was emptied");
  }
  m->nnzb = (int32_t)m->h_totals[0];
  m->nvals = m->h_totals[1];
  const int64_t* t = m->h_totals + 4;
  m->nprod = t[kTotNprod];
  m->stats.candidates = t[kTotCand];
  m->stats.products = t[kTotNprod];
  m->stats.nnzb = t[kTotNnzc];
  m->stats.nvals = t[kTotNvals];
  m->stats.useful_flops = 2.0 * (double)t[kTotFlopHalf];
  // a reserved multiply in stack panels launches every panel its capacity
  // allows; the device counted the ones that held a row
  if (m->stats.panels > 1 && t[kTotPanelUsed] > 0) m->stats.panels = (int32_t)t[kTotPanelUsed];
  return BSMM_OK;
}

// A multiply that failed after it began to rewrite C (device allocation or a
// HIP call): leave C a valid empty matrix without a product stack, so that no
// later call reads half-written storage, and report `code`.
bsmm_status empty_result(bsmm_matrix* C, hipStream_t s, bsmm_status code, const std::string& msg) {
  C->nnzb = 0;
  C->nvals = 0;
  C->nprod = 0;
  C->has_stack = false;
  C->stack_panelled = false;
  C->stats = bsmm_mult_stats{};
  std::fill(C->stats.variants, C->stats.variants + 4, -1);
  const int64_t zero[4] = {0, 0, 0, 0};
  if (ensure_storage(C->cur, C->nbrows, 0, 0) == hipSuccess &&
      hipMemsetAsync(C->cur.row_ptr.p, 0, sizeof(int32_t) * (C->nbrows + 1), s) == hipSuccess &&
      hipMemsetAsync(C->cur.blk_off.p, 0, sizeof(int64_t), s) == hipSuccess &&
      hipMemcpyAsync(C->dsz.p, zero, 3 * sizeof(int64_t), hipMemcpyHostToDevice, s) == hipSuccess)
    (void)hipStreamSynchronize(s);
  return fail(code, msg + " (the result matrix was left empty)");
}

// Tuning table of the small-block path: tuning key -> variant per shape class.
using ClassVariants = std::array<int32_t, 4>;
std::mutex g_tune_mu;
std::map<uint64_t, ClassVariants> g_tune;

uint64_t tune_key(const bsmm_matrix* A, const bsmm_matrix* B) {
  return (uint64_t)(A->row_edges & 0xffffu) | (uint64_t)(A->col_edges & 0xffffu) << 16 |
         (uint64_t)(B->col_edges & 0xffffu) << 32;
}

// Variants per class for a multiply with key `key` and largest block edge
// `edge` (a variant that does not serve the edge falls back to the default).
ClassVariants tuned_variants(uint64_t key, int32_t edge) {
  ClassVariants v{kSmallDefault, kSmallDefault, kSmallDefault, kSmallDefault};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) v = it->second;
  }
  for (auto& x : v)
    if (edge > small_variant_max_edge(x)) x = kSmallDefault;
  return v;
}

// Tuning table of the generic path: edge masks (A's rows, A's columns, B's
// columns) -> variant (bit 0: one 16x16 sub-tile for C blocks with both
// edges <= 16; bit 1: the matrix-core form where every inner edge is >= 16;
// bit 2: C_in loaded before each sub-tile's last chunk).
using MidKey = std::array<uint32_t, 3>;
std::map<MidKey, int32_t> g_tune_mid;

MidKey mid_key(const bsmm_matrix* A, const bsmm_matrix* B) { return {A->row_edges, A->col_edges, B->col_edges}; }

bool mid_wide(const bsmm_matrix* A) { return (A->col_edges & 0x7fffu) == 0; }  // no inner block edge below 16

// Variant of the generic path for A*B: the table entry, else the untuned
// choice (32x32 sub-tiles, the matrix-core form where allowed); bit 1 is
// dropped when an inner edge is below 16.
int32_t mid_variant(const bsmm_matrix* A, const bsmm_matrix* B) {
  const bool wide = mid_wide(A);
  int32_t v = wide ? 2 : 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_mid.find(mid_key(A, B));
    if (it != g_tune_mid.end()) v = it->second;
  }
  return wide ? v : (v & ~2);
}

struct EventPair {
  hipEvent_t e[2] = {nullptr, nullptr};
  ~EventPair() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

}  // namespace

// One small-block launch per distinct variant, over the classes that use it.
hipError_t launch_small_plan(const NumArgs& na, const bsmm_matrix* C, const ClassVariants& v, hipStream_t s) {
  int32_t done = 0;
  for (int c = 0; c < 4; ++c) {
    if (done & (1 << c)) continue;
    int32_t mask = 0;
    for (int d = c; d < 4; ++d)
      if (v[d] == v[c]) mask |= 1 << d;
    done |= mask;
    const hipError_t e =
        launch_numeric_small(na, C->class_list.p, C->class_start.p, C->class_q.p, C->prod_desc.p, v[c], mask, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

extern "C" {

const char* bsmm_last_error(void) { return g_err.c_str(); }

bsmm_status bsmm_create(bsmm_mat* out, int32_t nbrows, int32_t nbcols, const int32_t* row_sizes,
                        const int32_t* col_sizes, int32_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                        const double* values, int ptr_kind, void* stream) {
  g_err.clear();
  if (!out) return fail(BSMM_E_ARG, "out is NULL");
  if (nbrows < 0 || nbcols < 0 || nnzb < 0) return fail(BSMM_E_ARG, "negative size");
  if (ptr_kind != BSMM_PTR_HOST && ptr_kind != BSMM_PTR_DEVICE) return fail(BSMM_E_ARG, "bad ptr_kind");
  if ((nbrows > 0 && !row_sizes) || (nbcols > 0 && !col_sizes) || !row_ptr || (nnzb > 0 && !col_idx))
    return fail(BSMM_E_ARG, "NULL array");
  for (int32_t i = 0; i < nbrows; ++i)
    if (row_sizes[i] < 1) return fail(BSMM_E_ARG, "row size < 1");
  for (int32_t j = 0; j < nbcols; ++j)
    if (col_sizes[j] < 1) return fail(BSMM_E_ARG, "column size < 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<int32_t> rp(nbrows + 1), ci(nnzb);
  if (ptr_kind == BSMM_PTR_HOST) {
    std::memcpy(rp.data(), row_ptr, sizeof(int32_t) * (nbrows + 1));
    if (nnzb) std::memcpy(ci.data(), col_idx, sizeof(int32_t) * nnzb);
  } else {
    HIP_TRY(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int32_t) * (nbrows + 1), hipMemcpyDeviceToHost, s));
    if (nnzb) HIP_TRY(hipMemcpyAsync(ci.data(), col_idx, sizeof(int32_t) * nnzb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  bsmm_status st = check_pattern(nbrows, nbcols, nnzb, rp.data(), ci.data());
  if (st != BSMM_OK) return st;
  std::vector<int64_t> off(nnzb + 1);
  off[0] = 0;
  for (int32_t i = 0; i < nbrows; ++i)
    for (int32_t b = rp[i]; b < rp[i + 1]; ++b) off[b + 1] = off[b] + (int64_t)row_sizes[i] * col_sizes[ci[b]];
  const int64_t nvals = off[nnzb];

  bsmm_matrix* m = new (std::nothrow) bsmm_matrix();
  if (!m) return fail(BSMM_E_NOMEM, "host allocation failed");
  m->nbrows = nbrows;
  m->nbcols = nbcols;
  m->row_sizes.assign(row_sizes, row_sizes + nbrows);
  m->col_sizes.assign(col_sizes, col_sizes + nbcols);
  int u = nbrows > 0 ? row_sizes[0] : (nbcols > 0 ? col_sizes[0] : 0);
  for (int32_t i = 0; i < nbrows && u; ++i)
    if (row_sizes[i] != u) u = 0;
  for (int32_t j = 0; j < nbcols && u; ++j)
    if (col_sizes[j] != u) u = 0;
  m->uniform = u;
  int cu = nbcols > 0 ? col_sizes[0] : 0;
  for (int32_t j = 0; j < nbcols && cu; ++j)
    if (col_sizes[j] != cu) cu = 0;
  m->col_uniform = cu;
  for (int32_t i = 0; i < nbrows; ++i) m->max_edge = std::max(m->max_edge, row_sizes[i]);
  for (int32_t j = 0; j < nbcols; ++j) m->max_edge = std::max(m->max_edge, col_sizes[j]);
  for (int32_t i = 0; i < nbrows; ++i) m->row_edges |= 1u << (std::min(row_sizes[i], 32) - 1);
  for (int32_t j = 0; j < nbcols; ++j) m->col_edges |= 1u << (std::min(col_sizes[j], 32) - 1);
  std::fill(m->stats.variants, m->stats.variants + 4, -1);
  m->nnzb = nnzb;
  m->nvals = nvals;
  auto cleanup = [&](bsmm_status code, const std::string& msg) {
    bsmm_destroy(m);
    return fail(code, msg);
  };
  if (m->d_row_sizes.ensure(std::max(nbrows, 1)) != hipSuccess ||
      m->d_col_sizes.ensure(std::max(nbcols, 1)) != hipSuccess ||
      ensure_storage(m->cur, nbrows, nnzb, nvals) != hipSuccess || m->dsz.ensure(4) != hipSuccess ||
      m->norm_self.ensure(std::max(nnzb, 1)) != hipSuccess || m->frob_tmp.ensure(frobenius_tmp_elems()) != hipSuccess)
    return cleanup(BSMM_E_NOMEM, "device allocation failed");
  const int64_t sizes[4] = {nnzb, nvals, 0, 0};
  hipError_t e = hipSuccess;
  if (nbrows) e = hipMemcpyAsync(m->d_row_sizes.p, row_sizes, sizeof(int32_t) * nbrows, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && nbcols)
    e = hipMemcpyAsync(m->d_col_sizes.p, col_sizes, sizeof(int32_t) * nbcols, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->cur.row_ptr.p, rp.data(), sizeof(int32_t) * (nbrows + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && nnzb)
    e = hipMemcpyAsync(m->cur.col_idx.p, ci.data(), sizeof(int32_t) * nnzb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->cur.blk_off.p, off.data(), sizeof(int64_t) * (nnzb + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    if (values && nvals)
      e = hipMemcpyAsync(m->cur.values.p, values, sizeof(double) * nvals,
                         ptr_kind == BSMM_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s);
    else if (nvals)
      e = hipMemsetAsync(m->cur.values.p, 0, sizeof(double) * nvals, s);
  }
  if (e == hipSuccess) e = hipMemsetAsync(m->cur.values.p + nvals, 0, sizeof(double) * kValueSlack, s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->dsz.p, sizes, sizeof(sizes), hipMemcpyHostToDevice, s);
  // host buffers (rp, ci, off, sizes) die at return: finish the copies first
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(BSMM_E_HIP, std::string("create: ") + hipGetErrorString(e));
  *out = m;
  return BSMM_OK;
}

bsmm_status bsmm_destroy(bsmm_mat m) {
  if (!m) return BSMM_OK;
  (void)hipDeviceSynchronize();
  m->cur.release();
  m->spare.release();
  m->d_row_sizes.release();
  m->d_col_sizes.release();
  m->prod_ptr.release();
  m->prod.release();
  m->old_idx.release();
  m->norm_a.release();
  m->norm_b.release();
  m->bord.release();
  m->akeep.release();
  m->bnrm.release();
  m->bsorted.release();
  m->norm_self.release();
  for (auto& b : m->rows) b.release();
  for (auto& b : m->pre) b.release();
  m->scan_tmp.release();
  m->totals.release();
  m->fkeep.release();
  m->fvsz.release();
  m->fpos.release();
  m->fvoff.release();
  m->flags.release();
  m->work.release();
  m->wide.release();
  m->class_list.release();
  m->prod_desc.release();
  m->split_a.release();
  m->split_b.release();
  m->slice_a.release();
  m->slice_b.release();
  for (auto* b : {&m->slice_ea, &m->slice_eb, &m->slice_rowof}) b->release();
  m->class_cnt.release();
  m->class_np.release();
  m->class_q.release();
  m->class_pre.release();
  m->class_start.release();
  m->dsz.release();
  m->frob_tmp.release();
  m->huge.release();
  m->panels.release();
  if (m->h_totals) (void)hipHostFree(m->h_totals);
  drop_events(m);
  delete m;
  return BSMM_OK;
}

bsmm_status bsmm_norms(bsmm_mat m, double* out, void* stream) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  if (!out && blocks_bound(m) > 0) return fail(BSMM_E_ARG, "NULL output");
  HIP_TRY(launch_block_norms(m->cur.blk_off.p, m->cur.values.p, m->dsz.p, blocks_bound(m), max_block(m), out,
                             reinterpret_cast<hipStream_t>(stream)));
  return BSMM_OK;
}

bsmm_status bsmm_info(bsmm_mat m, int32_t* nbrows, int32_t* nbcols, int32_t* nnzb, int64_t* nvals) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  bsmm_status st = sync_sizes(m, nullptr);
  if (st != BSMM_OK) return st;
  if (nbrows) *nbrows = m->nbrows;
  if (nbcols) *nbcols = m->nbcols;
  if (nnzb) *nnzb = m->nnzb;
  if (nvals) *nvals = m->nvals;
  return BSMM_OK;
}

bsmm_status bsmm_export(bsmm_mat m, int32_t* row_ptr, int32_t* col_idx, double* values, int ptr_kind,
                        void* stream) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  if (ptr_kind != BSMM_PTR_HOST && ptr_kind != BSMM_PTR_DEVICE) return fail(BSMM_E_ARG, "bad ptr_kind");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bsmm_status st = sync_sizes(m, s);
  if (st != BSMM_OK) return st;
  const hipMemcpyKind k = ptr_kind == BSMM_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (row_ptr) HIP_TRY(hipMemcpyAsync(row_ptr, m->cur.row_ptr.p, sizeof(int32_t) * (m->nbrows + 1), k, s));
  if (col_idx && m->nnzb) HIP_TRY(hipMemcpyAsync(col_idx, m->cur.col_idx.p, sizeof(int32_t) * m->nnzb, k, s));
  if (values && m->nvals) HIP_TRY(hipMemcpyAsync(values, m->cur.values.p, sizeof(double) * m->nvals, k, s));
  HIP_TRY(hipStreamSynchronize(s));
  return BSMM_OK;
}

bsmm_status bsmm_export_stack(bsmm_mat C, int32_t* st_c, int32_t* st_a, int32_t* st_b, int64_t* nprod,
                              int ptr_kind, void* stream) {
  g_err.clear();
  if (!C) return fail(BSMM_E_ARG, "NULL handle");
  if (ptr_kind != BSMM_PTR_HOST && ptr_kind != BSMM_PTR_DEVICE) return fail(BSMM_E_ARG, "bad ptr_kind");
  bsmm_status st = sync_sizes(C, reinterpret_cast<hipStream_t>(stream));
  if (st != BSMM_OK) return st;
  if (C->stack_panelled)
    return fail(BSMM_E_UNSUPPORTED, "the last multiply built its product stack in panels, which are not kept");
  if (!C->has_stack) {
    if (nprod) *nprod = 0;
    return BSMM_OK;
  }
  if (nprod) *nprod = C->nprod;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t np = C->nprod;
  std::vector<int64_t> pp(C->nnzb + 1);
  std::vector<int32_t> a(np), b(np), c(np);
  std::vector<int2> ab(np);
  HIP_TRY(hipMemcpyAsync(pp.data(), C->prod_ptr.p, sizeof(int64_t) * (C->nnzb + 1), hipMemcpyDeviceToHost, s));
  if (np) {
    HIP_TRY(hipMemcpyAsync(ab.data(), C->prod.p, sizeof(int2) * np, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (int64_t y = 0; y < np; ++y) {
    a[y] = ab[y].x;
    b[y] = ab[y].y;
  }
  for (int32_t x = 0; x < C->nnzb; ++x)
    for (int64_t y = pp[x]; y < pp[x + 1]; ++y) c[y] = x;
  const hipMemcpyKind k = ptr_kind == BSMM_PTR_HOST ? hipMemcpyHostToHost : hipMemcpyHostToDevice;
  if (np) {
    if (st_c) HIP_TRY(hipMemcpyAsync(st_c, c.data(), sizeof(int32_t) * np, k, s));
    if (st_a) HIP_TRY(hipMemcpyAsync(st_a, a.data(), sizeof(int32_t) * np, k, s));
    if (st_b) HIP_TRY(hipMemcpyAsync(st_b, b.data(), sizeof(int32_t) * np, k, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return BSMM_OK;
}

bsmm_status bsmm_timing(bsmm_mat C, int enable) {
  g_err.clear();
  if (!C) return fail(BSMM_E_ARG, "NULL handle");
  drop_events(C);
  C->timing = enable != 0;
  return BSMM_OK;
}

bsmm_status bsmm_phase_times(bsmm_mat C, double* ms, int64_t* count) {
  g_err.clear();
  if (!C || !ms) return fail(BSMM_E_ARG, "NULL argument");
  for (int k = 0; k < BSMM_NPHASES; ++k) ms[k] = 0.0;
  const size_t n = C->events.size() / kEventsPerMultiply;
  for (size_t x = 0; x < n; ++x) {
    hipEvent_t* e = &C->events[x * kEventsPerMultiply];
    HIP_TRY(hipEventSynchronize(e[6]));
    float t;
    // e0 start, e1 after norms, e2 after count+scans, e3 before fill, e4 after fill, e5 after numeric, e6 end
    HIP_TRY(hipEventElapsedTime(&t, e[0], e[1]));
    ms[BSMM_PHASE_NORMS] += t;
    HIP_TRY(hipEventElapsedTime(&t, e[1], e[2]));
    ms[BSMM_PHASE_COUNT] += t;
    HIP_TRY(hipEventElapsedTime(&t, e[2], e[3]));
    ms[BSMM_PHASE_SIZING] += t;
    HIP_TRY(hipEventElapsedTime(&t, e[3], e[4]));
    ms[BSMM_PHASE_FILL] += t;
    HIP_TRY(hipEventElapsedTime(&t, e[4], e[5]));
    ms[BSMM_PHASE_NUMERIC] += t;
    HIP_TRY(hipEventElapsedTime(&t, e[0], e[6]));
    ms[BSMM_PHASE_TOTAL] += t;
  }
  if (count) *count = (int64_t)n;
  return BSMM_OK;
}

bsmm_status bsmm_stats(bsmm_mat C, bsmm_mult_stats* out) {
  g_err.clear();
  if (!C || !out) return fail(BSMM_E_ARG, "NULL argument");
  bsmm_status st = sync_sizes(C, nullptr);
  if (st != BSMM_OK) return st;
  *out = C->stats;
  return BSMM_OK;
}

bsmm_status bsmm_multiply(double alpha, bsmm_mat A, bsmm_mat B, double beta, bsmm_mat C_in, bsmm_mat C,
                          double filter_eps, int prec, void* stream) {
  g_err.clear();
  if (!A || !B || !C) return fail(BSMM_E_ARG, "NULL handle");
  if (!is_finite(alpha) || !is_finite(beta) || !is_finite(filter_eps))
    return fail(BSMM_E_ARG, "alpha, beta and filter_eps must be finite");
  if (prec != BSMM_FP64 && prec != BSMM_SPLIT_F32X2 && prec != BSMM_SPLIT_BF16X3 && prec != BSMM_SLICE_INT8X7)
    return fail(BSMM_E_ARG, "unknown precision");
  if (prec == BSMM_SPLIT_F32X2)
    return fail(BSMM_E_UNSUPPORTED, "the two-term FP32 split is not built (FP32 matrix cores run at twice the FP64 "
                                    "rate and the split needs three products, so it cannot beat FP64)");
  if (C == A || C == B) return fail(BSMM_E_ALIAS, "output must not be an input operand");
  if (A->nbcols != B->nbrows || !same_sizes(A->col_sizes, B->row_sizes))
    return fail(BSMM_E_SHAPE, "A column block sizes differ from B row block sizes");
  if (!same_sizes(C->row_sizes, A->row_sizes) || !same_sizes(C->col_sizes, B->col_sizes))
    return fail(BSMM_E_SHAPE, "C block sizes must be A's row sizes and B's column sizes");
  const bool use_old = beta != 0.0 && C_in != nullptr;
  if (use_old && (!same_sizes(C_in->row_sizes, A->row_sizes) || !same_sizes(C_in->col_sizes, B->col_sizes)))
    return fail(BSMM_E_SHAPE, "C_in block sizes must be A's row sizes and B's column sizes");
  const int uniform = (A->uniform && A->uniform == B->uniform) ? A->uniform : 0;
  const bool split = prec == BSMM_SPLIT_BF16X3;
  if (split && uniform != 23) return fail(BSMM_E_UNSUPPORTED, "split precision is built for uniform 23x23 blocks");
  const bool slice = prec == BSMM_SLICE_INT8X7;
  if (slice && uniform != 23)
    return fail(BSMM_E_UNSUPPORTED, "exact-slice precision is built for uniform 23x23 blocks");
  const bool use_eps = filter_eps > 0.0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int32_t nbrows = A->nbrows;
  bsmm_status st = ensure_pinned(C);
  if (st != BSMM_OK) return st;

  size_t ev = 0;
  if (C->timing) {
    ev = C->events.size();
    for (int k = 0; k < kEventsPerMultiply; ++k) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      C->events.push_back(e);
    }
  }
  mark(C, ev, 0, s);
  // Reserved output: every size stays on the device and nothing below
  // allocates or synchronises (graph-capturable); the bounds are capacities.
  const bool reserved = C->cap_nnzb > 0;
  // scratch
  if (C->flags.ensure(4) != hipSuccess || C->work.ensure(numeric_work_elems()) != hipSuccess || C->totals.ensure(kTotCount) != hipSuccess ||
      C->scan_tmp.ensure(scan_tmp_elems(nbrows) + 2) != hipSuccess)
    return fail(BSMM_E_NOMEM, "scratch allocation failed");
  for (int x = 0; x < 5; ++x)
    if (C->rows[x].ensure(nbrows + 1) != hipSuccess || C->pre[x].ensure(nbrows + 1) != hipSuccess)
      return fail(BSMM_E_NOMEM, "scratch allocation failed");
  if (C->wide.ensure(std::max(nbrows, 1)) != hipSuccess || C->huge.ensure(std::max(nbrows, 1)) != hipSuccess)
    return fail(BSMM_E_NOMEM, "scratch allocation failed");
  const double* normA = nullptr;
  const double* normB = nullptr;
  if (use_eps) {
    const int64_t ba = blocks_bound(A), bb = blocks_bound(B);
    if (C->norm_a.ensure(std::max<int64_t>(ba, 1)) != hipSuccess)
      return fail(BSMM_E_NOMEM, "scratch allocation failed");
    HIP_TRY(launch_block_norms(A->cur.blk_off.p, A->cur.values.p, A->dsz.p, ba, max_block(A), C->norm_a.p, s));
    normA = C->norm_a.p;
    if (B == A) {
      normB = normA;
    } else {
      if (C->norm_b.ensure(std::max<int64_t>(bb, 1)) != hipSuccess)
        return fail(BSMM_E_NOMEM, "scratch allocation failed");
      HIP_TRY(launch_block_norms(B->cur.blk_off.p, B->cur.values.p, B->dsz.p, bb, max_block(B), C->norm_b.p, s));
      normB = C->norm_b.p;
    }
  }
  // Filtered multiplies over long B rows enumerate only the kept products of
  // each A entry (a prefix of its B row in descending norm order); short rows
  // gain less from it than the sort costs.  Results are the same either way.
  const int64_t b_blocks = B->cap_nnzb > 0 ? B->cap_nnzb : B->nnzb;
  const bool sorted_mode = use_eps && b_blocks >= kSortedRowAvg * (int64_t)B->nbrows;
  if (sorted_mode) {
    const int64_t ba = blocks_bound(A), bb = blocks_bound(B);
    if (C->bord.ensure(std::max<int64_t>(bb, 1)) != hipSuccess ||
        C->bnrm.ensure(std::max<int64_t>(bb, 1)) != hipSuccess ||
        C->bsorted.ensure(std::max<int64_t>(B->nbrows, 1)) != hipSuccess ||
        C->akeep.ensure(std::max<int64_t>(ba, 1)) != hipSuccess)
      return fail(BSMM_E_NOMEM, "scratch allocation failed");
    HIP_TRY(launch_sort_row_norms(view(B), normB, C->bord.p, C->bnrm.p, C->bsorted.p, s));
  }
  // symbolic-pass flags, the wide- and huge-row counts, the fill forms needed
  HIP_TRY(launch_zero_u32(C->flags.p, 4, s));
  mark(C, ev, 1, s);

  SymArgs g{};
  g.A = view(A);
  g.B = view(B);
  if (use_old) g.Cin = view(C_in);
  g.use_old = use_old ? 1 : 0;
  g.use_eps = use_eps ? 1 : 0;
  g.eps = filter_eps;
  g.normA = normA;
  g.normB = normB;
  g.sorted_mode = sorted_mode ? 1 : 0;
  g.bord = C->bord.p;
  g.bnrm = C->bnrm.p;
  g.bsorted = C->bsorted.p;
  g.akeep = C->akeep.p;
  g.c_row_sizes = C->d_row_sizes.p;
  g.c_col_sizes = C->d_col_sizes.p;
  g.c_col_uniform = C->col_uniform;
  g.row_nc = C->rows[0].p;
  g.row_np = C->rows[1].p;
  g.row_nv = C->rows[2].p;
  g.row_ncand = C->rows[3].p;
  g.row_nf = C->rows[4].p;
  g.flags = C->flags.p;
  g.wide = C->wide.p;
  g.n_wide = reinterpret_cast<int32_t*>(C->flags.p + 1);
  g.huge = C->huge.p;
  g.n_huge = reinterpret_cast<int32_t*>(C->flags.p + 2);
  g.forms = C->flags.p + 3;
  g.totals = C->totals.p;
  HIP_TRY(launch_sym_count(g, s));
  {
    const int64_t* in[5];
    int64_t* outp[5];
    for (int x = 0; x < 5; ++x) {
      in[x] = C->rows[x].p;
      outp[x] = C->pre[x].p;
    }
    HIP_TRY(scan_rows(in, outp, 5, nbrows, C->scan_tmp.p, s));
  }
  HIP_TRY(launch_gather_totals(nbrows, C->pre[0].p, C->pre[1].p, C->pre[2].p, C->pre[3].p, C->pre[4].p,
                               C->flags.p, C->totals.p, s));
  mark(C, ev, 2, s);

  // The 23x23 paths may build and consume the stack in panels of block rows
  // (at most stack_limit products each); the other paths build it whole.
  const bool panel_ok = uniform == 23;
  int32_t npanels = 1;
  int32_t used_panels = 0;  // eager multiplies: the panels that hold a row (the rest are empty)
  uint32_t fill_mask = kFillAll;  // eager multiplies: only the fill forms the count pass found rows for
  int64_t nnzc = 0, nprod = 0, nvals = 0, ncand = 0, nflop_half = 0;
  int64_t nnzc_bound, nprod_bound, nvals_bound, stack_bound;
  if (reserved) {
    npanels = panel_ok ? C->res_panels : 1;
    HIP_TRY(launch_check_capacity(C->totals.p, C->cap_nnzb, C->cap_nvals, panel_ok ? C->cap_nprod : C->cap_stack,
                                  npanels > 1 ? 1 : 0, s));
    if (npanels > 1)
      HIP_TRY(launch_panel_rows(C->pre[1].p, nbrows, std::max<int64_t>(C->cap_stack / 2, 1), npanels, C->cap_stack,
                                C->panels.p, C->totals.p, s));
    nnzc_bound = C->cap_nnzb;
    nprod_bound = C->cap_stack;
    nvals_bound = C->cap_nvals;
    stack_bound = C->cap_stack;
  } else {
    HIP_TRY(hipMemcpyAsync(C->h_totals, C->totals.p, kTotCount * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    nnzc = C->h_totals[kTotNnzc];
    nprod = C->h_totals[kTotNprod];
    nvals = C->h_totals[kTotNvals];
    ncand = C->h_totals[kTotCand];
    nflop_half = C->h_totals[kTotFlopHalf];
    {
      // launch only the fill forms some row needs
      const int64_t nw = C->h_totals[kTotWide], nh = C->h_totals[kTotHuge];
      const uint32_t forms = (uint32_t)C->h_totals[kTotForms];
      fill_mask = (nw < nbrows ? kFillThin : 0u) | (nw > nh ? kFillTiny : 0u) |
                  ((forms & kFormSmall) ? kFillSmall : 0u) | ((forms & kFormLarge) ? kFillLarge : 0u) |
                  (nh > 0 ? kFillHuge : 0u);
    }
    const uint32_t flags = (uint32_t)C->h_totals[kTotFlags];
    if (flags & kFlagRowTooManyA)
      return fail(BSMM_E_UNSUPPORTED, "an A block row holds more than " + std::to_string(kMaxRowA) + " blocks");
    if (flags & kFlagRowTooManyC)
      return fail(BSMM_E_UNSUPPORTED,
                  "a result block row would hold more than " + std::to_string(kMaxRowBlocks) + " blocks");
    if (nnzc > 0x7fffffffLL) return fail(BSMM_E_CAPACITY, "result has more than 2^31-1 blocks");
    stack_bound = nprod;
    if (panel_ok && nprod > C->stack_limit) {
      const int64_t np = panels_for(nprod, C->stack_limit);
      if (np > kMaxPanels)
        return fail(BSMM_E_CAPACITY, std::to_string(nprod) + " block products need more than " +
                                         std::to_string(kMaxPanels) + " stack panels at the stack limit of " +
                                         std::to_string(C->stack_limit) + " (bsmm_set_stack_limit)");
      npanels = (int32_t)np;
      if (C->panels.ensure(npanels + 1) != hipSuccess) return fail(BSMM_E_NOMEM, "scratch allocation failed");
      HIP_TRY(launch_panel_rows(C->pre[1].p, nbrows, std::max<int64_t>(C->stack_limit / 2, 1), npanels,
                                C->stack_limit, C->panels.p, C->totals.p, s));
      HIP_TRY(hipMemcpyAsync(C->h_totals + kTotCount, C->totals.p + kTotPanelMax, 2 * sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (C->h_totals[kTotCount] > C->stack_limit)
        return fail(BSMM_E_CAPACITY, "a stack panel would hold " + std::to_string(C->h_totals[kTotCount]) +
                                         " block products, above the stack limit of " +
                                         std::to_string(C->stack_limit) +
                                         " (a block row holds more than half of it; bsmm_set_stack_limit)");
      stack_bound = C->stack_limit;
      used_panels = (int32_t)C->h_totals[kTotCount + 1];
    } else if (nprod > 0x7fffffffLL) {
      return fail(BSMM_E_CAPACITY, "more than 2^31-1 block products");
    }
    nnzc_bound = nnzc;
    nprod_bound = nprod;
    nvals_bound = nvals;
  }

  // Every check that can reject the call has run: from here on C's storage
  // and stack are rewritten.  A resource failure past this point leaves C a
  // valid empty matrix without a stack (empty_result).
  C->has_stack = false;
  C->stack_panelled = false;
  // output storage: in place -> write the spare storage and swap afterwards
  const bool in_place = use_old && C_in == C;
  Storage& out = in_place ? C->spare : C->cur;
  if (ensure_storage(out, nbrows, nnzc_bound, nvals_bound) != hipSuccess ||
      C->prod_ptr.ensure(nnzc_bound + 1) != hipSuccess ||
      C->prod.ensure(std::max<int64_t>(stack_bound, 1)) != hipSuccess ||
      C->old_idx.ensure(std::max<int64_t>(nnzc_bound, 1)) != hipSuccess)
    return empty_result(C, s, BSMM_E_NOMEM, "device allocation for the result failed");
  const bool small = !split && !slice && uniform != 23 && std::max(A->max_edge, B->max_edge) <= kSmallEdge;
  if (split) {
    if (C->split_a.ensure(split_elems(std::max<int64_t>(blocks_bound(A), 1))) != hipSuccess ||
        C->split_b.ensure(split_elems(std::max<int64_t>(blocks_bound(B), 1))) != hipSuccess)
      return empty_result(C, s, BSMM_E_NOMEM, "device allocation for the split operands failed");
  }
  if (slice) {
    const int64_t ba = std::max<int64_t>(blocks_bound(A), 1), bb = std::max<int64_t>(blocks_bound(B), 1);
    if (C->slice_a.ensure(slice_bytes(ba)) != hipSuccess || C->slice_b.ensure(slice_bytes(bb)) != hipSuccess ||
        C->slice_ea.ensure(23 * std::max<int64_t>(A->nbrows, 1)) != hipSuccess ||
        C->slice_eb.ensure(23 * std::max<int64_t>(B->nbcols, 1)) != hipSuccess ||
        C->slice_rowof.ensure(ba) != hipSuccess)
      return empty_result(C, s, BSMM_E_NOMEM, "device allocation for the slice operands failed");
  }
  if (small) {
    const int64_t ncl = class_list_tmp_elems(nnzc_bound), nce = class_entries(nnzc_bound);
    if (C->class_list.ensure(2 * std::max<int64_t>(nnzc_bound, 1)) != hipSuccess ||
        C->prod_desc.ensure(std::max<int64_t>(nprod_bound, 1)) != hipSuccess ||
        C->class_cnt.ensure(ncl) != hipSuccess || C->class_pre.ensure(ncl) != hipSuccess ||
        C->class_np.ensure(std::max<int64_t>(nce, 1)) != hipSuccess || C->class_q.ensure(nce + 1) != hipSuccess ||
        C->class_start.ensure(5) != hipSuccess ||
        C->scan_tmp.ensure(std::max({scan_tmp_elems(nbrows), scan_tmp_elems(ncl), scan_tmp_elems(nce)}) + 2) !=
            hipSuccess)
      return empty_result(C, s, BSMM_E_NOMEM, "device allocation for the block classes failed");
  }
  // a reallocation above may have freed C_in's storage only if C_in == C and
  // `out` is cur; that case is excluded by writing the spare.
  if (use_old) g.Cin = view(C_in);
  mark(C, ev, 3, s);
  HIP_W(launch_finish_rows(nbrows, C->pre[0].p, C->pre[1].p, C->pre[2].p, out.row_ptr.p, C->prod_ptr.p,
                             out.blk_off.p, C->totals.p, s));
  g.c_row_ptr = out.row_ptr.p;
  g.row_pstart = C->pre[1].p;
  g.row_vstart = C->pre[2].p;
  g.c_col_idx = out.col_idx.p;
  g.c_blk_off = out.blk_off.p;
  g.prod_ptr = C->prod_ptr.p;
  g.c_old_idx = C->old_idx.p;
  g.prod = C->prod.p;

  NumArgs na{};
  na.A = g.A;
  na.B = g.B;
  na.Cin = g.Cin;
  na.use_old = g.use_old;
  na.alpha = alpha;
  na.beta = beta;
  na.nnzc_bound = nnzc_bound;
  na.totals = C->totals.p;
  na.c_row_sizes = C->d_row_sizes.p;
  na.c_col_sizes = C->d_col_sizes.p;
  na.c_col_idx = out.col_idx.p;
  na.c_blk_off = out.blk_off.p;
  na.prod_ptr = C->prod_ptr.p;
  na.c_old_idx = C->old_idx.p;
  na.prod = C->prod.p;
  na.c_values = out.values.p;
  const int32_t midv = mid_variant(A, B);
  na.wide_inner = (midv >> 1) & 1;
  na.mid_t16 = midv & 1;
  na.mid_cpre = (midv >> 2) & 1;
  na.uniform = uniform;
  na.c_row_ptr = out.row_ptr.p;
  ClassVariants variants{-1, -1, -1, -1};
  // One pass per stack panel: fill the panel's rows (pattern and products),
  // then multiply them.  With panels, the fill phase time covers the first
  // panel's fill and the numeric phase everything after it.
  for (int32_t pnl = 0; pnl < npanels; ++pnl) {
    g.panel = npanels > 1 ? C->panels.p + pnl : nullptr;
    na.panel = g.panel;
    HIP_W(launch_sym_fill(g, fill_mask, s));
    if (pnl == 0) mark(C, ev, 4, s);
    if (split) {
      if (pnl == 0) {
        HIP_W(launch_split_bf16x3(A->cur.values.p, A->dsz.p, blocks_bound(A), 0, C->split_a.p, s));
        HIP_W(launch_split_bf16x3(B->cur.values.p, B->dsz.p, blocks_bound(B), 1, C->split_b.p, s));
      }
      HIP_W(launch_numeric_split23(na, C->split_a.p, C->split_b.p, C->work.p, s));
    } else if (slice) {
      if (pnl == 0) {
        HIP_W(launch_slice_int8x7(A->cur.values.p, A->dsz.p, blocks_bound(A), 0, A->cur.row_ptr.p, A->nbrows,
                                    nullptr, A->nbrows, C->slice_rowof.p, C->slice_ea.p, C->slice_a.p, s));
        HIP_W(launch_slice_int8x7(B->cur.values.p, B->dsz.p, blocks_bound(B), 1, nullptr, 0, B->cur.col_idx.p,
                                    B->nbcols, nullptr, C->slice_eb.p, C->slice_b.p, s));
      }
      HIP_W(launch_numeric_slice23(na, out.row_ptr.p, nbrows, C->slice_a.p, C->slice_b.p, C->slice_ea.p,
                                     C->slice_eb.p, C->work.p, s));
    } else if (small) {
      HIP_W(launch_class_lists(na, C->class_cnt.p, C->class_pre.p, C->scan_tmp.p, C->class_list.p,
                                 C->class_start.p, C->class_np.p, C->class_q.p, C->prod_desc.p, s));
      variants = tuned_variants(tune_key(A, B), std::max(A->max_edge, B->max_edge));
      HIP_W(launch_small_plan(na, C, variants, s));
      C->small_args = na;
    } else {
      HIP_W(launch_numeric(na, uniform, C->work.p, s));
      if (uniform != 23) variants = {midv, -1, -1, -1};
    }
  }
  if (!small && uniform != 23) C->mid_args = na;
  mark(C, ev, 5, s);
  HIP_W(launch_finish_multiply(C->totals.p, out.values.p, C->dsz.p, s));
  mark(C, ev, 6, s);

  if (in_place) std::swap(C->cur, C->spare);
  C->has_stack = npanels == 1;
  C->stack_panelled = npanels > 1;
  C->stats.panels = used_panels > 0 ? used_panels : npanels;
  C->stats.path = split ? BSMM_PATH_SPLIT23 : slice ? BSMM_PATH_SLICE23 : small ? BSMM_PATH_SMALL : uniform == 23 ? BSMM_PATH_TILE23 : BSMM_PATH_GENERIC;
  std::copy(variants.begin(), variants.end(), C->stats.variants);
  if (reserved) return BSMM_OK;
  C->nnzb = (int32_t)nnzc;
  C->nvals = nvals;
  C->nprod = nprod;
  C->stats.candidates = ncand;
  C->stats.products = nprod;
  C->stats.nnzb = nnzc;
  C->stats.nvals = nvals;
  C->stats.useful_flops = 2.0 * (double)nflop_half;
  if (C->norm_self.ensure(std::max<int64_t>(nnzc, 1)) != hipSuccess)
    return empty_result(C, s, BSMM_E_NOMEM, "scratch allocation failed");
  return BSMM_OK;
}

bsmm_status bsmm_filter(bsmm_mat m, double eps, void* stream) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  if (!is_finite(eps)) return fail(BSMM_E_ARG, "eps must be finite");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bsmm_status st = ensure_pinned(m);
  if (st != BSMM_OK) return st;
  const bool reserved = m->cap_nnzb > 0;
  const int64_t bound = reserved ? m->cap_nnzb : m->nnzb;
  const int64_t vbound = reserved ? m->cap_nvals : m->nvals;
  if (m->norm_self.ensure(std::max<int64_t>(bound, 1)) != hipSuccess || m->fkeep.ensure(bound + 1) != hipSuccess ||
      m->fvsz.ensure(bound + 1) != hipSuccess || m->fpos.ensure(bound + 1) != hipSuccess ||
      m->fvoff.ensure(bound + 1) != hipSuccess ||
      m->scan_tmp.ensure(std::max(scan_tmp_elems(bound), scan_tmp_elems(m->nbrows)) + 2) != hipSuccess ||
      ensure_storage(m->spare, m->nbrows, bound, vbound) != hipSuccess)
    return fail(BSMM_E_NOMEM, "scratch allocation failed");
  HIP_TRY(launch_block_norms(m->cur.blk_off.p, m->cur.values.p, m->dsz.p, bound, max_block(m), m->norm_self.p, s));
  HIP_TRY(launch_filter(m->cur.row_ptr.p, m->cur.col_idx.p, m->cur.blk_off.p, m->cur.values.p, m->nbrows, m->dsz.p,
                        bound, m->norm_self.p, eps, m->fkeep.p, m->fvsz.p, m->fpos.p, m->fvoff.p, m->scan_tmp.p,
                        m->spare.row_ptr.p, m->spare.col_idx.p, m->spare.blk_off.p, m->spare.values.p, s));
  std::swap(m->cur, m->spare);
  m->has_stack = false;  // block indices changed
  m->stack_panelled = false;
  if (reserved) return BSMM_OK;
  HIP_TRY(hipMemcpyAsync(m->h_totals, m->dsz.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  m->nnzb = (int32_t)m->h_totals[0];
  m->nvals = m->h_totals[1];
  return BSMM_OK;
}

}  // extern "C"

namespace {

// Scratch of bsmm_filter_noalloc: file-scope device memory (one copy on every
// GPU the library runs on, held until the process ends).  Host code never
// passes `scratch` itself to a kernel: it takes the device address from
// hipGetSymbolAddress, once per device, with that device current.
constexpr int64_t kNoAllocMaxBlocks = 131072;
constexpr size_t kNoAllocScratchBytes = 6u << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (nullptr on failure,
// with the reason in g_err).
void* noalloc_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    g_err = "no current HIP device (or device index beyond " + std::to_string(kMaxDevices) + ")";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      g_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

bsmm_status bsmm_filter_noalloc(bsmm_mat m, double eps, void* stream) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  if (!is_finite(eps)) return fail(BSMM_E_ARG, "eps must be finite");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool reserved = m->cap_nnzb > 0;
  const int64_t bound = reserved ? m->cap_nnzb : m->nnzb;
  const int64_t vbound = reserved ? m->cap_nvals : m->nvals;
  if (bound > kNoAllocMaxBlocks)
    return fail(BSMM_E_CAPACITY, "bsmm_filter_noalloc handles at most " + std::to_string(kNoAllocMaxBlocks) +
                                     " blocks (reserved capacity for a reserved matrix); this matrix has " +
                                     std::to_string(bound));
  // the result goes to the matrix's second storage, which must already exist
  if (!m->spare.row_ptr.p || m->spare.row_ptr.cap < m->nbrows + 1 || m->spare.col_idx.cap < std::max<int64_t>(bound, 1) ||
      m->spare.blk_off.cap < bound + 1 || m->spare.values.cap < vbound + kValueSlack)
    return fail(BSMM_E_CAPACITY, "bsmm_filter_noalloc needs the matrix's second storage at its size: reserve the "
                                 "matrix (bsmm_reserve) or filter it once with bsmm_filter first");
  // scratch layout: norms[bound], keep[bound+1], vsz[bound+1], keep_pos[bound+1],
  // voff[bound+1], scan temporaries; each part 256-byte aligned
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t nb = up(sizeof(double) * std::max<int64_t>(bound, 1));
  const size_t ni = up(sizeof(int64_t) * (bound + 1));
  const size_t nt = up(sizeof(int64_t) * (std::max(scan_tmp_elems(bound), scan_tmp_elems(m->nbrows)) + 2));
  if (nb + 4 * ni + nt > kNoAllocScratchBytes)
    return fail(BSMM_E_CAPACITY, "bsmm_filter_noalloc: the scan temporaries of " + std::to_string(m->nbrows) +
                                     " block rows exceed the fixed scratch");
  unsigned char* base = static_cast<unsigned char*>(noalloc_scratch());
  if (!base) return fail(BSMM_E_HIP, g_err);
  double* norms = reinterpret_cast<double*>(base);
  int64_t* keep = reinterpret_cast<int64_t*>(base + nb);
  int64_t* vsz = reinterpret_cast<int64_t*>(base + nb + ni);
  int64_t* kpos = reinterpret_cast<int64_t*>(base + nb + 2 * ni);
  int64_t* voff = reinterpret_cast<int64_t*>(base + nb + 3 * ni);
  int64_t* tmp = reinterpret_cast<int64_t*>(base + nb + 4 * ni);
  // every scratch entry the kernels read is written first by this call
  // (flags past the live block count are written as zeros), so stale
  // contents of an earlier call do not matter
  HIP_TRY(launch_block_norms(m->cur.blk_off.p, m->cur.values.p, m->dsz.p, bound, max_block(m), norms, s));
  HIP_TRY(launch_filter(m->cur.row_ptr.p, m->cur.col_idx.p, m->cur.blk_off.p, m->cur.values.p, m->nbrows, m->dsz.p,
                        bound, norms, eps, keep, vsz, kpos, voff, tmp, m->spare.row_ptr.p, m->spare.col_idx.p,
                        m->spare.blk_off.p, m->spare.values.p, s));
  std::swap(m->cur, m->spare);
  m->has_stack = false;  // block indices changed
  m->stack_panelled = false;
  if (reserved) return BSMM_OK;
  int64_t sizes[2] = {0, 0};  // pageable host memory: a synchronous read-back, no allocation
  HIP_TRY(hipMemcpyAsync(sizes, m->dsz.p, sizeof(sizes), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  m->nnzb = (int32_t)sizes[0];
  m->nvals = sizes[1];
  return BSMM_OK;
}

bsmm_status bsmm_reserve(bsmm_mat m, int64_t max_nnzb, int64_t max_nvals, int64_t max_products, void* stream) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  if (max_nnzb < 1 || max_nvals < 1 || max_products < 1) return fail(BSMM_E_ARG, "capacities must be >= 1");
  if (max_nnzb > 0x7fffffffLL) return fail(BSMM_E_CAPACITY, "the block capacity is limited to 2^31-1");
  // a uniform 23x23 output takes its products in stack panels of at most
  // stack_limit entries; other outputs hold the whole stack
  const bool panel_ok = m->uniform == 23;
  if (!panel_ok && max_products > 0x7fffffffLL)
    return fail(BSMM_E_CAPACITY, "the product capacity is limited to 2^31-1 unless the blocks are 23x23");
  const int64_t cstack = panel_ok ? std::min(max_products, m->stack_limit) : max_products;
  const int64_t npanels = cstack < max_products ? panels_for(max_products, m->stack_limit) : 1;
  if (npanels > kMaxPanels)
    return fail(BSMM_E_CAPACITY, "the product capacity needs more than " + std::to_string(kMaxPanels) +
                                     " stack panels at the stack limit of " + std::to_string(m->stack_limit));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bsmm_status st = sync_sizes(m, s);
  if (st != BSMM_OK) return st;
  st = ensure_pinned(m);
  if (st != BSMM_OK) return st;
  const int64_t cb = std::max<int64_t>(max_nnzb, m->nnzb), cv = std::max<int64_t>(max_nvals, m->nvals);
  const int64_t cp = max_products;
  const int32_t nbrows = m->nbrows;
  // grow the current storage without losing its contents
  if (m->cur.col_idx.cap < cb || m->cur.blk_off.cap < cb + 1 || m->cur.values.cap < cv + kValueSlack) {
    Storage fresh;
    if (ensure_storage(fresh, nbrows, cb, cv) != hipSuccess) {
      fresh.release();
      return fail(BSMM_E_NOMEM, "device allocation for the reservation failed");
    }
    HIP_TRY(hipMemcpyAsync(fresh.row_ptr.p, m->cur.row_ptr.p, sizeof(int32_t) * (nbrows + 1),
                           hipMemcpyDeviceToDevice, s));
    if (m->nnzb)
      HIP_TRY(hipMemcpyAsync(fresh.col_idx.p, m->cur.col_idx.p, sizeof(int32_t) * m->nnzb, hipMemcpyDeviceToDevice,
                             s));
    HIP_TRY(hipMemcpyAsync(fresh.blk_off.p, m->cur.blk_off.p, sizeof(int64_t) * (m->nnzb + 1),
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(fresh.values.p, m->cur.values.p, sizeof(double) * (m->nvals + kValueSlack),
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    m->cur.release();
    m->cur = fresh;
  }
  const int64_t ncl = class_list_tmp_elems(cb), nce = class_entries(cb);
  const int64_t tmp = std::max({scan_tmp_elems(nbrows), scan_tmp_elems(ncl), scan_tmp_elems(cb), scan_tmp_elems(nce)}) + 2;
  // the small-block path's descriptors and class lists (16 bytes per
  // product) only where that path can write this matrix: C's block edges are
  // A's row and B's column edges, so an edge above kSmallEdge rules it out
  const bool small_ok = m->max_edge <= kSmallEdge;
  bool ok = ensure_storage(m->spare, nbrows, cb, cv) == hipSuccess && m->prod_ptr.ensure(cb + 1) == hipSuccess &&
            m->prod.ensure(cstack) == hipSuccess &&
            m->panels.ensure(npanels + 1) == hipSuccess &&
            m->old_idx.ensure(cb) == hipSuccess &&
            (!small_ok ||
             (m->prod_desc.ensure(cp) == hipSuccess && m->class_list.ensure(2 * cb) == hipSuccess &&
              m->class_cnt.ensure(ncl) == hipSuccess && m->class_pre.ensure(ncl) == hipSuccess &&
              m->class_start.ensure(5) == hipSuccess && m->class_np.ensure(nce) == hipSuccess &&
              m->class_q.ensure(nce + 1) == hipSuccess)) &&
            m->scan_tmp.ensure(tmp) == hipSuccess && m->totals.ensure(kTotCount) == hipSuccess &&
            m->flags.ensure(4) == hipSuccess && m->work.ensure(numeric_work_elems()) == hipSuccess &&
            m->norm_a.ensure(cb) == hipSuccess && m->norm_b.ensure(cb) == hipSuccess &&
            m->norm_self.ensure(cb) == hipSuccess && m->fkeep.ensure(cb + 1) == hipSuccess &&
            m->fvsz.ensure(cb + 1) == hipSuccess && m->fpos.ensure(cb + 1) == hipSuccess &&
            m->fvoff.ensure(cb + 1) == hipSuccess;
  for (int x = 0; x < 5 && ok; ++x)
    ok = m->rows[x].ensure(nbrows + 1) == hipSuccess && m->pre[x].ensure(nbrows + 1) == hipSuccess;
  ok = ok && m->wide.ensure(std::max(nbrows, 1)) == hipSuccess && m->huge.ensure(std::max(nbrows, 1)) == hipSuccess;
  if (!ok) return fail(BSMM_E_NOMEM, "device allocation for the reservation failed");
  // counters read back before the first reserved multiply: zero
  if (!m->has_stack) {
    HIP_TRY(hipMemsetAsync(m->totals.p, 0, kTotCount * sizeof(int64_t), s));
    HIP_TRY(hipStreamSynchronize(s));
  } else {
    const int64_t t[kTotCount] = {m->stats.nnzb, m->nprod, m->stats.nvals, m->stats.candidates, 0,
                                  (int64_t)(m->stats.useful_flops / 2), 0, 0};
    HIP_TRY(hipMemcpyAsync(m->totals.p, t, sizeof(t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  m->cap_nnzb = cb;
  m->cap_nvals = cv;
  m->cap_nprod = cp;
  m->cap_stack = cstack;
  m->res_panels = (int32_t)npanels;
  return BSMM_OK;
}

bsmm_status bsmm_set_stack_limit(bsmm_mat m, int64_t max_products) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  if (max_products < 2 || max_products > 0x7fffffffLL)
    return fail(BSMM_E_ARG, "the stack limit must be in 2 .. 2^31-1 products");
  if (m->cap_nnzb > 0) return fail(BSMM_E_ARG, "set the stack limit before bsmm_reserve");
  m->stack_limit = max_products;
  return BSMM_OK;
}

bsmm_status bsmm_frobenius(bsmm_mat m, double* out, void* stream) {
  g_err.clear();
  if (!m || !out) return fail(BSMM_E_ARG, "NULL argument");
  HIP_TRY(launch_frobenius(m->cur.values.p, m->dsz.p + 1, m->frob_tmp.p, out, reinterpret_cast<hipStream_t>(stream)));
  return BSMM_OK;
}

struct bsmm_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

bsmm_status bsmm_capture_begin(void* stream) {
  g_err.clear();
  if (!stream) return fail(BSMM_E_ARG, "capture needs a created stream, not the default stream");
  HIP_TRY(hipStreamBeginCapture(reinterpret_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal));
  return BSMM_OK;
}

bsmm_status bsmm_capture_end(void* stream, bsmm_graph* out) {
  g_err.clear();
  if (!stream || !out) return fail(BSMM_E_ARG, "NULL argument");
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamEndCapture(reinterpret_cast<hipStream_t>(stream), &graph));
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(BSMM_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  bsmm_graph g = new (std::nothrow) bsmm_graph_s();
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return fail(BSMM_E_NOMEM, "host allocation failed");
  }
  g->graph = graph;
  g->exec = exec;
  *out = g;
  return BSMM_OK;
}

bsmm_status bsmm_graph_launch(bsmm_graph g, void* stream) {
  g_err.clear();
  if (!g) return fail(BSMM_E_ARG, "NULL graph");
  HIP_TRY(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)));
  return BSMM_OK;
}

bsmm_status bsmm_graph_destroy(bsmm_graph g) {
  if (!g) return BSMM_OK;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return BSMM_OK;
}

bsmm_status bsmm_tune_small(double alpha, bsmm_mat A, bsmm_mat B, double beta, bsmm_mat C_in, bsmm_mat C,
                            double filter_eps, int32_t reps, int32_t* variants_out, double* ms_out, void* stream) {
  g_err.clear();
  if (!variants_out) return fail(BSMM_E_ARG, "NULL variants_out");
  if (reps < 1 || reps > 1000) return fail(BSMM_E_ARG, "reps must be in 1 .. 1000");
  if (C && C == C_in && beta != 0.0) return fail(BSMM_E_ARG, "tuning needs C_in distinct from C_out");
  if (C && C->cap_nnzb > 0) return fail(BSMM_E_ARG, "tuning does not take a reserved output");
  bsmm_status st = bsmm_multiply(alpha, A, B, beta, C_in, C, filter_eps, BSMM_FP64, stream);
  if (st != BSMM_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::fill(variants_out, variants_out + 4, -1);
  if (ms_out) std::fill(ms_out, ms_out + 4 * kSmallVariants, 0.0);
  if (C->stats.path != BSMM_PATH_SMALL) {
    HIP_TRY(hipStreamSynchronize(s));
    return BSMM_OK;
  }
  // Each launch recomputes C_out's values from A, B and C_in (never from
  // C_out itself), so repeated launches leave the same result.
  const NumArgs& na = C->small_args;
  EventPair ev;
  HIP_TRY(hipEventCreate(&ev.e[0]));
  HIP_TRY(hipEventCreate(&ev.e[1]));
  double best_ms[4] = {HUGE_VAL, HUGE_VAL, HUGE_VAL, HUGE_VAL};
  ClassVariants best{kSmallDefault, kSmallDefault, kSmallDefault, kSmallDefault};
  const int32_t edge = std::max(A->max_edge, B->max_edge);
  for (int32_t v = 0; v < kSmallVariants; ++v) {
    if (edge > small_variant_max_edge(v)) continue;  // not valid for these sizes: not timed
    for (int c = 0; c < 4; ++c) {
      HIP_TRY(hipEventRecord(ev.e[0], s));
      for (int32_t r = 0; r < reps; ++r)
        HIP_TRY(launch_numeric_small(na, C->class_list.p, C->class_start.p, C->class_q.p, C->prod_desc.p, v, 1 << c,
                                     s));
      HIP_TRY(hipEventRecord(ev.e[1], s));
      HIP_TRY(hipEventSynchronize(ev.e[1]));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
      if (ms_out) ms_out[4 * v + c] = ms;
      if (ms < best_ms[c]) {
        best_ms[c] = ms;
        best[c] = v;
      }
    }
  }
  HIP_TRY(launch_small_plan(na, C, best, s));
  HIP_TRY(hipStreamSynchronize(s));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(A, B)] = best;
  }
  std::copy(best.begin(), best.end(), C->stats.variants);
  std::copy(best.begin(), best.end(), variants_out);
  return BSMM_OK;
}

bsmm_status bsmm_tune_mid(double alpha, bsmm_mat A, bsmm_mat B, double beta, bsmm_mat C_in, bsmm_mat C,
                          double filter_eps, int32_t reps, int32_t* variant_out, double* ms_out, void* stream) {
  g_err.clear();
  if (!variant_out) return fail(BSMM_E_ARG, "NULL variant_out");
  if (reps < 1 || reps > 1000) return fail(BSMM_E_ARG, "reps must be in 1 .. 1000");
  if (C && C == C_in && beta != 0.0) return fail(BSMM_E_ARG, "tuning needs C_in distinct from C_out");
  if (C && C->cap_nnzb > 0) return fail(BSMM_E_ARG, "tuning does not take a reserved output");
  bsmm_status st = bsmm_multiply(alpha, A, B, beta, C_in, C, filter_eps, BSMM_FP64, stream);
  if (st != BSMM_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  *variant_out = -1;
  if (ms_out) std::fill(ms_out, ms_out + BSMM_MID_VARIANTS, 0.0);
  if (C->stats.path != BSMM_PATH_GENERIC) {
    HIP_TRY(hipStreamSynchronize(s));
    return BSMM_OK;
  }
  // Each launch recomputes C_out's values from A, B and C_in (never from
  // C_out itself), so repeated launches leave the same result.
  NumArgs na = C->mid_args;
  EventPair ev;
  HIP_TRY(hipEventCreate(&ev.e[0]));
  HIP_TRY(hipEventCreate(&ev.e[1]));
  const bool wide = mid_wide(A);
  double best_ms = HUGE_VAL;
  int32_t best = 0;
  for (int32_t v = 0; v < BSMM_MID_VARIANTS; ++v) {
    if ((v & 2) && !wide) continue;  // the matrix-core form needs inner edges >= 16: not timed
    na.wide_inner = (v >> 1) & 1;
    na.mid_t16 = v & 1;
    na.mid_cpre = (v >> 2) & 1;
    HIP_TRY(hipEventRecord(ev.e[0], s));
    for (int32_t r = 0; r < reps; ++r) HIP_TRY(launch_numeric(na, 0, C->work.p, s));
    HIP_TRY(hipEventRecord(ev.e[1], s));
    HIP_TRY(hipEventSynchronize(ev.e[1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    if (ms_out) ms_out[v] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  na.wide_inner = (best >> 1) & 1;
  na.mid_t16 = best & 1;
  na.mid_cpre = (best >> 2) & 1;
  HIP_TRY(launch_numeric(na, 0, C->work.p, s));
  HIP_TRY(hipStreamSynchronize(s));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_mid[mid_key(A, B)] = best;
  }
  C->mid_args = na;
  C->stats.variants[0] = best;
  *variant_out = best;
  return BSMM_OK;
}

bsmm_status bsmm_mid_key(bsmm_mat A, bsmm_mat B, uint32_t* masks) {
  g_err.clear();
  if (!A || !B || !masks) return fail(BSMM_E_ARG, "NULL argument");
  const MidKey k = mid_key(A, B);
  std::copy(k.begin(), k.end(), masks);
  return BSMM_OK;
}

bsmm_status bsmm_mid_set(const uint32_t* masks, int32_t variant) {
  g_err.clear();
  if (!masks) return fail(BSMM_E_ARG, "NULL masks");
  if (variant < -1 || variant >= BSMM_MID_VARIANTS) return fail(BSMM_E_ARG, "variant out of range");
  const MidKey k{masks[0], masks[1], masks[2]};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (variant < 0)
    g_tune_mid.erase(k);
  else
    g_tune_mid[k] = variant;
  return BSMM_OK;
}

bsmm_status bsmm_mid_get(const uint32_t* masks, int32_t* variant) {
  g_err.clear();
  if (!masks || !variant) return fail(BSMM_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_mid.find(MidKey{masks[0], masks[1], masks[2]});
  *variant = it == g_tune_mid.end() ? -1 : it->second;
  return BSMM_OK;
}

bsmm_status bsmm_mid_entries(uint32_t* masks, int32_t* variants, int32_t cap, int32_t* n) {
  g_err.clear();
  if (!n || cap < 0 || (cap > 0 && (!masks || !variants))) return fail(BSMM_E_ARG, "bad arguments");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int32_t i = 0;
  for (const auto& kv : g_tune_mid) {
    if (i >= cap) break;
    std::copy(kv.first.begin(), kv.first.end(), masks + 3 * i);
    variants[i] = kv.second;
    ++i;
  }
  *n = (int32_t)g_tune_mid.size();
  return BSMM_OK;
}

bsmm_status bsmm_small_variant(int32_t v, int32_t* depths) {
  g_err.clear();
  if (!depths) return fail(BSMM_E_ARG, "NULL depths");
  if (v < 0 || v >= kSmallVariants) return fail(BSMM_E_ARG, "variant out of range");
  small_variant_depths(v, depths);
  return BSMM_OK;
}

bsmm_status bsmm_tune_key(bsmm_mat A, bsmm_mat B, uint64_t* key) {
  g_err.clear();
  if (!A || !B || !key) return fail(BSMM_E_ARG, "NULL argument");
  if (std::max(A->max_edge, B->max_edge) > kSmallEdge)
    return fail(BSMM_E_UNSUPPORTED, "a block edge exceeds " + std::to_string(kSmallEdge));
  *key = tune_key(A, B);
  return BSMM_OK;
}

bsmm_status bsmm_tune_set(uint64_t key, const int32_t* variants) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!variants) {
    g_tune.erase(key);
    return BSMM_OK;
  }
  ClassVariants v;
  for (int c = 0; c < 4; ++c) {
    if (variants[c] < 0 || variants[c] >= kSmallVariants) return fail(BSMM_E_ARG, "variant out of range");
    v[c] = variants[c];
  }
  g_tune[key] = v;
  return BSMM_OK;
}

bsmm_status bsmm_tune_get(uint64_t key, int32_t* variants) {
  g_err.clear();
  if (!variants) return fail(BSMM_E_ARG, "NULL variants");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  for (int c = 0; c < 4; ++c) variants[c] = it == g_tune.end() ? -1 : it->second[c];
  return BSMM_OK;
}

bsmm_status bsmm_tune_entries(uint64_t* keys, int32_t* variants, int32_t cap, int32_t* n) {
  g_err.clear();
  if (!n || cap < 0 || (cap > 0 && (!keys || !variants))) return fail(BSMM_E_ARG, "bad arguments");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int32_t i = 0;
  for (const auto& kv : g_tune) {
    if (i >= cap) break;
    keys[i] = kv.first;
    for (int c = 0; c < 4; ++c) variants[4 * i + c] = kv.second[c];
    ++i;
  }
  *n = (int32_t)g_tune.size();
  return BSMM_OK;
}

}  // extern "C"
