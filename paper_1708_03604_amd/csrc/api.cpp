// C-ABI of libbsmm: validation, device storage, and the multiply pipeline
//   norms -> symbolic count -> scans -> (one sync to size C) -> symbolic fill
//   -> numeric (with the alpha/beta finalisation fused in).
// The operations follow Section 2 of the paper (blocked CSR, pairwise block
// products, on-the-fly norm filter); see include/bsmm.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
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

// Pattern + values of one matrix.  Values carry 64 doubles of slack so that
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

constexpr int64_t kValueSlack = 64;

}  // namespace

struct bsmm_matrix {
  int32_t nbrows = 0, nbcols = 0;
  std::vector<int32_t> row_sizes, col_sizes;
  DBuf<int32_t> d_row_sizes, d_col_sizes;
  int32_t nnzb = 0;
  int64_t nvals = 0;
  int uniform = 0;  // common block edge if every row and column size is equal, else 0
  Storage cur, spare;
  // product stack of the last multiply that wrote this matrix
  DBuf<int64_t> prod_ptr;
  DBuf<int32_t> prod_a, prod_b, old_idx;
  int64_t nprod = 0;
  bool has_stack = false;
  bsmm_mult_stats stats{};
  // scratch
  DBuf<double> norm_a, norm_b, norm_self;
  DBuf<int64_t> rows[5], pre[5], scan_tmp, totals, fkeep, fvsz, fpos, fvoff;
  DBuf<uint32_t> flags;
  DBuf<int32_t> work;
  int64_t* h_totals = nullptr;  // pinned, 8 entries
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
    if (hipHostMalloc(reinterpret_cast<void**>(&m->h_totals), 8 * sizeof(int64_t), 0) != hipSuccess) {
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

}  // namespace

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
  m->nnzb = nnzb;
  m->nvals = nvals;
  auto cleanup = [&](bsmm_status code, const std::string& msg) {
    bsmm_destroy(m);
    return fail(code, msg);
  };
  if (m->d_row_sizes.ensure(std::max(nbrows, 1)) != hipSuccess ||
      m->d_col_sizes.ensure(std::max(nbcols, 1)) != hipSuccess ||
      ensure_storage(m->cur, nbrows, nnzb, nvals) != hipSuccess)
    return cleanup(BSMM_E_NOMEM, "device allocation failed");
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
  // host buffers (rp, ci, off) die at return: finish the copies first
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
  m->prod_a.release();
  m->prod_b.release();
  m->old_idx.release();
  m->norm_a.release();
  m->norm_b.release();
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
  if (m->h_totals) (void)hipHostFree(m->h_totals);
  drop_events(m);
  delete m;
  return BSMM_OK;
}

bsmm_status bsmm_norms(bsmm_mat m, double* out, void* stream) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  if (!out && m->nnzb > 0) return fail(BSMM_E_ARG, "NULL output");
  HIP_TRY(launch_block_norms(m->cur.blk_off.p, m->cur.values.p, m->nnzb, out,
                             reinterpret_cast<hipStream_t>(stream)));
  return BSMM_OK;
}

bsmm_status bsmm_info(bsmm_mat m, int32_t* nbrows, int32_t* nbcols, int32_t* nnzb, int64_t* nvals) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
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
  if (!C->has_stack) {
    if (nprod) *nprod = 0;
    return BSMM_OK;
  }
  if (nprod) *nprod = C->nprod;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t np = C->nprod;
  std::vector<int64_t> pp(C->nnzb + 1);
  std::vector<int32_t> a(np), b(np), c(np);
  HIP_TRY(hipMemcpyAsync(pp.data(), C->prod_ptr.p, sizeof(int64_t) * (C->nnzb + 1), hipMemcpyDeviceToHost, s));
  if (np) {
    HIP_TRY(hipMemcpyAsync(a.data(), C->prod_a.p, sizeof(int32_t) * np, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(b.data(), C->prod_b.p, sizeof(int32_t) * np, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
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
  *out = C->stats;
  return BSMM_OK;
}

bsmm_status bsmm_multiply(double alpha, bsmm_mat A, bsmm_mat B, double beta, bsmm_mat C_in, bsmm_mat C,
                          double filter_eps, int prec, void* stream) {
  g_err.clear();
  if (!A || !B || !C) return fail(BSMM_E_ARG, "NULL handle");
  if (!is_finite(alpha) || !is_finite(beta) || !is_finite(filter_eps))
    return fail(BSMM_E_ARG, "alpha, beta and filter_eps must be finite");
  if (prec != BSMM_FP64) return fail(BSMM_E_ARG, "unknown precision");
  if (C == A || C == B) return fail(BSMM_E_ALIAS, "output must not be an input operand");
  if (A->nbcols != B->nbrows || !same_sizes(A->col_sizes, B->row_sizes))
    return fail(BSMM_E_SHAPE, "A column block sizes differ from B row block sizes");
  if (!same_sizes(C->row_sizes, A->row_sizes) || !same_sizes(C->col_sizes, B->col_sizes))
    return fail(BSMM_E_SHAPE, "C block sizes must be A's row sizes and B's column sizes");
  const bool use_old = beta != 0.0 && C_in != nullptr;
  if (use_old && (!same_sizes(C_in->row_sizes, A->row_sizes) || !same_sizes(C_in->col_sizes, B->col_sizes)))
    return fail(BSMM_E_SHAPE, "C_in block sizes must be A's row sizes and B's column sizes");
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
  // scratch
  if (C->flags.ensure(1) != hipSuccess || C->work.ensure(1) != hipSuccess || C->totals.ensure(8) != hipSuccess ||
      C->scan_tmp.ensure(scan_tmp_elems(nbrows) + 2) != hipSuccess)
    return fail(BSMM_E_NOMEM, "scratch allocation failed");
  for (int x = 0; x < 5; ++x)
    if (C->rows[x].ensure(nbrows + 1) != hipSuccess || C->pre[x].ensure(nbrows + 1) != hipSuccess)
      return fail(BSMM_E_NOMEM, "scratch allocation failed");
  const double* normA = nullptr;
  const double* normB = nullptr;
  if (use_eps) {
    if (C->norm_a.ensure(std::max(A->nnzb, 1)) != hipSuccess) return fail(BSMM_E_NOMEM, "scratch allocation failed");
    HIP_TRY(launch_block_norms(A->cur.blk_off.p, A->cur.values.p, A->nnzb, C->norm_a.p, s));
    normA = C->norm_a.p;
    if (B == A) {
      normB = normA;
    } else {
      if (C->norm_b.ensure(std::max(B->nnzb, 1)) != hipSuccess) return fail(BSMM_E_NOMEM, "scratch allocation failed");
      HIP_TRY(launch_block_norms(B->cur.blk_off.p, B->cur.values.p, B->nnzb, C->norm_b.p, s));
      normB = C->norm_b.p;
    }
  }
  HIP_TRY(hipMemsetAsync(C->flags.p, 0, sizeof(uint32_t), s));
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
  g.c_row_sizes = C->d_row_sizes.p;
  g.c_col_sizes = C->d_col_sizes.p;
  g.row_nc = C->rows[0].p;
  g.row_np = C->rows[1].p;
  g.row_nv = C->rows[2].p;
  g.row_ncand = C->rows[3].p;
  g.row_nf = C->rows[4].p;
  g.flags = C->flags.p;
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
  HIP_TRY(hipMemcpyAsync(C->h_totals, C->totals.p, 6 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t nnzc = C->h_totals[0], nprod = C->h_totals[1], nvals = C->h_totals[2], ncand = C->h_totals[3];
  const uint32_t flags = (uint32_t)C->h_totals[4];
  const int64_t nflop_half = C->h_totals[5];
  if (flags & kFlagRowTooManyA)
    return fail(BSMM_E_UNSUPPORTED, "an A block row holds more than " + std::to_string(kMaxRowA) + " blocks");
  if (flags & kFlagRowTooManyC)
    return fail(BSMM_E_UNSUPPORTED,
                "a result block row would hold more than " + std::to_string(kMaxRowBlocks) + " blocks");
  if (nnzc > 0x7fffffffLL) return fail(BSMM_E_CAPACITY, "result has more than 2^31-1 blocks");
  if (nprod > 0x7fffffffLL) return fail(BSMM_E_CAPACITY, "more than 2^31-1 block products");

  // output storage: in place -> write the spare storage and swap afterwards
  const bool in_place = use_old && C_in == C;
  Storage& out = in_place ? C->spare : C->cur;
  if (ensure_storage(out, nbrows, nnzc, nvals) != hipSuccess || C->prod_ptr.ensure(nnzc + 1) != hipSuccess ||
      C->prod_a.ensure(std::max<int64_t>(nprod, 1)) != hipSuccess ||
      C->prod_b.ensure(std::max<int64_t>(nprod, 1)) != hipSuccess ||
      C->old_idx.ensure(std::max<int64_t>(nnzc, 1)) != hipSuccess)
    return fail(BSMM_E_NOMEM, "device allocation for the result failed");
  // a reallocation above may have freed C_in's storage only if C_in == C and
  // `out` is cur; that case is excluded by writing the spare.
  if (use_old) g.Cin = view(C_in);
  mark(C, ev, 3, s);
  HIP_TRY(launch_finish_rows(nbrows, C->pre[0].p, C->pre[1].p, C->pre[2].p, out.row_ptr.p, C->prod_ptr.p,
                             out.blk_off.p, s));
  g.c_row_ptr = out.row_ptr.p;
  g.row_pstart = C->pre[1].p;
  g.row_vstart = C->pre[2].p;
  g.c_col_idx = out.col_idx.p;
  g.c_blk_off = out.blk_off.p;
  g.prod_ptr = C->prod_ptr.p;
  g.c_old_idx = C->old_idx.p;
  g.prod_a = C->prod_a.p;
  g.prod_b = C->prod_b.p;
  HIP_TRY(launch_sym_fill(g, s));
  mark(C, ev, 4, s);

  NumArgs na{};
  na.A = g.A;
  na.B = g.B;
  na.Cin = g.Cin;
  na.use_old = g.use_old;
  na.alpha = alpha;
  na.beta = beta;
  na.nnzc = (int32_t)nnzc;
  na.c_row_sizes = C->d_row_sizes.p;
  na.c_col_sizes = C->d_col_sizes.p;
  na.c_col_idx = out.col_idx.p;
  na.c_blk_off = out.blk_off.p;
  na.prod_ptr = C->prod_ptr.p;
  na.c_old_idx = C->old_idx.p;
  na.prod_a = C->prod_a.p;
  na.prod_b = C->prod_b.p;
  na.c_values = out.values.p;
  const int uniform = (A->uniform && A->uniform == B->uniform) ? A->uniform : 0;
  HIP_TRY(launch_numeric(na, uniform, C->work.p, s));
  mark(C, ev, 5, s);
  HIP_TRY(hipMemsetAsync(out.values.p + nvals, 0, sizeof(double) * kValueSlack, s));
  mark(C, ev, 6, s);

  if (in_place) std::swap(C->cur, C->spare);
  C->nnzb = (int32_t)nnzc;
  C->nvals = nvals;
  C->nprod = nprod;
  C->has_stack = true;
  C->stats.candidates = ncand;
  C->stats.products = nprod;
  C->stats.nnzb = nnzc;
  C->stats.nvals = nvals;
  C->stats.useful_flops = 2.0 * (double)nflop_half;
  return BSMM_OK;
}

bsmm_status bsmm_filter(bsmm_mat m, double eps, void* stream) {
  g_err.clear();
  if (!m) return fail(BSMM_E_ARG, "NULL handle");
  if (!is_finite(eps)) return fail(BSMM_E_ARG, "eps must be finite");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bsmm_status st = ensure_pinned(m);
  if (st != BSMM_OK) return st;
  const int32_t nnzb = m->nnzb;
  if (m->norm_self.ensure(std::max(nnzb, 1)) != hipSuccess || m->fkeep.ensure(nnzb + 1) != hipSuccess ||
      m->fvsz.ensure(nnzb + 1) != hipSuccess || m->fpos.ensure(nnzb + 1) != hipSuccess ||
      m->fvoff.ensure(nnzb + 1) != hipSuccess || m->scan_tmp.ensure(scan_tmp_elems(nnzb) + 2) != hipSuccess ||
      ensure_storage(m->spare, m->nbrows, nnzb, m->nvals) != hipSuccess)
    return fail(BSMM_E_NOMEM, "scratch allocation failed");
  HIP_TRY(launch_block_norms(m->cur.blk_off.p, m->cur.values.p, nnzb, m->norm_self.p, s));
  HIP_TRY(launch_filter(m->cur.row_ptr.p, m->cur.col_idx.p, m->cur.blk_off.p, m->cur.values.p, m->nbrows, nnzb,
                        m->norm_self.p, eps, m->fkeep.p, m->fvsz.p, m->fpos.p, m->fvoff.p, m->scan_tmp.p,
                        m->spare.row_ptr.p, m->spare.col_idx.p, m->spare.blk_off.p, m->spare.values.p, s));
  HIP_TRY(hipMemcpyAsync(m->h_totals, m->fpos.p + nnzb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(m->h_totals + 1, m->fvoff.p + nnzb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t new_nnzb = m->h_totals[0], new_nvals = m->h_totals[1];
  HIP_TRY(hipMemsetAsync(m->spare.values.p + new_nvals, 0, sizeof(double) * kValueSlack, s));
  std::swap(m->cur, m->spare);
  m->nnzb = (int32_t)new_nnzb;
  m->nvals = new_nvals;
  m->has_stack = false;  // block indices changed
  return BSMM_OK;
}

}  // extern "C"
