// Symbolic phase of the block-sparse multiply: result pattern and product
// stack, with the on-the-fly norm filter applied to every candidate product.
//
// Section 2 of the paper: the local multiply loops over A block rows and, for
// each, over the B blocks reached through A's columns; a block product is kept
// only if the product of the two block norms exceeds the threshold.  Here one
// workgroup owns one C block row i.  The candidates (A(i,k), B(k,j)) of the
// row are enumerated as a flat index over the concatenated B rows, so all 256
// lanes stay busy even when B rows are short.  Kept candidates are merged by
// block column in an LDS open-addressing hash, which gives the row's distinct
// columns and per-column product counts; ranking the columns gives the sorted
// pattern, and a scan of the counts gives each C block's slice of the stack.
//
// Two passes share the enumeration: the count pass sizes the outputs, the fill
// pass writes them.  Both take exactly the same keep/drop decisions.
#include "block_scan.h"
#include "bsmm_internal.h"

namespace bsmm {

constexpr int kHashBits = 11;
constexpr int kHugeHashBits = 12;  // huge forms: 4096 slots, at most half full
static_assert((1 << kHashBits) == kHashSlots, "hash size");
static_assert(kLargeRowA % kSymThreads == 0 && kMaxRowA % kSymThreads == 0, "A chunking");
static_assert(kLargeRowBlocks % kSymThreads == 0 && kMaxRowBlocks % kSymThreads == 0, "row chunking");
static_assert(2 * kLargeRowBlocks <= kHashSlots && 2 * kMaxRowBlocks <= (1 << kHugeHashBits), "hash load");

// Size of C's block column j (a kernel argument when every column has it:
// no gather per candidate).
__device__ __forceinline__ int32_t col_size(const SymArgs& g, int32_t j) {
  return g.c_col_uniform ? g.c_col_uniform : g.c_col_sizes[j];
}

// Rows of the current fill panel, and the stack position its index 0 holds.
__device__ __forceinline__ bool in_panel(const SymArgs& g, int32_t i) {
  return !g.panel || (i >= g.panel[0] && i < g.panel[1]);
}
__device__ __forceinline__ int64_t panel_base(const SymArgs& g) { return g.panel ? g.row_pstart[g.panel[0]] : 0; }

template <int HB>
__device__ __forceinline__ uint32_t hash_of(int32_t j) { return ((uint32_t)j * 2654435761u) >> (32 - HB); }

// Insert block column j into a table of 2^HB slots; returns its slot (or -1
// if the table is full).
template <int HB>
__device__ __forceinline__ int hash_insert(int32_t* hkey, int32_t j, bool* fresh) {
  constexpr int kSlots = 1 << HB;
  uint32_t h = hash_of<HB>(j);
  for (int probe = 0; probe < kSlots; ++probe) {
    const int32_t prev = atomicCAS(&hkey[h], -1, j);
    if (prev == -1) {
      *fresh = true;
      return (int)h;
    }
    if (prev == j) {
      *fresh = false;
      return (int)h;
    }
    h = (h + 1) & (kSlots - 1);
  }
  *fresh = false;
  return -1;
}

template <int HB>
__device__ __forceinline__ int hash_find(const int32_t* hkey, int32_t j) {
  constexpr int kSlots = 1 << HB;
  uint32_t h = hash_of<HB>(j);
  for (int probe = 0; probe < kSlots; ++probe) {
    const int32_t k = hkey[h];
    if (k == j) return (int)h;
    if (k == -1) return -1;
    h = (h + 1) & (kSlots - 1);
  }
  return -1;
}


// Row state in LDS common to both passes.
template <int RA>
struct RowA {
  int32_t qs[RA];        // first B block of B row k_p
  int32_t ks[RA];        // inner block size of k_p
  int32_t pre[RA + 1];   // exclusive prefix of the enumerated candidates per entry
  double nrm[RA];        // norm of A(i, k_p)
  int8_t srt[RA];        // B row k_p enumerated in norm order (its kept prefix only)
};

// Kept prefix of A entry e (norm a) on B row k (sorted, n blocks from q0):
// the number of its entries whose product with a passes the filter.
__device__ __forceinline__ int32_t kept_prefix(const SymArgs& g, double a, int32_t q0, int32_t n) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (a * g.bnrm[q0 + mid] > g.eps) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Load the A entries of row i and the candidate prefix.  Returns the number of
// candidates the passes enumerate (every product of an entry on an unsorted B
// row, only the kept prefix on a sorted one), or -1 if the row is outside the
// supported limits; *full_out receives the candidates before the filter.
template <int RA>
__device__ int32_t load_row(const SymArgs& g, int32_t i, RowA<RA>& ra, int32_t* a0_out, int32_t* na_out,
                            int64_t* full_out) {
  const int tid = threadIdx.x;
  const int32_t a0 = g.A.row_ptr[i];
  const int32_t nA = g.A.row_ptr[i + 1] - a0;
  *a0_out = a0;
  *na_out = nA;
  if (nA > RA) return -1;
  constexpr int kPer = RA / kSymThreads;
  int32_t len[kPer];
  int64_t mysum = 0, myfull = 0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int32_t p = tid * kPer + u;
    len[u] = 0;
    if (p < nA) {
      const int32_t k = g.A.col_idx[a0 + p];
      const int32_t qs = g.B.row_ptr[k];
      const int32_t n = g.B.row_ptr[k + 1] - qs;
      const double a = g.use_eps ? g.normA[a0 + p] : 0.0;
      const bool srt = g.sorted_mode && g.bsorted[k];
      len[u] = srt ? kept_prefix(g, a, qs, n) : n;
      if (srt) g.akeep[a0 + p] = len[u];
      myfull += n;
      ra.qs[p] = qs;
      ra.ks[p] = g.A.col_sizes[k];
      ra.nrm[p] = a;
      ra.srt[p] = srt ? 1 : 0;
    }
    mysum += len[u];
  }
  int64_t total, full;
  int64_t run = block_exclusive_scan<kSymThreads>(mysum, &total);
  if (g.sorted_mode) (void)block_exclusive_scan<kSymThreads>(myfull, &full);  // uniform
  else full = total;  // every candidate enumerated
  *full_out = full;
  if (total > 0x7fffffffLL) return -1;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int32_t p = tid * kPer + u;
    if (p < nA) ra.pre[p] = (int32_t)run;
    run += len[u];
  }
  if (tid == 0) ra.pre[nA] = (int32_t)total;
  __syncthreads();
  return (int32_t)total;
}

// Candidate t of the row -> (A entry p, B block q), p the last entry with
// pre[p] <= t, found from *hint (an entry with pre[*hint] <= t: each thread
// meets its candidates in increasing order) by trying the next two entries
// before a binary search; *hint becomes p.
template <int RA>
__device__ __forceinline__ void candidate(const RowA<RA>& ra, int32_t nA, int32_t t, int32_t* hint, int32_t* p_out,
                                          int32_t* q_out) {
  int lo = *hint;
  if (lo + 1 < nA && ra.pre[lo + 1] <= t) {
    ++lo;
    if (lo + 1 < nA && ra.pre[lo + 1] <= t) {
      int hi = nA - 1;
      ++lo;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ra.pre[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
    }
  }
  *hint = lo;
  *p_out = lo;
  *q_out = ra.qs[lo] + (t - ra.pre[lo]);
}

// B block of the r-th enumerated candidate of an entry whose B row starts at
// q0: the r-th block in norm order on a sorted row, else the r-th stored.
__device__ __forceinline__ int32_t cand_block(const SymArgs& g, bool srt, int32_t q0, int32_t r) {
  return srt ? g.bord[q0 + r] : q0 + r;
}

template <int RA>
__device__ __forceinline__ bool keep_product(const SymArgs& g, const RowA<RA>& ra, int32_t p, int32_t q) {
  if (!g.use_eps) return true;
  const double prod = ra.nrm[p] * g.normB[q];
  return prod > g.eps;
}

// ------------------------------------------------------------------ count

// Candidates a thread takes at a time in the row passes: their index and
// norm loads are issued together, so a workgroup keeps several gathers in
// flight per thread (rows of thousands of candidates are latency-bound).
constexpr int kCandBatch = 4;

// Candidates [lo, hi) of a row pass, one contiguous segment per wave: lanes
// take consecutive candidates (coalesced loads) and a lane's next candidate is
// 64 further on, usually in the same or the next A entry, so the entry lookup
// from the previous one rarely needs its binary search.
constexpr int kSymWaves = kSymThreads / 64;
__device__ __forceinline__ void wave_segment(int32_t lo, int32_t hi, int32_t* s0, int32_t* s1) {
  const int32_t seg = ((hi - lo + kSymWaves * 64 - 1) / (kSymWaves * 64)) * 64;
  const int32_t w = (int32_t)(threadIdx.x >> 6);
  *s0 = min(hi, lo + w * seg);
  *s1 = min(hi, *s0 + seg);
}

// LDS of one workgroup of the count pass.  The hash always has the form's
// full size (the row's distinct columns are what the pass counts); the A
// entries of the row take RA slots.
template <int RA, int HB>
struct CountShared {
  int32_t hkey[1 << HB];
  RowA<RA> ra;
  int32_t s_nc;
  unsigned long long s_sumn;
  unsigned long long s_np;
  unsigned long long s_nf;
  int s_bad;
};

// Count C block row i (one workgroup).  A row beyond the form's limits (more
// than RA A blocks, more than RC distinct columns) is listed for the huge
// form when DEFER is set (nothing else is written), else flagged.
template <int RA, int HB, int RC, bool DEFER>
__device__ void count_row(const SymArgs& g, int32_t i, CountShared<RA, HB>& sh) {
  int32_t* const hkey = sh.hkey;
  RowA<RA>& ra = sh.ra;
  int32_t& s_nc = sh.s_nc;
  unsigned long long& s_sumn = sh.s_sumn;
  unsigned long long& s_np = sh.s_np;
  unsigned long long& s_nf = sh.s_nf;
  int& s_bad = sh.s_bad;
  const int tid = threadIdx.x;
  {
    for (int h = tid; h < (1 << HB); h += kSymThreads) hkey[h] = -1;
    if (tid == 0) {
      s_nc = 0;
      s_sumn = 0;
      s_np = 0;
      s_nf = 0;
      s_bad = 0;
    }
    __syncthreads();
    int32_t a0, nA;
    int64_t full;
    const int32_t T = load_row(g, i, ra, &a0, &nA, &full);
    if (T < 0) {
      if (DEFER) {
        if (tid == 0) g.huge[atomicAdd(g.n_huge, 1)] = i;
      } else if (tid == 0) {
        atomicOr(g.flags, kFlagRowTooManyA);
        g.row_nc[i] = 0;
        g.row_np[i] = 0;
        g.row_nv[i] = 0;
        g.row_ncand[i] = 0;
        g.row_nf[i] = 0;
      }
      __syncthreads();
      return;
    }
    uint32_t np = 0;
    uint64_t nf = 0;
    int32_t hint = 0;  // A entry of this thread's last candidate
    int32_t s0, s1;
    wave_segment(0, T, &s0, &s1);
    // kCandBatch candidates per thread at a time, their global loads issued together
    for (int32_t tb = s0 + (tid & 63); tb < s1; tb += kCandBatch * 64) {
      int32_t pp[kCandBatch], jj[kCandBatch];
      bool kk[kCandBatch];
#pragma unroll
      for (int u = 0; u < kCandBatch; ++u) {
        const int32_t t = tb + u * 64;
        int32_t p = 0, q = 0;
        bool srt = false;
        if (t < s1) {
          candidate(ra, nA, t, &hint, &p, &q);
          srt = ra.srt[p] != 0;
          if (srt) q = g.bord[q];  // a kept candidate by construction
        }
        pp[u] = p;
        kk[u] = t < s1 && (srt || keep_product(g, ra, p, q));
        jj[u] = t < s1 ? g.B.col_idx[q] : 0;
      }
#pragma unroll
      for (int u = 0; u < kCandBatch; ++u) {
        if (!kk[u]) continue;
        ++np;
        const int32_t j = jj[u];
        nf += (uint64_t)col_size(g, j) * (uint64_t)ra.ks[pp[u]];
        bool fresh;
        const int h = hash_insert<HB>(hkey, j, &fresh);
        if (h < 0) {
          s_bad = 1;
        } else if (fresh) {
          atomicAdd(&s_nc, 1);
          atomicAdd(&s_sumn, (unsigned long long)col_size(g, j));
        }
      }
    }
    if (g.use_old) {
      const int32_t o1 = g.Cin.row_ptr[i + 1];
      for (int32_t q = g.Cin.row_ptr[i] + tid; q < o1; q += kSymThreads) {
        const int32_t j = g.Cin.col_idx[q];
        bool fresh;
        const int h = hash_insert<HB>(hkey, j, &fresh);
        if (h < 0) {
          s_bad = 1;
        } else if (fresh) {
          atomicAdd(&s_nc, 1);
          atomicAdd(&s_sumn, (unsigned long long)col_size(g, j));
        }
      }
    }
    if (np) {
      atomicAdd(&s_np, (unsigned long long)np);
      atomicAdd(&s_nf, (unsigned long long)nf);
    }
    __syncthreads();
    if (tid == 0) {
      const bool bad = s_bad || s_nc > RC;
      if (bad && DEFER) {
        g.huge[atomicAdd(g.n_huge, 1)] = i;
      } else {
        if (bad) atomicOr(g.flags, kFlagRowTooManyC);
        g.row_nc[i] = bad ? 0 : s_nc;
        g.row_np[i] = bad ? 0 : (int64_t)s_np;
        g.row_nv[i] = bad ? 0 : (int64_t)g.c_row_sizes[i] * (int64_t)s_sumn;
        g.row_ncand[i] = full;
        g.row_nf[i] = bad ? 0 : (int64_t)g.c_row_sizes[i] * (int64_t)s_nf;
        // the fill forms beyond the tiny one this row needs (few rows do)
        if (DEFER && !bad && (nA > kTinyRowA || s_nc > kTinyRowC))
          atomicOr(g.forms, (nA <= kSmallRowA && s_nc <= kSmallRowC) ? kFormSmall : kFormLarge);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ thin rows
// Rows with at most kThinA stored A blocks, kThinT candidates and kThinO C_in
// blocks (block-diagonal and nearly block-diagonal matrices: millions of rows
// of one candidate each) are counted and filled by one thread each, with the
// same results as the workgroup forms: columns ascending, a C block's products
// in ascending A entry order.  The count pass lists every other row in
// g.wide; the workgroup forms walk only that list.
constexpr int kThinA = 4, kThinT = 8, kThinO = 8, kThinC = kThinT + kThinO;

struct ThinRow {
  int32_t a0, T, n, nc, o0, no;
  int32_t cj[kThinT], cq[kThinT], cp[kThinT];  // kept candidates in order: column, B block, A entry
  int32_t col[kThinC];                         // distinct columns, ascending
  int32_t oj[kThinO];                          // C_in columns of the row
  uint64_t nf;                                 // sum over kept candidates of n_j * k_p
};

// Element x of a register array by a run-time index (unrolled selects).
template <int N, class T>
__device__ __forceinline__ T thin_sel(const T (&a)[N], int x) {
  T v = a[0];
#pragma unroll
  for (int y = 1; y < N; ++y) v = (x == y) ? a[y] : v;
  return v;
}

// Add v to the ascending distinct list col[0..nc).
__device__ __forceinline__ void thin_insert(ThinRow& r, int32_t v) {
  bool dup = false;
#pragma unroll
  for (int x = 0; x < kThinC; ++x) dup = dup || (x < r.nc && r.col[x] == v);
  if (dup) return;
#pragma unroll
  for (int x = 0; x < kThinC; ++x) {
    if (x < r.nc && r.col[x] > v) {
      const int32_t t = r.col[x];
      r.col[x] = v;
      v = t;
    }
  }
#pragma unroll
  for (int x = 0; x < kThinC; ++x)
    if (x == r.nc) r.col[x] = v;
  ++r.nc;
}

// Load row i if it is thin; false (and nothing else done) if it is not.
__device__ bool thin_load(const SymArgs& g, int32_t i, ThinRow& r) {
  r.a0 = g.A.row_ptr[i];
  const int32_t nA = g.A.row_ptr[i + 1] - r.a0;
  if (nA > kThinA) return false;
  int32_t qs[kThinA], pre[kThinA + 1], ks[kThinA];
  double nrm[kThinA];
  pre[0] = 0;
#pragma unroll
  for (int p = 0; p < kThinA; ++p) {
    qs[p] = 0;
    ks[p] = 0;
    nrm[p] = 0.0;
    int32_t len = 0;
    if (p < nA) {
      const int32_t k = g.A.col_idx[r.a0 + p];
      qs[p] = g.B.row_ptr[k];
      len = g.B.row_ptr[k + 1] - qs[p];
      ks[p] = g.A.col_sizes[k];
      nrm[p] = g.use_eps ? g.normA[r.a0 + p] : 0.0;
    }
    pre[p + 1] = pre[p] + len;
  }
  r.T = pre[kThinA];
  if (r.T > kThinT) return false;
  r.o0 = 0;
  r.no = 0;
  if (g.use_old) {
    r.o0 = g.Cin.row_ptr[i];
    r.no = g.Cin.row_ptr[i + 1] - r.o0;
    if (r.no > kThinO) return false;
  }
  r.n = 0;
  r.nc = 0;
  r.nf = 0;
#pragma unroll
  for (int t = 0; t < kThinT; ++t) {
    if (t < r.T) {
      int p = 0;
#pragma unroll
      for (int x = 1; x < kThinA; ++x) p += (pre[x] <= t) ? 1 : 0;  // pre is non-decreasing
      const int32_t q = thin_sel(qs, p) + (t - thin_sel(pre, p));
      const bool keep = !g.use_eps || thin_sel(nrm, p) * g.normB[q] > g.eps;
      if (keep) {
        const int32_t j = g.B.col_idx[q];
#pragma unroll
        for (int x = 0; x < kThinT; ++x) {
          if (x == r.n) {
            r.cj[x] = j;
            r.cq[x] = q;
            r.cp[x] = p;
          }
        }
        ++r.n;
        r.nf += (uint64_t)col_size(g, j) * (uint64_t)thin_sel(ks, p);
      }
    }
  }
#pragma unroll
  for (int x = 0; x < kThinT; ++x)
    if (x < r.n) thin_insert(r, r.cj[x]);
#pragma unroll
  for (int x = 0; x < kThinO; ++x) {
    r.oj[x] = -1;
    if (x < r.no) {
      r.oj[x] = g.Cin.col_idx[r.o0 + x];
      thin_insert(r, r.oj[x]);
    }
  }
  return true;
}

// Count pass of the thin rows; every other row goes to the list g.wide.
__global__ __launch_bounds__(256) void k_sym_count_thin(SymArgs g) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= g.A.nbrows) return;
  ThinRow r;
  if (!thin_load(g, i, r)) {
    g.wide[atomicAdd(g.n_wide, 1)] = i;
    return;
  }
  int64_t sumn = 0;
#pragma unroll
  for (int x = 0; x < kThinC; ++x)
    if (x < r.nc) sumn += col_size(g, r.col[x]);
  const int64_t m = g.c_row_sizes[i];
  g.row_nc[i] = r.nc;
  g.row_np[i] = r.n;
  g.row_nv[i] = m * sumn;
  g.row_ncand[i] = r.T;
  g.row_nf[i] = m * (int64_t)r.nf;
}

// Fill pass of the thin rows.  With panels it also closes the panel's
// product offsets: the entry of the first C block after the panel gets the
// start of the next row's products (the value that row's fill writes later),
// which the numeric kernels read as the panel's end.
__global__ __launch_bounds__(256) void k_sym_fill_thin(SymArgs g) {
  if (g.totals[kTotAbort]) return;
  if (g.panel && blockIdx.x == 0 && threadIdx.x == 0)
    g.prod_ptr[g.c_row_ptr[g.panel[1]]] = g.row_pstart[g.panel[1]];
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= g.A.nbrows) return;
  if (!in_panel(g, i)) return;
  ThinRow r;
  if (!thin_load(g, i, r)) return;
  const int32_t crow = g.c_row_ptr[i];
  const int64_t prow = g.row_pstart[i], vrow = g.row_vstart[i];
  const int64_t srow = prow - panel_base(g);  // stack position of the row's first product
  const int64_t m = g.c_row_sizes[i];
  int64_t pc = 0, vc = 0;
#pragma unroll
  for (int x = 0; x < kThinC; ++x) {
    if (x < r.nc) {
      const int32_t j = r.col[x];
      int32_t o = -1;
#pragma unroll
      for (int y = 0; y < kThinO; ++y)
        if (y < r.no && r.oj[y] == j) o = r.o0 + y;
      g.c_col_idx[crow + x] = j;
      g.c_old_idx[crow + x] = o;
      g.prod_ptr[crow + x] = prow + pc;
      g.c_blk_off[crow + x] = vrow + m * vc;
#pragma unroll
      for (int y = 0; y < kThinT; ++y) {
        if (y < r.n && r.cj[y] == j) {
          g.prod[srow + pc] = make_int2(r.a0 + r.cp[y], r.cq[y]);
          ++pc;
        }
      }
      vc += col_size(g, j);
    }
  }
}

constexpr int kCountSmallRowA = 256;

// Small form (13 KB of LDS, eight workgroups per CU): the listed (not thin)
// rows of at most 256 A blocks, one workgroup per row.
__global__ __launch_bounds__(kSymThreads) void k_sym_count_small(SymArgs g) {
  __shared__ CountShared<kCountSmallRowA, kHashBits> sh;
  const int32_t nw = *g.n_wide;
  for (int32_t x = blockIdx.x; x < nw; x += gridDim.x) {
    const int32_t i = g.wide[x];
    if (g.A.row_ptr[i + 1] - g.A.row_ptr[i] > kCountSmallRowA) continue;  // uniform
    count_row<kCountSmallRowA, kHashBits, kLargeRowBlocks, true>(g, i, sh);
  }
}

// Large form: the longer rows (and rows beyond the limits, which it reports).
// Workgroup w of G owns list entries w, w+G, w+2G, ...; it looks at 256 of
// them at a time, one per thread, and counts the long rows in turn, so long
// rows spread over the whole grid while short ones cost one load each.
__global__ __launch_bounds__(kSymThreads) void k_sym_count_large(SymArgs g) {
  __shared__ CountShared<kLargeRowA, kHashBits> sh;
  __shared__ int32_t rows[kSymThreads];
  __shared__ int32_t nrows;
  const int tid = threadIdx.x;
  const int64_t G = gridDim.x;
  const int32_t nw = *g.n_wide;
  for (int64_t x0 = blockIdx.x; x0 < nw; x0 += G * kSymThreads) {
    if (tid == 0) nrows = 0;
    __syncthreads();
    const int64_t x = x0 + G * tid;
    const int32_t i = x < nw ? g.wide[x] : 0;
    if (x < nw && g.A.row_ptr[i + 1] - g.A.row_ptr[i] > kCountSmallRowA)
      rows[atomicAdd(&nrows, 1)] = i;
    __syncthreads();
    const int32_t n = nrows;
    for (int32_t x = 0; x < n; ++x) count_row<kLargeRowA, kHashBits, kLargeRowBlocks, true>(g, rows[x], sh);
  }
}

// Huge form (56 KB of LDS): the rows the other forms listed in g.huge (more
// than kLargeRowA A blocks or kLargeRowBlocks result blocks), one workgroup
// per row; rows beyond kMaxRowA / kMaxRowBlocks are flagged.
__global__ __launch_bounds__(kSymThreads) void k_sym_count_huge(SymArgs g) {
  __shared__ CountShared<kMaxRowA, kHugeHashBits> sh;
  const int32_t nh = *g.n_huge;
  for (int32_t x = blockIdx.x; x < nh; x += gridDim.x)
    count_row<kMaxRowA, kHugeHashBits, kMaxRowBlocks, false>(g, g.huge[x], sh);
}

// ------------------------------------------------------------------ fill

// Row state of the fill pass (the count pass also needs the inner sizes).
template <int RA>
struct RowFill {
  int32_t qs[RA];        // first B block of B row k_p
  int32_t pre[RA + 1];   // exclusive prefix of the enumerated candidates per entry
  double nrm[RA];        // norm of A(i, k_p)
  int8_t srt[RA];        // B row k_p enumerated in norm order (its kept prefix only)
};

// Capacities of one form of the fill pass: 2^HB hash slots, at most RA
// stored A blocks and RB result blocks per row, and the row's candidates
// cached in chunks of CC (each holds the hash slot of its block column, or -1
// when the filter drops it).  The fill runs in two forms: a small one (34 KB
// of LDS, four workgroups per CU) for the rows that fit it, and a large one
// (78 KB, two per CU) for the rest; rows do not interact, so each form takes
// its own rows.
template <int HB, int RA, int RB, int CC>
struct FillCaps {
  static constexpr int kBits = HB, kSlots = 1 << HB, kRowA = RA, kRowC = RB, kCand = CC;
  static_assert(kSlots <= 32767, "slots must fit in int16");
  static_assert((RA % kSymThreads == 0 || RA < kSymThreads) && RB % kSymThreads == 0, "row chunking");
  static_assert(2 * RB <= kSlots, "hash load at most one half");
};
using FillTiny = FillCaps<9, kTinyRowA, kTinyRowC, 4096>;
using FillSmall = FillCaps<10, kSmallRowA, kSmallRowC, 4096>;
struct FillNone {  // no form: no row fits
  static constexpr int kRowA = -1, kRowC = -1;
};
using FillLarge = FillCaps<kHashBits, kLargeRowA, kLargeRowBlocks, 8192>;
using FillHuge = FillCaps<kHugeHashBits, kMaxRowA, kMaxRowBlocks, 8192>;

template <int RA>
__device__ int32_t load_row_fill(const SymArgs& g, int32_t i, RowFill<RA>& ra, int32_t* a0_out, int32_t* na_out) {
  const int tid = threadIdx.x;
  const int32_t a0 = g.A.row_ptr[i];
  const int32_t nA = g.A.row_ptr[i + 1] - a0;
  *a0_out = a0;
  *na_out = nA;
  if (nA > RA) return -1;
  constexpr int kPer = RA >= kSymThreads ? RA / kSymThreads : 1;
  int32_t len[kPer];
  int64_t mysum = 0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int32_t p = tid * kPer + u;
    len[u] = 0;
    if (p < nA) {  // nA <= RA
      const int32_t k = g.A.col_idx[a0 + p];
      const int32_t qs = g.B.row_ptr[k];
      const bool srt = g.sorted_mode && g.bsorted[k];
      // the count pass left a sorted entry's kept prefix in akeep
      len[u] = srt ? g.akeep[a0 + p] : g.B.row_ptr[k + 1] - qs;
      ra.qs[p] = qs;
      ra.nrm[p] = g.use_eps ? g.normA[a0 + p] : 0.0;
      ra.srt[p] = srt ? 1 : 0;
    }
    mysum += len[u];
  }
  int64_t total;
  int64_t run = block_exclusive_scan<kSymThreads>(mysum, &total);
  if (total > 0x7fffffffLL) return -1;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int32_t p = tid * kPer + u;
    if (p < nA) ra.pre[p] = (int32_t)run;
    run += len[u];
  }
  if (tid == 0) ra.pre[nA] = (int32_t)total;
  __syncthreads();
  return (int32_t)total;
}

// The A entry of candidate t: the last entry p in [lo, hi] with pre[p] <= t.
template <int RA>
__device__ __forceinline__ int32_t fill_entry_in(const RowFill<RA>& ra, int32_t lo, int32_t hi, int32_t t) {
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ra.pre[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int RA>
__device__ __forceinline__ int32_t fill_entry_of(const RowFill<RA>& ra, int32_t nA, int32_t t) {
  return fill_entry_in(ra, 0, nA - 1, t);
}

// The same from an entry `hint` with pre[hint] <= t (each thread meets its
// candidates in increasing order): the next two entries are tried before a
// binary search over the rest, so long B rows cost one LDS read per
// candidate instead of a search.
template <int RA>
__device__ __forceinline__ int32_t fill_entry_from(const RowFill<RA>& ra, int32_t nA, int32_t hint, int32_t t) {
  if (hint + 1 >= nA || ra.pre[hint + 1] > t) return hint;
  if (hint + 2 >= nA || ra.pre[hint + 2] > t) return hint + 1;
  return fill_entry_in(ra, hint + 2, nA - 1, t);
}

template <int RA>
__device__ __forceinline__ bool fill_keep(const SymArgs& g, const RowFill<RA>& ra, int32_t p, int32_t q) {
  if (!g.use_eps) return true;
  const double prod = ra.nrm[p] * g.normB[q];
  return prod > g.eps;
}

// LDS of one workgroup of the fill pass.
template <class Cap>
struct FillShared {
  int32_t hkey[Cap::kSlots];
  int32_t hcnt[Cap::kSlots];  // product count per slot, then the slot's rank
  int32_t hold[Cap::kSlots];
  RowFill<Cap::kRowA> ra;
  int32_t ekey[Cap::kRowC];
  int32_t eslot[Cap::kRowC];
  int32_t spre[Cap::kRowC];
  int32_t cursor[Cap::kRowC];
  int32_t svs[Cap::kRowC];
  int16_t cslot[Cap::kCand];
  int32_t s_ne;
};

// Fill C block row i (one workgroup).  After the hash has merged the kept
// candidates by column, the columns are ranked (sorted pattern), the counts
// scanned (each C block's slice of the stack), and the products placed in
// ascending A entry order, i.e. ascending k (the candidates of one A entry
// have distinct columns, so within a C block the entries order its products).
template <class Cap>
__device__ void fill_row(const SymArgs& g, int32_t i, FillShared<Cap>& sh) {
  int32_t* const hkey = sh.hkey;
  int32_t* const hcnt = sh.hcnt;
  int32_t* const hold = sh.hold;
  RowFill<Cap::kRowA>& ra = sh.ra;
  int32_t* const ekey = sh.ekey;
  int32_t* const eslot = sh.eslot;
  int32_t* const spre = sh.spre;
  int32_t* const cursor = sh.cursor;
  int32_t* const svs = sh.svs;
  int16_t* const cslot = sh.cslot;
  constexpr int kHashBitsF = Cap::kBits;
  constexpr int kHashSlotsF = Cap::kSlots;
  constexpr int kMaxRowBlocksF = Cap::kRowC;
  constexpr int kCandCacheF = Cap::kCand;
  const int tid = threadIdx.x;
  constexpr int kPer = kMaxRowBlocksF / kSymThreads;
  {
    for (int h = tid; h < kHashSlotsF; h += kSymThreads) {
      hkey[h] = -1;
      hcnt[h] = 0;
      hold[h] = -1;
    }
    if (tid == 0) sh.s_ne = 0;
    __syncthreads();
    int32_t a0, nA;
    const int32_t T = load_row_fill(g, i, ra, &a0, &nA);
    if (T < 0) return;  // uniform over the workgroup; reported by the count pass
    const bool one_chunk = T <= kCandCacheF;
    int32_t hint = 0;  // A entry of this thread's last candidate
    int32_t s0, s1;
    wave_segment(0, T, &s0, &s1);
    for (int32_t tb = s0 + (tid & 63); tb < s1; tb += kCandBatch * 64) {
      int32_t jj[kCandBatch];
      bool kk[kCandBatch];
#pragma unroll
      for (int u = 0; u < kCandBatch; ++u) {
        const int32_t t = tb + u * 64;
        const int32_t p = t < s1 ? (hint = fill_entry_from(ra, nA, hint, t)) : 0;
        const bool srt = ra.srt[p] != 0;
        const int32_t q = t < s1 ? cand_block(g, srt, ra.qs[p], t - ra.pre[p]) : 0;
        kk[u] = t < s1 && (srt || fill_keep(g, ra, p, q));
        jj[u] = t < s1 ? g.B.col_idx[q] : 0;
      }
#pragma unroll
      for (int u = 0; u < kCandBatch; ++u) {
        const int32_t t = tb + u * 64;
        int h = -1;
        if (kk[u]) {
          bool fresh;
          h = hash_insert<kHashBitsF>(hkey, jj[u], &fresh);
          if (h >= 0) atomicAdd(&hcnt[h], 1);
        }
        if (one_chunk && t < s1) cslot[t] = (int16_t)h;
      }
    }
    if (g.use_old) {
      const int32_t o1 = g.Cin.row_ptr[i + 1];
      for (int32_t q = g.Cin.row_ptr[i] + tid; q < o1; q += kSymThreads) {
        bool fresh;
        const int h = hash_insert<kHashBitsF>(hkey, g.Cin.col_idx[q], &fresh);
        if (h >= 0) hold[h] = q;
      }
    }
    __syncthreads();
    for (int h = tid; h < kHashSlotsF; h += kSymThreads) {
      if (hkey[h] >= 0) {
        const int e = atomicAdd(&sh.s_ne, 1);
        if (e < kMaxRowBlocksF) {
          ekey[e] = hkey[h];
          eslot[e] = h;
        }
      }
    }
    __syncthreads();
    const int32_t nC = sh.s_ne;
    if (nC > kMaxRowBlocksF) return;  // reported by the count pass
    // Rank the distinct columns (rank = number of smaller columns), move the
    // counts into rank order and leave each slot's rank in hcnt.
    const int32_t crow = g.c_row_ptr[i];
    for (int e = tid; e < nC; e += kSymThreads) {
      const int32_t key = ekey[e];
      int r = 0;
      for (int e2 = 0; e2 < nC; ++e2) r += (ekey[e2] < key) ? 1 : 0;
      const int h = eslot[e];
      spre[r] = hcnt[h];
      hcnt[h] = r;
      svs[r] = col_size(g, key);
      g.c_col_idx[crow + r] = key;
      g.c_old_idx[crow + r] = hold[h];
    }
    __syncthreads();
    // Scan the per-column product counts and value sizes in rank order.
    {
      int32_t cnt[kPer];
      int32_t vs[kPer];
      int64_t sc = 0, sv = 0;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int r = tid * kPer + u;
        cnt[u] = r < nC ? spre[r] : 0;
        vs[u] = r < nC ? svs[r] : 0;
        sc += cnt[u];
        sv += vs[u];
      }
      int64_t tc, tv;
      int64_t rc = block_exclusive_scan<kSymThreads>(sc, &tc);
      int64_t rv = block_exclusive_scan<kSymThreads>(sv, &tv);
      const int64_t prow = g.row_pstart[i];
      const int64_t vrow = g.row_vstart[i];
      const int64_t m = g.c_row_sizes[i];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int r = tid * kPer + u;
        if (r < nC) {
          spre[r] = (int32_t)rc;
          cursor[r] = 0;
          g.prod_ptr[crow + r] = prow + rc;
          g.c_blk_off[crow + r] = vrow + m * rv;
        }
        rc += cnt[u];
        rv += vs[u];
      }
    }
    // svs is free after the scan: it holds the round masks of the placement
    uint32_t* const rmask = reinterpret_cast<uint32_t*>(svs);
    for (int r = tid; r < nC; r += kSymThreads) rmask[r] = 0;
    __syncthreads();
    const int64_t prow = g.row_pstart[i] - panel_base(g);  // stack position of the row's first product
    int32_t chint = 0;  // A entry of this thread's last candidate in the chunk passes
    for (int32_t t0 = 0; t0 < T; t0 += kCandCacheF) {
      const int32_t t1 = T - t0 > kCandCacheF ? t0 + kCandCacheF : T;
      if (!one_chunk) {
        int32_t c0, c1;
        wave_segment(t0, t1, &c0, &c1);
        for (int32_t tb = c0 + (tid & 63); tb < c1; tb += kCandBatch * 64) {
          int32_t jj[kCandBatch];
          bool kk[kCandBatch];
#pragma unroll
          for (int u = 0; u < kCandBatch; ++u) {
            const int32_t t = tb + u * 64;
            const int32_t p = t < c1 ? (chint = fill_entry_from(ra, nA, chint, t)) : 0;
            const bool srt = ra.srt[p] != 0;
            const int32_t q = t < c1 ? cand_block(g, srt, ra.qs[p], t - ra.pre[p]) : 0;
            kk[u] = t < c1 && (srt || fill_keep(g, ra, p, q));
            jj[u] = t < c1 ? g.B.col_idx[q] : 0;
          }
#pragma unroll
          for (int u = 0; u < kCandBatch; ++u) {
            const int32_t t = tb + u * 64;
            if (t < c1) cslot[t - t0] = (int16_t)(kk[u] ? hash_find<kHashBitsF>(hkey, jj[u]) : -1);
          }
        }
        __syncthreads();
      }
      // Place the chunk's kept candidates in rounds of 32 A entries: mark
      // which entries of the round reach each C block (one bit per entry),
      // then a candidate's place is its block's cursor plus the number of
      // earlier entries of the round that reach the same block, and the
      // cursors advance by the round's counts.  A round needs three barriers
      // however many entries it holds.
      const int32_t pl = fill_entry_of(ra, nA, t1 - 1);
      for (int32_t r0 = fill_entry_of(ra, nA, t0); r0 <= pl; r0 += 32) {
        const int32_t r1 = r0 + 32 <= pl + 1 ? r0 + 32 : pl + 1;
        const int32_t tb = ra.pre[r0] > t0 ? ra.pre[r0] : t0;
        const int32_t te = ra.pre[r1] < t1 ? ra.pre[r1] : t1;
        int32_t w0, w1;
        wave_segment(tb, te, &w0, &w1);
        int32_t rh = r0;  // pre[r0] <= tb: a valid hint for every candidate of the round
        for (int32_t t = w0 + (tid & 63); t < w1; t += 64) {
          const int h = cslot[t - t0];
          rh = fill_entry_from(ra, nA, rh, t);
          if (h >= 0) atomicOr(&rmask[hcnt[h]], 1u << (rh - r0));
        }
        __syncthreads();
        rh = r0;
        for (int32_t t = w0 + (tid & 63); t < w1; t += 64) {
          const int h = cslot[t - t0];
          rh = fill_entry_from(ra, nA, rh, t);
          if (h >= 0) {
            const int r = hcnt[h];
            const int32_t p = rh;
            const uint32_t below = rmask[r] & ((1u << (p - r0)) - 1u);
            const int32_t pos = spre[r] + cursor[r] + __builtin_popcount(below);
            g.prod[prow + pos] = make_int2(a0 + p, cand_block(g, ra.srt[p] != 0, ra.qs[p], t - ra.pre[p]));
          }
        }
        __syncthreads();
        for (int r = tid; r < nC; r += kSymThreads) {
          const uint32_t mk = rmask[r];
          if (mk) {
            cursor[r] += __builtin_popcount(mk);
            rmask[r] = 0;
          }
        }
        __syncthreads();
      }
    }
  }
}

template <class Cap>
__device__ __forceinline__ bool fill_fits(const SymArgs& g, int32_t i) {
  return g.A.row_ptr[i + 1] - g.A.row_ptr[i] <= Cap::kRowA && g.c_row_ptr[i + 1] - g.c_row_ptr[i] <= Cap::kRowC;
}

__device__ __forceinline__ bool fill_fits_small(const SymArgs& g, int32_t i) { return fill_fits<FillSmall>(g, i); }

// Small forms, one workgroup per row: of the listed (not thin) rows, form Cap
// takes the ones that fit it but not the next smaller form Below (tiny: 21 KB
// of LDS, seven workgroups per CU; small: 34 KB, four).
template <class Cap, class Below>
__global__ __launch_bounds__(kSymThreads) void k_sym_fill_form(SymArgs g) {
  __shared__ FillShared<Cap> sh;
  if (g.totals[kTotAbort]) return;
  const int32_t nw = *g.n_wide;
  for (int32_t x = blockIdx.x; x < nw; x += gridDim.x) {
    const int32_t i = g.wide[x];
    // uniform: every thread reads the same sizes
    if (!in_panel(g, i) || !fill_fits<Cap>(g, i) || fill_fits<Below>(g, i)) continue;
    fill_row<Cap>(g, i, sh);
    __syncthreads();
  }
}

// Large form: the rows the small forms leave that fit it, found as in the
// count pass (workgroup w of G looks at list entries w, w+G, ... 256 at a
// time).
__global__ __launch_bounds__(kSymThreads) void k_sym_fill_large(SymArgs g) {
  __shared__ FillShared<FillLarge> sh;
  __shared__ int32_t rows[kSymThreads];
  __shared__ int32_t nrows;
  if (g.totals[kTotAbort]) return;
  const int tid = threadIdx.x;
  const int64_t G = gridDim.x;
  const int32_t nw = *g.n_wide;
  for (int64_t x0 = blockIdx.x; x0 < nw; x0 += G * kSymThreads) {
    if (tid == 0) nrows = 0;
    __syncthreads();
    const int64_t x = x0 + G * tid;
    const int32_t i = x < nw ? g.wide[x] : 0;
    if (x < nw && in_panel(g, i) && !fill_fits_small(g, i) && fill_fits<FillLarge>(g, i))
      rows[atomicAdd(&nrows, 1)] = i;
    __syncthreads();
    const int32_t n = nrows;
    for (int32_t x = 0; x < n; ++x) {
      fill_row<FillLarge>(g, rows[x], sh);
      __syncthreads();
    }
  }
}

// Huge form (136 KB of LDS, one workgroup per CU): the rows the count pass
// listed in g.huge, one workgroup per row.
__global__ __launch_bounds__(kSymThreads) void k_sym_fill_huge(SymArgs g) {
  __shared__ FillShared<FillHuge> sh;
  if (g.totals[kTotAbort]) return;
  const int32_t nh = *g.n_huge;
  for (int32_t x = blockIdx.x; x < nh; x += gridDim.x) {
    const int32_t i = g.huge[x];
    if (!in_panel(g, i)) continue;  // uniform
    fill_row<FillHuge>(g, i, sh);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ norm order

// One workgroup per B block row (grid-strided): a bitonic sort in LDS of the
// row's (norm, block) pairs into descending norm, ties by ascending block, the
// row padded to a power of two with entries that sort last.  A row of more
// than kSortRow blocks keeps its stored order (bsorted[k] = 0).
__global__ __launch_bounds__(256) void k_sort_row_norms(MatView B, const double* __restrict__ normB,
                                                        int32_t* __restrict__ bord, double* __restrict__ bnrm,
                                                        uint8_t* __restrict__ bsorted) {
  __shared__ double key[kSortRow];
  __shared__ int32_t idx[kSortRow];
  const int tid = threadIdx.x;
  for (int32_t k = blockIdx.x; k < B.nbrows; k += gridDim.x) {
    const int32_t q0 = B.row_ptr[k], n = B.row_ptr[k + 1] - q0;  // uniform over the workgroup
    if (n > kSortRow) {
      if (tid == 0) bsorted[k] = 0;
      continue;
    }
    int32_t m = 1;
    while (m < n) m <<= 1;
    for (int32_t x = tid; x < m; x += 256) {
      key[x] = x < n ? normB[q0 + x] : -1.0;  // norms are >= 0: padding sorts last
      idx[x] = x < n ? q0 + x : 0x7fffffff;
    }
    __syncthreads();
    for (int32_t size = 2; size <= m; size <<= 1) {
      for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
        for (int32_t x = tid; x < m; x += 256) {
          const int32_t y = x ^ stride;
          if (y > x) {
            // y before x in the final order: larger norm, or equal norm and smaller block
            const bool y_first = key[y] > key[x] || (key[y] == key[x] && idx[y] < idx[x]);
            const bool forward = (x & size) == 0;  // this run ends in final order
            if (y_first == forward) {
              const double tk = key[x];
              key[x] = key[y];
              key[y] = tk;
              const int32_t ti = idx[x];
              idx[x] = idx[y];
              idx[y] = ti;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int32_t x = tid; x < n; x += 256) {
      bord[q0 + x] = idx[x];
      bnrm[q0 + x] = key[x];
    }
    if (tid == 0) bsorted[k] = 1;
    __syncthreads();
  }
}

hipError_t launch_sort_row_norms(const MatView& B, const double* normB, int32_t* bord, double* bnrm,
                                 uint8_t* bsorted, hipStream_t s) {
  if (B.nbrows <= 0) return hipSuccess;
  const int grid = B.nbrows < 65536 ? B.nbrows : 65536;
  hipLaunchKernelGGL(k_sort_row_norms, dim3(grid), dim3(256), 0, s, B, normB, bord, bnrm, bsorted);
  return hipGetLastError();
}

hipError_t launch_sym_count(const SymArgs& a, hipStream_t s) {
  if (a.A.nbrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_count_thin, dim3((a.A.nbrows + 255) / 256), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int grid = a.A.nbrows < 65536 ? a.A.nbrows : 65536;
  hipLaunchKernelGGL(k_sym_count_small, dim3(grid), dim3(kSymThreads), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sym_count_large, dim3(a.A.nbrows < 8192 ? a.A.nbrows : 8192), dim3(kSymThreads), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sym_count_huge, dim3(a.A.nbrows < 1024 ? a.A.nbrows : 1024), dim3(kSymThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sym_fill(const SymArgs& a, uint32_t launch_mask, hipStream_t s) {
  if (a.A.nbrows <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  // the thin form also writes a stack panel's end offset (prod_ptr after the
  // panel's last C block), which the numeric pass reads: with panels it runs
  // whether or not any row is thin
  if ((launch_mask & kFillThin) || a.panel) {
    hipLaunchKernelGGL(k_sym_fill_thin, dim3((a.A.nbrows + 255) / 256), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int grid = a.A.nbrows < 65536 ? a.A.nbrows : 65536;
  if (launch_mask & kFillTiny) {
    hipLaunchKernelGGL((k_sym_fill_form<FillTiny, FillNone>), dim3(grid), dim3(kSymThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (launch_mask & kFillSmall) {
    hipLaunchKernelGGL((k_sym_fill_form<FillSmall, FillTiny>), dim3(grid), dim3(kSymThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (launch_mask & kFillLarge) {
    hipLaunchKernelGGL(k_sym_fill_large, dim3(a.A.nbrows < 8192 ? a.A.nbrows : 8192), dim3(kSymThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (launch_mask & kFillHuge) {
    // With stack panels, one workgroup per listed row: a panel's rows lie
    // anywhere in the list (a strided walk would give some workgroups two of
    // them and others none), and a workgroup whose row is outside the panel
    // ends at once (a panelled multiply runs for seconds, so the empty
    // workgroups cost nothing that shows).
    const int huge_grid = a.panel ? grid : (a.A.nbrows < 512 ? a.A.nbrows : 512);
    hipLaunchKernelGGL(k_sym_fill_huge, dim3(huge_grid), dim3(kSymThreads), 0, s, a);
    e = hipGetLastError();
  }
  return e;
}

// c_row_ptr (int32) from the int64 prefix of per-row block counts; closes the
// product and value offset arrays with their totals.
__global__ __launch_bounds__(256) void k_finish_rows(int32_t nbrows, const int64_t* __restrict__ nc_pre,
                                                     const int64_t* __restrict__ np_pre,
                                                     const int64_t* __restrict__ nv_pre,
                                                     int32_t* __restrict__ c_row_ptr, int64_t* __restrict__ prod_ptr,
                                                     int64_t* __restrict__ c_blk_off,
                                                     const int64_t* __restrict__ totals) {
  if (totals[kTotAbort]) return;
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i <= nbrows) c_row_ptr[i] = (int32_t)nc_pre[i];
  if (i == 0) {
    const int64_t nnzc = nc_pre[nbrows];
    prod_ptr[nnzc] = np_pre[nbrows];
    c_blk_off[nnzc] = nv_pre[nbrows];
  }
}

hipError_t launch_finish_rows(int32_t nbrows, const int64_t* nc_pre, const int64_t* np_pre, const int64_t* nv_pre,
                              int32_t* c_row_ptr, int64_t* prod_ptr, int64_t* c_blk_off, const int64_t* totals,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_finish_rows, dim3((nbrows + 1 + 255) / 256), dim3(256), 0, s, nbrows, nc_pre, np_pre, nv_pre,
                     c_row_ptr, prod_ptr, c_blk_off, totals);
  return hipGetLastError();
}

// totals[0..5] = totals of the per-row counts and the flags (see kTot*).
__global__ void k_gather_totals(int32_t n, const int64_t* nc_pre, const int64_t* np_pre, const int64_t* nv_pre,
                                const int64_t* cand_pre, const int64_t* nf_pre, const uint32_t* flags,
                                int64_t* totals) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    totals[0] = nc_pre[n];
    totals[1] = np_pre[n];
    totals[2] = nv_pre[n];
    totals[3] = cand_pre[n];
    totals[4] = (int64_t)*flags;
    totals[5] = nf_pre[n];
    totals[kTotAbort] = 0;
    totals[kTotWide] = (int64_t)flags[1];
    totals[kTotHuge] = (int64_t)flags[2];
    totals[kTotForms] = (int64_t)flags[3];
  }
}

hipError_t launch_gather_totals(int32_t n, const int64_t* nc_pre, const int64_t* np_pre, const int64_t* nv_pre,
                                const int64_t* cand_pre, const int64_t* nf_pre, const uint32_t* flags,
                                int64_t* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_totals, dim3(1), dim3(64), 0, s, n, nc_pre, np_pre, nv_pre, cand_pre, nf_pre, flags,
                     totals);
  return hipGetLastError();
}

}  // namespace bsmm
