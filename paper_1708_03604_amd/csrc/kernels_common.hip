// Block norms, device-wide exclusive scans and the block filter.
//
// Norm order (matches the documented reading of the filter in Section 2 of the
// paper): lane l of a wave sums x_e^2 for e = l, l+64, ... with fused
// multiply-add, then partial l += partial l+d for d = 32..1, then a correctly
// rounded square root.
#include "block_scan.h"
#include "bsmm_internal.h"

namespace bsmm {

// ---------------------------------------------------------------- norms

__global__ __launch_bounds__(256) void k_block_norms(const int64_t* __restrict__ blk_off,
                                                     const double* __restrict__ values,
                                                     const int64_t* __restrict__ d_nnzb,
                                                     double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int32_t nnzb = (int32_t)*d_nnzb;
  const int32_t nwaves = gridDim.x * (blockDim.x >> 6);
  for (int32_t b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < nnzb; b += nwaves) {
    const int64_t o = blk_off[b];
    const int64_t n = blk_off[b + 1] - o;
    const double* x = values + o;
    double p = 0.0;
    // sixteen loads in flight (a 23x23 block in one round), then the FMAs in
    // ascending e; elements past the block count as +0, which leaves p as is
    for (int64_t e = lane; e < n; e += 16 * 64) {
      double v[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) v[t] = (e + 64 * t < n) ? x[e + 64 * t] : 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) p = fma(v[t], v[t], p);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const double other = __shfl_down(p, d, 64);
      if (lane < d) p = p + other;
    }
    if (lane == 0) out[b] = sqrt(p);
  }
}

// Blocks of at most kNormSmall values: four blocks per wave, 16 lanes each.
// Lane j of a group keeps the partials j, j+16, j+32 and j+48 of the 64-lane
// order above (element e feeds partial e mod 64, ascending e), and the tree
// adds them in the same order: partials l and l+32 within the lane, then l
// and l+16 within the lane, then across lanes for 8, 4, 2, 1.  Results are
// bit-identical to k_block_norms.
constexpr int kNormSmall = 256;

__global__ __launch_bounds__(256) void k_block_norms_small(const int64_t* __restrict__ blk_off,
                                                           const double* __restrict__ values,
                                                           const int64_t* __restrict__ d_nnzb,
                                                           double* __restrict__ out) {
  const int lane = threadIdx.x & 63, grp = lane >> 4, j = lane & 15;
  const int32_t nnzb = (int32_t)*d_nnzb;
  const int32_t nwaves = gridDim.x * (blockDim.x >> 6);
  for (int32_t b0 = 4 * (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); b0 < nnzb; b0 += 4 * nwaves) {
    const int32_t b = b0 + grp;
    const bool ok = b < nnzb;
    const int64_t o = ok ? blk_off[b] : 0;
    const int64_t n = ok ? blk_off[b + 1] - o : 0;
    const double* x = values + o;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
    for (int64_t e = j; e < n; e += 64) {
      q0 = fma(x[e], x[e], q0);
      if (e + 16 < n) q1 = fma(x[e + 16], x[e + 16], q1);
      if (e + 32 < n) q2 = fma(x[e + 32], x[e + 32], q2);
      if (e + 48 < n) q3 = fma(x[e + 48], x[e + 48], q3);
    }
    q0 = q0 + q2;
    q1 = q1 + q3;
    q0 = q0 + q1;
#pragma unroll
    for (int d = 8; d >= 1; d >>= 1) {
      const double other = __shfl_down(q0, d, 16);
      if (j < d) q0 = q0 + other;
    }
    if (ok && j == 0) out[b] = sqrt(q0);
  }
}

hipError_t launch_block_norms(const int64_t* blk_off, const double* values, const int64_t* d_nnzb, int64_t bound,
                              int64_t max_block, double* out, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  if (max_block <= kNormSmall) {
    int64_t blocks = (bound + 15) / 16;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_block_norms_small, dim3((uint32_t)blocks), dim3(256), 0, s, blk_off, values, d_nnzb, out);
    return hipGetLastError();
  }
  int64_t blocks = (bound + 3) / 4;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_block_norms, dim3((uint32_t)blocks), dim3(256), 0, s, blk_off, values, d_nnzb, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- scans

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;


__global__ __launch_bounds__(kScanThreads) void k_scan_partial(const int64_t* __restrict__ in, int64_t n,
                                                               int64_t* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    const int64_t i = base + (int64_t)u * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  int64_t tot;
  block_exclusive_scan<kScanThreads>(s, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of the chunk sums in place; partial[nchunks] = total.
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(int64_t* __restrict__ partial, int64_t nchunks) {
  int64_t carry = 0;
  for (int64_t base = 0; base < nchunks; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nchunks ? partial[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan<kScanThreads>(v, &tot);
    if (i < nchunks) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) partial[nchunks] = carry;
}

// out[i] = sum of in[0..i), out[n] = total; each thread owns kScanItems consecutive items.
__global__ __launch_bounds__(kScanThreads) void k_scan_final(const int64_t* __restrict__ in, int64_t n,
                                                             const int64_t* __restrict__ partial,
                                                             int64_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    v[u] = (base + u < n) ? in[base + u] : 0;
    s += v[u];
  }
  int64_t tot;
  int64_t run = partial[blockIdx.x] + block_exclusive_scan<kScanThreads>(s, &tot);
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    if (base + u < n) out[base + u] = run;
    run += v[u];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partial[gridDim.x];
}

__global__ void k_zero_i64(int64_t* p) {
  if (threadIdx.x == 0) p[0] = 0;
}

// Device-wide exclusive scan: out[0..n] (n+1 entries), out[n] = total.
// tmp needs scan_tmp_elems(n) int64 entries.  in and out must not overlap.
int64_t scan_tmp_elems(int64_t n) { return (n + kScanChunk - 1) / kScanChunk + 2; }

hipError_t scan_exclusive(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
  const int64_t nchunks = (n + kScanChunk - 1) / kScanChunk;
  if (nchunks == 0) {
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_partial, dim3((unsigned)nchunks), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s, tmp, nchunks);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nchunks), dim3(kScanThreads), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

// Exclusive scans of up to 8 int64 arrays of length n in one workgroup:
// out[a][0..n] with out[a][n] = total.  Used for the per-row counts, where n
// (block rows) is small enough that one workgroup sweeping the rows beats
// three launches per array.
constexpr int kRowScanThreads = 1024;
struct ScanSet {
  const int64_t* in[8];
  int64_t* out[8];
};

__global__ __launch_bounds__(kRowScanThreads) void k_scan_rows(ScanSet set, int narr, int64_t n) {
  __shared__ int64_t wsum[8][kRowScanThreads / 64];
  __shared__ int64_t carry[8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < 8) carry[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += kRowScanThreads) {
    const int64_t i = base + threadIdx.x;
    int64_t x[8], v[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      v[a] = (a < narr && i < n) ? set.in[a][i] : 0;
      x[a] = v[a];
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int64_t y = __shfl_up(x[a], d, 64);
        if (lane >= d) x[a] += y;
      }
    }
    if (lane == 63) {
#pragma unroll
      for (int a = 0; a < 8; ++a) wsum[a][wave] = x[a];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (a >= narr) continue;
      int64_t off = carry[a];
      for (int w = 0; w < wave; ++w) off += wsum[a][w];
      if (i < n) set.out[a][i] = off + x[a] - v[a];
    }
    __syncthreads();
    if (threadIdx.x < narr) {
      int64_t tot = 0;
      for (int w = 0; w < kRowScanThreads / 64; ++w) tot += wsum[threadIdx.x][w];
      carry[threadIdx.x] += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x < narr) set.out[threadIdx.x][n] = carry[threadIdx.x];
}

// ---------------------------------------------------------------- small helpers

__global__ void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// Multiply epilogue on the device: zero the value slack after the result and
// record the result's sizes (or the error) in the output's size record.
__global__ void k_finish_multiply(const int64_t* __restrict__ totals, double* __restrict__ values,
                                  int64_t* __restrict__ dsz) {
  const int t = threadIdx.x;
  const bool ok = totals[kTotAbort] == 0;
  if (ok)
    for (int x = t; x < kValueSlackDoubles; x += 64) values[totals[kTotNvals] + x] = 0.0;
  if (t == 0) {
    dsz[0] = ok ? totals[kTotNnzc] : 0;
    dsz[1] = ok ? totals[kTotNvals] : 0;
    dsz[2] = ok ? 0 : (totals[kTotFlags] | kErrCapacity * (totals[kTotFlags] == 0));
  }
}

hipError_t launch_finish_multiply(const int64_t* totals, double* values, int64_t* dsz, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_multiply, dim3(1), dim3(64), 0, s, totals, values, dsz);
  return hipGetLastError();
}

// Reserved capacity check: raises totals[kTotAbort] if the result does not fit
// (or the symbolic pass flagged a row); every later kernel then does nothing.
__global__ void k_check_capacity(int64_t* __restrict__ totals, int64_t cap_nnzb, int64_t cap_nvals,
                                 int64_t cap_nprod, int big_stack) {
  if (threadIdx.x != 0) return;
  const bool bad = totals[kTotFlags] != 0 || totals[kTotNnzc] > cap_nnzb || totals[kTotNvals] > cap_nvals ||
                   totals[kTotNprod] > cap_nprod || totals[kTotNnzc] > 0x7fffffffLL ||
                   (!big_stack && totals[kTotNprod] > 0x7fffffffLL);
  totals[kTotAbort] = bad ? 1 : 0;
}

hipError_t launch_check_capacity(int64_t* totals, int64_t cap_nnzb, int64_t cap_nvals, int64_t cap_nprod,
                                 int big_stack, hipStream_t s) {
  hipLaunchKernelGGL(k_check_capacity, dim3(1), dim3(64), 0, s, totals, cap_nnzb, cap_nvals, cap_nprod, big_stack);
  return hipGetLastError();
}

// ---------------------------------------------------------------- stack panels

// Row panels of a stack built and consumed in parts.  With R the most
// products of one block row, panel starts lie w = max(cap - R, half) products
// apart: panel p is rows [panels[p], panels[p+1]) with panels[p] the first row
// whose products start at or after p*w (np_pre: exclusive prefix of the
// per-row product counts), panels[np] = nbrows.  A panel then holds at most
// w + R products, which is cap whenever R <= cap - half, so a panel is as
// full as the limit allows and the fill of its rows has as many rows to
// spread over the CUs as the limit lets it have.  totals[kTotPanelMax]
// receives the most products of any panel (above cap the multiply is aborted:
// later kernels do nothing) and totals[kTotPanelUsed] the number of panels
// that hold a row.
__global__ __launch_bounds__(256) void k_panel_rows(const int64_t* __restrict__ np_pre, int32_t nbrows, int64_t half,
                                                    int32_t np, int64_t cap, int32_t* __restrict__ panels,
                                                    int64_t* __restrict__ totals) {
  __shared__ int32_t bnd[kMaxPanels + 1];
  __shared__ unsigned long long most, row_most;
  __shared__ int32_t used;
  if (threadIdx.x == 0) {
    most = 0;
    row_most = 0;
    used = 0;
  }
  __syncthreads();
  unsigned long long r = 0;
  for (int32_t i = threadIdx.x; i < nbrows; i += blockDim.x) {
    const unsigned long long d = (unsigned long long)(np_pre[i + 1] - np_pre[i]);
    r = d > r ? d : r;
  }
  atomicMax(&row_most, r);
  __syncthreads();
  const int64_t R = (int64_t)row_most;
  const int64_t w = cap - R > half ? cap - R : half;
  for (int32_t p = threadIdx.x; p <= np; p += blockDim.x) {
    int32_t lo = 0, hi = nbrows;
    if (p == np) {
      lo = nbrows;
    } else {
      const int64_t t = (int64_t)p * w;
      while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (np_pre[mid] < t) lo = mid + 1;
        else hi = mid;
      }
    }
    bnd[p] = lo;
    panels[p] = lo;
  }
  __syncthreads();
  for (int32_t p = threadIdx.x; p < np; p += blockDim.x) {
    atomicMax(&most, (unsigned long long)(np_pre[bnd[p + 1]] - np_pre[bnd[p]]));
    if (bnd[p] < bnd[p + 1]) atomicAdd(&used, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    totals[kTotPanelMax] = (int64_t)most;
    totals[kTotPanelUsed] = used;
    if ((int64_t)most > cap) totals[kTotAbort] = 1;
  }
}

hipError_t launch_panel_rows(const int64_t* np_pre, int32_t nbrows, int64_t half, int32_t np, int64_t cap,
                             int32_t* panels, int64_t* totals, hipStream_t s) {
  if (np < 1 || np > kMaxPanels) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_panel_rows, dim3(1), dim3(256), 0, s, np_pre, nbrows, half, np, cap, panels, totals);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Frobenius norm

// Fixed-order sum of squares: workgroup g sums a contiguous slice of the
// values (thread t takes every 256th element from t, fused multiply-add),
// then a pairwise tree over the 256 threads; the final pass adds the
// per-workgroup partials the same way and takes the square root.
constexpr int kFrobGroups = 256;

__device__ double block_tree_sum(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if ((int)threadIdx.x < d) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + d];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(256) void k_frob_partial(const double* __restrict__ values,
                                                      const int64_t* __restrict__ d_nvals,
                                                      double* __restrict__ partial) {
  const int64_t n = *d_nvals;
  const int64_t per = (n + kFrobGroups - 1) / kFrobGroups;
  const int64_t b0 = per * blockIdx.x;
  const int64_t b1 = b0 + per < n ? b0 + per : n;
  double p = 0.0;
  // sixteen loads in flight, then the FMAs in ascending e (elements past the
  // slice count as +0, which leaves p as is)
  for (int64_t e = b0 + threadIdx.x; e < b1; e += 16 * 256) {
    double v[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = (e + 256 * t < b1) ? values[e + 256 * t] : 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) p = fma(v[t], v[t], p);
  }
  const double t = block_tree_sum(p);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_frob_final(const double* __restrict__ partial, double* __restrict__ out) {
  const double t = block_tree_sum(partial[threadIdx.x]);
  if (threadIdx.x == 0) out[0] = sqrt(t);
}

int64_t frobenius_tmp_elems() { return kFrobGroups; }

hipError_t launch_frobenius(const double* values, const int64_t* d_nvals, double* partial, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_frob_partial, dim3(kFrobGroups), dim3(256), 0, s, values, d_nvals, partial);
  hipLaunchKernelGGL(k_frob_final, dim3(1), dim3(256), 0, s, partial, out);
  return hipGetLastError();
}

// The same for n <= kRowScanThreads * kRowScanItems rows in one pass: each
// thread loads its kRowScanItems consecutive rows of every array first (one
// round of loads instead of one per 1024 rows), the workgroup scans the
// per-thread sums, and each thread writes its rows' prefixes.
constexpr int kRowScanItems = 4;
__global__ __launch_bounds__(kRowScanThreads) void k_scan_rows_one(ScanSet set, int narr, int64_t n) {
  __shared__ int64_t wsum[8][kRowScanThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)threadIdx.x * kRowScanItems;
  int64_t v[8][kRowScanItems], x[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    x[a] = 0;
#pragma unroll
    for (int u = 0; u < kRowScanItems; ++u) {
      v[a][u] = (a < narr && i0 + u < n) ? set.in[a][i0 + u] : 0;
      x[a] += v[a][u];
    }
  }
  int64_t t[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) t[a] = x[a];
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int64_t y = __shfl_up(x[a], d, 64);
      if (lane >= d) x[a] += y;
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int a = 0; a < 8; ++a) wsum[a][wave] = x[a];
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (a >= narr) continue;
    int64_t run = x[a] - t[a];
    for (int w = 0; w < wave; ++w) run += wsum[a][w];
#pragma unroll
    for (int u = 0; u < kRowScanItems; ++u) {
      if (i0 + u < n) set.out[a][i0 + u] = run;
      run += v[a][u];
    }
  }
  if (threadIdx.x < narr) {
    int64_t tot = 0;
    for (int w = 0; w < kRowScanThreads / 64; ++w) tot += wsum[threadIdx.x][w];
    set.out[threadIdx.x][n] = tot;
  }
}

hipError_t scan_rows(const int64_t* const* in, int64_t* const* out, int narr, int64_t n, int64_t* tmp,
                     hipStream_t s) {
  if (n > (1 << 16)) {
    for (int a = 0; a < narr; ++a) {
      hipError_t e = scan_exclusive(in[a], n, out[a], tmp, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  ScanSet set{};
  for (int a = 0; a < narr; ++a) {
    set.in[a] = in[a];
    set.out[a] = out[a];
  }
  if (n <= (int64_t)kRowScanThreads * kRowScanItems)
    hipLaunchKernelGGL(k_scan_rows_one, dim3(1), dim3(kRowScanThreads), 0, s, set, narr, n);
  else
    hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(kRowScanThreads), 0, s, set, narr, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- filter

// keep[b] = 1 if eps <= 0 or norm > eps; vsz[b] = its value count if kept.
// Entries from the matrix's block count up to the launch bound are zero, so
// the scans may run over the bound.
__global__ __launch_bounds__(256) void k_filter_flags(const int64_t* __restrict__ blk_off,
                                                      const double* __restrict__ norms,
                                                      const int64_t* __restrict__ d_nnzb, int64_t bound,
                                                      double eps, int64_t* __restrict__ keep,
                                                      int64_t* __restrict__ vsz) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= bound) return;
  const bool live = b < *d_nnzb;
  const bool k = live && ((eps <= 0.0) || (norms[b] > eps));
  keep[b] = k ? 1 : 0;
  vsz[b] = k ? (blk_off[b + 1] - blk_off[b]) : 0;
}

// One wave per source block: copy kept blocks to their compacted position.
__global__ __launch_bounds__(256) void k_filter_compact(const int64_t* __restrict__ d_nnzb,
                                                        const int64_t* __restrict__ keep_pos,
                                                        const int64_t* __restrict__ voff,
                                                        const int32_t* __restrict__ col_idx,
                                                        const int64_t* __restrict__ blk_off,
                                                        const double* __restrict__ values,
                                                        int32_t* __restrict__ out_col_idx,
                                                        int64_t* __restrict__ out_blk_off,
                                                        double* __restrict__ out_values) {
  const int lane = threadIdx.x & 63;
  const int32_t nnzb = (int32_t)*d_nnzb;
  const int32_t nwaves = gridDim.x * 4;
  for (int32_t b = blockIdx.x * 4 + (threadIdx.x >> 6); b < nnzb; b += nwaves) {
    const int64_t pos = keep_pos[b];
    if (keep_pos[b + 1] == pos) continue;  // dropped
    const int64_t src = blk_off[b], n = blk_off[b + 1] - src, dst = voff[b];
    if (lane == 0) {
      out_col_idx[pos] = col_idx[b];
      out_blk_off[pos] = dst;
    }
    for (int64_t e = lane; e < n; e += 64) out_values[dst + e] = values[src + e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out_blk_off[keep_pos[nnzb]] = voff[nnzb];
}

__global__ __launch_bounds__(256) void k_filter_rowptr(int32_t nbrows, const int32_t* __restrict__ row_ptr,
                                                       const int64_t* __restrict__ keep_pos,
                                                       int32_t* __restrict__ out_row_ptr) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i <= nbrows) out_row_ptr[i] = (int32_t)keep_pos[row_ptr[i]];
}

// New sizes into the size record (in place: d_nnzb may be dsz itself), and
// zero slack after the new values.
__global__ void k_filter_finish(const int64_t* __restrict__ keep_pos, const int64_t* __restrict__ voff,
                                int64_t bound, double* __restrict__ out_values, int64_t* __restrict__ dsz) {
  const int64_t nv = voff[bound];
  const int t = threadIdx.x;
  for (int x = t; x < kValueSlackDoubles; x += 64) out_values[nv + x] = 0.0;
  __syncthreads();
  if (t == 0) {
    dsz[0] = keep_pos[bound];
    dsz[1] = nv;
  }
}

hipError_t launch_filter(const int32_t* row_ptr, const int32_t* col_idx, const int64_t* blk_off,
                         const double* values, int32_t nbrows, int64_t* dsz, int64_t bound, const double* norms,
                         double eps, int64_t* keep, int64_t* vsz, int64_t* keep_pos, int64_t* voff, int64_t* tmp,
                         int32_t* out_row_ptr, int32_t* out_col_idx, int64_t* out_blk_off,
                         double* out_values, hipStream_t s) {
  if (bound > 0) {
    hipLaunchKernelGGL(k_filter_flags, dim3((uint32_t)((bound + 255) / 256)), dim3(256), 0, s, blk_off, norms, dsz,
                       bound, eps, keep, vsz);
  }
  hipError_t e = scan_exclusive(keep, bound, keep_pos, tmp, s);
  if (e != hipSuccess) return e;
  e = scan_exclusive(vsz, bound, voff, tmp, s);
  if (e != hipSuccess) return e;
  int64_t blocks = (bound + 3) / 4;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_filter_compact, dim3((uint32_t)blocks), dim3(256), 0, s, dsz, keep_pos, voff, col_idx,
                     blk_off, values, out_col_idx, out_blk_off, out_values);
  hipLaunchKernelGGL(k_filter_rowptr, dim3((nbrows + 1 + 255) / 256), dim3(256), 0, s, nbrows, row_ptr, keep_pos,
                     out_row_ptr);
  hipLaunchKernelGGL(k_filter_finish, dim3(1), dim3(64), 0, s, keep_pos, voff, bound, out_values, dsz);
  return hipGetLastError();
}

}  // namespace bsmm
