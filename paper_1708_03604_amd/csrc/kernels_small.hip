// Batched block products for matrices whose block edges are all <= 16, such
// as the 5/13 atom blocks of the amorphous-material benchmark (Section 3.2):
// every (m, n, k) combination of the stack runs in one persistent launch.
//
// C blocks are partitioned by padded shape class (MP, NP) in {8, 16}^2 (edges
// up to 8 are padded to 8, the rest to 16).  One launch walks the four class
// lists in turn; within a class every wave owns one C block at a time and
// accumulates the whole block in registers, so no C block has two writers
// and results do not depend on scheduling.
//
// Register tile.  Lane l = 16*s + 4*rho + gam owns rows rho*RM .. rho*RM+RM-1
// and columns gam*RN .. gam*RN+RN-1 of the padded MP x NP block
// (RM = MP/4, RN = NP/4) for inner indices t = s, s+4, s+8, s+12 (K slice s).
// At the end of a C block the four K slices are summed with cross-lane swaps.
//
// Operands.  A product's A block (m x k, row-major) and B block (k x n) are
// contiguous in memory; the wave loads them as one run of m*k + k*n doubles
// (lane l takes elements l, l+64, ...), so every load is coalesced whatever
// the sizes.  Products are fetched D steps before they are multiplied (D
// register slots) and written one step ahead into one of two LDS stages: A
// transposed (row t holds A(:, t)) and B as is, both with a row stride of 18
// doubles, so a lane reads its RM rows and RN columns of inner index t with
// 16-byte loads.  Padding rows and columns are never zeroed: a padded row or
// column of A or B only reaches padded outputs, which are never stored.
#include <type_traits>

#include "bsmm_internal.h"

namespace bsmm {

namespace {

// f(integral_constant<int, I>) for I = B .. E-1, unrolled at compile time.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>());
    static_for<B + 1, E>(f);
  }
}

// ------------------------------------------------------------ class lists

constexpr int kClassThreads = 256;
constexpr int kClassPer = 8;
constexpr int kClassChunk = kClassThreads * kClassPer;  // C blocks per workgroup

__device__ __forceinline__ int shape_class(const int32_t* __restrict__ c_col_idx,
                                           const int32_t* __restrict__ c_col_sizes,
                                           const int64_t* __restrict__ c_blk_off, int32_t c, int32_t* mn) {
  const int32_t n = c_col_sizes[c_col_idx[c]];
  const int32_t m = (int32_t)((c_blk_off[c + 1] - c_blk_off[c]) / n);
  *mn = m | (n << 8);
  return (m > 8 ? 2 : 0) + (n > 8 ? 1 : 0);
}

// Exclusive scan of a packed counter (four 16-bit fields) over 256 threads.
__device__ uint64_t class_scan(uint64_t v, uint64_t* total) {
  __shared__ uint64_t wsum[kClassThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint64_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kClassThreads / 64; ++w) {
    if (w < wave) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// cnt[cls * nchunks + chunk] = number of C blocks of class cls in the chunk.
__global__ __launch_bounds__(kClassThreads) void k_class_count(const int64_t* __restrict__ totals, int32_t nchunks,
                                                               const int32_t* __restrict__ c_col_idx,
                                                               const int32_t* __restrict__ c_col_sizes,
                                                               const int64_t* __restrict__ c_blk_off,
                                                               int64_t* __restrict__ cnt) {
  const int32_t nnzc = live_nnzc(totals);
  const int32_t chunk = blockIdx.x;
  uint64_t packed = 0;
#pragma unroll
  for (int u = 0; u < kClassPer; ++u) {
    const int32_t c = chunk * kClassChunk + threadIdx.x * kClassPer + u;
    if (c < nnzc) {
      int32_t mn;
      packed += 1ull << (16 * shape_class(c_col_idx, c_col_sizes, c_blk_off, c, &mn));
    }
  }
  uint64_t total;
  (void)class_scan(packed, &total);
  if (threadIdx.x < 4) cnt[(int64_t)threadIdx.x * nchunks + chunk] = (int64_t)((total >> (16 * threadIdx.x)) & 0xffff);
}

// Stable partition of the C blocks by class (classes in order 0..3, each in
// ascending C block order) into list, two int4 per C block:
//   {m | n << 8, first product, product count, 0}, {C offset, C_in offset or -1}
// cls_start[0..4] = class boundaries.
__global__ __launch_bounds__(kClassThreads) void k_class_scatter(
    const int64_t* __restrict__ totals, int32_t nchunks, const int32_t* __restrict__ c_col_idx, const int32_t* __restrict__ c_col_sizes,
    const int64_t* __restrict__ c_blk_off, const int64_t* __restrict__ prod_ptr,
    const int32_t* __restrict__ c_old_idx, const int64_t* __restrict__ old_off, int use_old,
    const int64_t* __restrict__ off, int4* __restrict__ list, int32_t* __restrict__ cls_start) {
  const int32_t nnzc = live_nnzc(totals);
  const int32_t chunk = blockIdx.x;
  int cls[kClassPer];
  int32_t mn[kClassPer];
  uint64_t packed = 0;
#pragma unroll
  for (int u = 0; u < kClassPer; ++u) {
    const int32_t c = chunk * kClassChunk + threadIdx.x * kClassPer + u;
    cls[u] = -1;
    if (c < nnzc) {
      cls[u] = shape_class(c_col_idx, c_col_sizes, c_blk_off, c, &mn[u]);
      packed += 1ull << (16 * cls[u]);
    }
  }
  uint64_t total;
  uint64_t run = class_scan(packed, &total);
#pragma unroll
  for (int u = 0; u < kClassPer; ++u) {
    if (cls[u] >= 0) {
      const int32_t c = chunk * kClassChunk + threadIdx.x * kClassPer + u;
      const int64_t pos = off[(int64_t)cls[u] * nchunks + chunk] + (int64_t)((run >> (16 * cls[u])) & 0xffff);
      const int64_t p0 = prod_ptr[c];
      const int32_t o = use_old ? c_old_idx[c] : -1;
      const int64_t coff = c_blk_off[c];
      const int64_t ooff = o >= 0 ? old_off[o] : -1;
      list[2 * pos] = make_int4(mn[u], (int32_t)p0, (int32_t)(prod_ptr[c + 1] - p0), 0);
      list[2 * pos + 1] = make_int4((int32_t)(uint32_t)coff, (int32_t)(uint32_t)((uint64_t)coff >> 32),
                                    (int32_t)(uint32_t)ooff, (int32_t)(uint32_t)((uint64_t)ooff >> 32));
      run += 1ull << (16 * cls[u]);
    }
  }
  if (chunk == 0 && threadIdx.x <= 4) cls_start[threadIdx.x] = (int32_t)off[(int64_t)threadIdx.x * nchunks];
}

// ------------------------------------------------------------ numeric

constexpr int kStride = 18;                  // doubles per LDS row
constexpr int kOperand = 16 * kStride;       // one staged operand (16 inner rows)
constexpr int kStage = 2 * kOperand;         // A^T then B
constexpr int kXcds = 8;
constexpr int kChunk = 16;                   // C blocks per scheduling chunk (<= 64)

__device__ __forceinline__ void swap32(double& lo, double& hi) {
  // lanes 0-31 end with (lo, partner lo), lanes 32-63 with (partner hi, hi)
  const unsigned long long l = __double_as_longlong(lo), h = __double_as_longlong(hi);
  const auto r0 = __builtin_amdgcn_permlane32_swap((unsigned)l, (unsigned)h, false, false);
  const auto r1 = __builtin_amdgcn_permlane32_swap((unsigned)(l >> 32), (unsigned)(h >> 32), false, false);
  lo = __longlong_as_double((long long)(((unsigned long long)r1[0] << 32) | r0[0]));
  hi = __longlong_as_double((long long)(((unsigned long long)r1[1] << 32) | r0[1]));
}

__device__ __forceinline__ void swap16(double& lo, double& hi) {
  // within each 32-lane half: lanes 0-15 end with (lo, partner lo), 16-31 with (partner hi, hi)
  const unsigned long long l = __double_as_longlong(lo), h = __double_as_longlong(hi);
  const auto r0 = __builtin_amdgcn_permlane16_swap((unsigned)l, (unsigned)h, false, false);
  const auto r1 = __builtin_amdgcn_permlane16_swap((unsigned)(l >> 32), (unsigned)(h >> 32), false, false);
  lo = __longlong_as_double((long long)(((unsigned long long)r1[0] << 32) | r0[0]));
  hi = __longlong_as_double((long long)(((unsigned long long)r1[1] << 32) | r0[1]));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SmallOps {
  const double* Av;
  const double* Bv;
  const double* Ov;
  const int4* list;
  const int4* desc;
  double* Cv;
  double alpha, beta;
};

__device__ __forceinline__ int64_t make64(int32_t lo, int32_t hi) {
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// One class: C blocks list[L0, L1) padded to MP x NP, D products in flight.
//
// The wave walks its C blocks (chunks of kChunk list entries) as one stream of
// slots: one slot per product, and one empty slot for a C block without
// products.  A slot carries the operand loads of its product and, on the last
// slot of a C block, the block's finishing data.  Every slot issues exactly
// ROWS vector loads (lanes past the product's elements reread its first
// element), so the compiler can count outstanding loads exactly and the D
// slots in flight never force each other to complete early.  Indices come
// from scalar loads of the list entry and of the product descriptor, both
// read in sequential order.
template <int MP, int NP, int D>
__device__ __forceinline__ void small_class(const SmallOps& P, double* __restrict__ wl, int32_t L0, int32_t L1,
                                            int32_t xcd, int32_t wpx, int32_t wix, int lane) {
  constexpr int RM = MP / 4, RN = NP / 4, V = RM * RN;
  constexpr int ROWS = (MP * 16 + 16 * NP) / 64;  // element rows of the largest product (k = 16)
  static_assert(V % 4 == 0 && D % 2 == 0, "tile shape");
  const int s = lane >> 4, rho = (lane >> 2) & 3, gam = lane & 3;

  // This XCD's part of the list, taken in chunks of kChunk C blocks.
  const int32_t L = L1 - L0;
  const int32_t X0 = L0 + (int32_t)((int64_t)L * xcd / kXcds);
  const int32_t X1 = L0 + (int32_t)((int64_t)L * (xcd + 1) / kXcds);
  if (X0 + wix * kChunk >= X1) return;

  // ---- fetch cursor: entry fe of chunk fq (entries fe .. fe_end-1), product fp
  int32_t fq = wix, fe = X0 + wix * kChunk, fe_end = min(fe + kChunk, X1);
  bool fok = true;
  int32_t fmn = 0, fp = 0, fpe = 0;
  int64_t fcoff = 0, fooff = -1;
  auto load_entry = [&]() {
    const int4 a = P.list[2 * (int64_t)fe];
    const int4 b = P.list[2 * (int64_t)fe + 1];
    fmn = a.x;
    fp = a.y;
    fpe = a.y + a.z;
    fcoff = make64(b.x, b.y);
    fooff = make64(b.z, b.w);
  };
  auto next_entry = [&]() {
    ++fe;
    if (fe >= fe_end) {
      fq += wpx;
      fe = X0 + fq * kChunk;
      if (fe >= X1) {
        fok = false;
        return;
      }
      fe_end = min(fe + kChunk, X1);
    }
    load_entry();
  };
  load_entry();

  // ---- slots: product X lives in slot X % D from its fetch to its stage write
  double sv[D][ROWS];
  int32_t sok[D], smk[D], skn[D], sk[D], sn[D], slast[D], smn[D];
  int64_t scoff[D], sooff[D];
  auto fetch = [&](auto slot) {
    constexpr int d = decltype(slot)::value;
    int64_t ao = 0, bo = 0;
    int32_t mk = 0, kn = 0;
    sok[d] = fok;
    if (fok) {
      const int32_t m = fmn & 255, n = fmn >> 8;
      const bool empty = fp == fpe;
      int32_t k = 0;
      if (!empty) {
        const int4 dsc = P.desc[fp];
        ao = make64(dsc.x, dsc.y & 0xffffff);
        k = (int32_t)((uint32_t)dsc.y >> 24);
        bo = make64(dsc.z, dsc.w);
        mk = m * k;
        kn = k * n;
        ++fp;
      }
      smk[d] = mk;
      skn[d] = kn;
      sk[d] = k;
      sn[d] = n;
      slast[d] = fp == fpe;
      smn[d] = fmn;
      scoff[d] = fcoff;
      sooff[d] = fooff;
      if (fp == fpe) next_entry();
    }
    // ROWS loads, always: element e of the run A block ++ B block, or the
    // product's first element for lanes past its end
    const int32_t tot = mk + kn;
    const double* pa = P.Av + ao;
    const double* pb = P.Bv + bo - mk;
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const int e = lane + 64 * j;
      const double* src = e < mk ? pa + e : (e < tot ? pb + e : pa);
      sv[d][j] = *src;
    }
  };
  // what each LDS stage holds: valid slot, inner size, and the finishing data
  // of its C block if the slot is the block's last
  int32_t stok[2] = {0, 0}, stk[2] = {0, 0}, stlast[2] = {0, 0}, stmn[2] = {0, 0};
  int64_t stcoff[2] = {0, 0}, stooff[2] = {-1, -1};
  auto stage_write = [&](auto slot, auto stage) {
    constexpr int d = decltype(slot)::value;
    constexpr int st = decltype(stage)::value;
    const int32_t mk = smk[d], kn = skn[d], k = sk[d], n = sn[d];
    stok[st] = sok[d];
    stk[st] = k;
    stlast[st] = slast[d];
    stmn[st] = smn[d];
    stcoff[st] = scoff[d];
    stooff[st] = sooff[d];
    if (k == 0) return;
    const float rk = 1.0f / (float)k, rn = 1.0f / (float)n;
    double* At = wl + st * kStage;
    double* Bs = At + kOperand;
    const int32_t tot = mk + kn;
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const int e = lane + 64 * j;
      if (e < mk) {
        const int r = (int)(((float)e + 0.5f) * rk);
        const int t = e - r * k;
        At[t * kStride + r] = sv[d][j];
      } else if (e < tot) {
        const int e2 = e - mk;
        const int t = (int)(((float)e2 + 0.5f) * rn);
        const int c = e2 - t * n;
        Bs[t * kStride + c] = sv[d][j];
      }
    }
  };

  double acc[V];
#pragma unroll
  for (int x = 0; x < V; ++x) acc[x] = 0.0;
  auto compute = [&](auto stage) {
    constexpr int st = decltype(stage)::value;
    const int32_t k = stk[st];
    const double* At = wl + st * kStage + rho * RM;
    const double* Bs = wl + st * kStage + kOperand + gam * RN;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (4 * j < k) {
        const int t = s + 4 * j;
        if (t < k) {
          double a[RM], b[RN];
#pragma unroll
          for (int h = 0; h < RM / 2; ++h) {
            const double2 v = reinterpret_cast<const double2*>(At + t * kStride)[h];
            a[2 * h] = v.x;
            a[2 * h + 1] = v.y;
          }
#pragma unroll
          for (int h = 0; h < RN / 2; ++h) {
            const double2 v = reinterpret_cast<const double2*>(Bs + t * kStride)[h];
            b[2 * h] = v.x;
            b[2 * h + 1] = v.y;
          }
#pragma unroll
          for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int jj = 0; jj < RN; ++jj) acc[i * RN + jj] = fma(a[i], b[jj], acc[i * RN + jj]);
        }
      }
    }
  };

  // Finish the C block whose last product stage fs held: sum the K slices,
  // park alpha*acc row-major in stage fs (free once multiplied), add
  // beta*C_in and store coalesced.
  auto finish = [&](auto freestage) {
    constexpr int fs = decltype(freestage)::value;
    double* const tile = wl + fs * kStage;
#pragma unroll
    for (int x = 0; x < V / 2; ++x) {
      swap32(acc[x], acc[x + V / 2]);
      acc[x] = acc[x] + acc[x + V / 2];
    }
#pragma unroll
    for (int x = 0; x < V / 4; ++x) {
      swap16(acc[x], acc[x + V / 4]);
      acc[x] = acc[x] + acc[x + V / 4];
    }
    const int32_t m = stmn[fs] & 255, n = stmn[fs] >> 8;
    // this lane's outputs are tile slots y = (V/4)*s + x
#pragma unroll
    for (int x = 0; x < V / 4; ++x) {
      const int y = (V / 4) * s + x;
      const int R = rho * RM + y / RN, Cc = gam * RN + y % RN;
      if (R < m && Cc < n) tile[R * n + Cc] = P.alpha * acc[x];
    }
    wave_sync();
    const int32_t mnv = m * n;
    double* out = P.Cv + stcoff[fs];
    const int64_t oo = stooff[fs];
    if (oo >= 0) {
      const double* ov = P.Ov + oo;
      double ol[MP * NP / 64];
#pragma unroll
      for (int u = 0; u < MP * NP / 64; ++u) {
        const int e = lane + 64 * u;
        ol[u] = ov[e < mnv ? e : 0];
      }
#pragma unroll
      for (int u = 0; u < MP * NP / 64; ++u) {
        const int e = lane + 64 * u;
        if (e < mnv) out[e] = tile[e] + P.beta * ol[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < MP * NP / 64; ++u) {
        const int e = lane + 64 * u;
        if (e < mnv) out[e] = tile[e];
      }
    }
    wave_sync();
#pragma unroll
    for (int x = 0; x < V; ++x) acc[x] = 0.0;
  };

  // Prime: slots 0..D-1, slot 0 into stage 0, slot 0 refilled.
  static_for<0, D>([&](auto d) { fetch(d); });
  stage_write(std::integral_constant<int, 0>(), std::integral_constant<int, 0>());
  fetch(std::integral_constant<int, 0>());

  // Step i (slot n = i mod D, in stage n & 1): write slot n+1 into the other
  // stage, refill its register slot with slot n+1+D, multiply slot n, and if
  // slot n ends its C block, finish the block.
  bool more = true;
  while (more) {
    static_for<0, D>([&](auto idx) {
      constexpr int i = decltype(idx)::value;
      constexpr int nx = (i + 1) % D;
      constexpr int st = i & 1;
      if (!more) return;
      if (!stok[st]) {
        more = false;
        return;
      }
      stage_write(std::integral_constant<int, nx>(), std::integral_constant<int, st ^ 1>());
      fetch(std::integral_constant<int, nx>());
      wave_sync();
      compute(std::integral_constant<int, st>());
      if (stlast[st]) {
        wave_sync();
        finish(std::integral_constant<int, st>());
      }
    });
  }
}

__global__ __launch_bounds__(256) void k_numeric_small(const double* __restrict__ Av, const double* __restrict__ Bv,
                                                       const double* __restrict__ Ov, const int4* __restrict__ list,
                                                       const int32_t* __restrict__ cls_start,
                                                       const int4* __restrict__ desc, double* __restrict__ Cv,
                                                       double alpha, double beta) {
  __shared__ __align__(16) double lds[4][2 * kStage];
  const SmallOps P{Av, Bv, Ov, list, desc, Cv, alpha, beta};
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t xcd = blockIdx.x % kXcds;
  const int32_t wpx = (int32_t)(gridDim.x / kXcds) * 4;
  const int32_t wix = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x / kXcds) * 4 + wv);
  double* wl = &lds[wv][0];
  int32_t b[5];
#pragma unroll
  for (int x = 0; x < 5; ++x) b[x] = cls_start[x];
  small_class<8, 8, 4>(P, wl, b[0], b[1], xcd, wpx, wix, lane);
  small_class<8, 16, 2>(P, wl, b[1], b[2], xcd, wpx, wix, lane);
  small_class<16, 8, 2>(P, wl, b[2], b[3], xcd, wpx, wix, lane);
  small_class<16, 16, 2>(P, wl, b[3], b[4], xcd, wpx, wix, lane);
}

}  // namespace

int64_t class_list_tmp_elems(int64_t nnzc_bound) {
  const int64_t nchunks = (nnzc_bound + kClassChunk - 1) / kClassChunk;
  return 4 * nchunks + 1;
}

hipError_t launch_class_lists(const NumArgs& a, int64_t* cnt, int64_t* cnt_pre, int64_t* tmp, int4* list,
                              int32_t* cls_start, hipStream_t s) {
  const int32_t nchunks = (int32_t)((a.nnzc_bound + kClassChunk - 1) / kClassChunk);
  if (nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_class_count, dim3(nchunks), dim3(kClassThreads), 0, s, a.totals, nchunks, a.c_col_idx,
                     a.c_col_sizes, a.c_blk_off, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive(cnt, 4 * (int64_t)nchunks, cnt_pre, tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_class_scatter, dim3(nchunks), dim3(kClassThreads), 0, s, a.totals, nchunks, a.c_col_idx,
                     a.c_col_sizes, a.c_blk_off, a.prod_ptr, a.c_old_idx, a.use_old ? a.Cin.blk_off : a.c_blk_off,
                     a.use_old, cnt_pre, list, cls_start);
  return hipGetLastError();
}

hipError_t launch_numeric_small(const NumArgs& a, const int4* list, const int32_t* cls_start, const int4* desc,
                                hipStream_t s) {
  if (a.nnzc_bound <= 0) return hipSuccess;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int32_t blocks = cus * 4;  // four workgroups of 4 waves per CU
  blocks = ((blocks + kXcds - 1) / kXcds) * kXcds;
  hipLaunchKernelGGL(k_numeric_small, dim3(blocks), dim3(256), 0, s, a.A.values, a.B.values,
                     a.use_old ? a.Cin.values : a.c_values, list, cls_start, desc, a.c_values, a.alpha, a.beta);
  return hipGetLastError();
}

}  // namespace bsmm
