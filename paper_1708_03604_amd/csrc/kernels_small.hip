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
// each contiguous in memory; the wave loads them with lane l taking elements
// l, l+64, ..., so every load is coalesced whatever the sizes.  Products are
// fetched D steps before they are multiplied (D register slots) and copied
// one step ahead, exactly as stored, into one of two LDS stages (contiguous
// writes, free of bank conflicts).  A lane then reads A(r, t) and B(t, c) for
// its RM rows and RN columns with 8-byte loads.  Padding rows and columns are
// never zeroed: they only reach padded outputs, which are never stored.
#include <type_traits>

#include "block_scan.h"
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

// Schedule of the numeric kernel, shared with the list layout: each class
// list is cut into 8 XCD parts (part x runs on XCD x); a part's C blocks are
// dealt to its wpx waves in chunks of kChunk consecutive blocks, round robin,
// so at any time an XCD works on a few consecutive block rows (their A blocks
// stay in its L2).  The list is stored so that each wave's chunks are
// contiguous: a wave then reads its entries and descriptors sequentially.
constexpr int kXcds = 8;
constexpr int kChunk = 16;

// First stored position (within a part of n entries) of wave w's entries.
// Parts hold fewer than 2^31 entries (C has fewer than 2^31 blocks), so the
// arithmetic is 32-bit: divisions by the run-time wave count stay cheap.
__device__ __forceinline__ int64_t wave_base(int64_t n, int32_t wpx, int32_t w) {
  const uint32_t n32 = (uint32_t)n, wp = (uint32_t)wpx, w32 = (uint32_t)w;
  const uint32_t nch = (n32 + kChunk - 1) / kChunk;
  const uint32_t q = nch / wp, r = nch - q * wp;
  const uint32_t chunks = q * w32 + (r < w32 ? r : w32);
  uint32_t e = chunks * kChunk;
  // the last chunk is the only one that may be short
  if (nch > 0 && (nch - 1) % wp < w32) e -= nch * kChunk - n32;
  return (int64_t)e;
}

// Stored position of the t-th entry (natural order) of a part of n entries.
__device__ __forceinline__ int64_t stored_pos(int64_t t, int64_t n, int32_t wpx) {
  const uint32_t t32 = (uint32_t)t, wp = (uint32_t)wpx;
  const uint32_t c = t32 / kChunk, u = t32 - c * kChunk;
  const uint32_t cq = c / wp, w = c - cq * wp;
  return wave_base(n, wpx, (int32_t)w) + (int64_t)cq * kChunk + u;
}

__device__ __forceinline__ int shape_class(const int32_t* __restrict__ c_col_idx,
                                           const int32_t* __restrict__ c_col_sizes,
                                           const int64_t* __restrict__ c_blk_off, int32_t c, int32_t* mn) {
  const int32_t n = c_col_sizes[c_col_idx[c]];
  const int32_t m = (int32_t)((uint32_t)(c_blk_off[c + 1] - c_blk_off[c]) / (uint32_t)n);
  *mn = m | (n << 8);
  return (m > 8 ? 2 : 0) + (n > 8 ? 1 : 0);
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
  (void)block_exclusive_scan<kClassThreads>(packed, &total);
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
    const int64_t* __restrict__ off, int4* __restrict__ list, int32_t* __restrict__ cls_start,
    int64_t* __restrict__ cnp, int32_t wpx) {
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
  uint64_t run = block_exclusive_scan<kClassThreads>(packed, &total);
#pragma unroll
  for (int u = 0; u < kClassPer; ++u) {
    if (cls[u] >= 0) {
      const int32_t c = chunk * kClassChunk + threadIdx.x * kClassPer + u;
      const int64_t nat = off[(int64_t)cls[u] * nchunks + chunk] + (int64_t)((run >> (16 * cls[u])) & 0xffff);
      // natural position -> stored position (see stored_pos)
      const int64_t L0 = off[(int64_t)cls[u] * nchunks], L = off[(int64_t)(cls[u] + 1) * nchunks] - L0;
      const int64_t t = nat - L0;
      int x = 0;
      while (x < kXcds - 1 && L * (x + 1) / kXcds <= t) ++x;
      const int64_t p0x = L * x / kXcds, nx = L * (x + 1) / kXcds - p0x;
      const int64_t pos = L0 + p0x + stored_pos(t - p0x, nx, wpx);
      const int64_t p0 = prod_ptr[c];
      const int32_t o = use_old ? c_old_idx[c] : -1;
      const int64_t coff = c_blk_off[c];
      const int64_t ooff = o >= 0 ? old_off[o] : -1;
      const int32_t np = (int32_t)(prod_ptr[c + 1] - p0);
      list[2 * pos] = make_int4(mn[u], (int32_t)p0, np, 0);
      cnp[pos] = np;
      list[2 * pos + 1] = make_int4((int32_t)(uint32_t)coff, (int32_t)(uint32_t)((uint64_t)coff >> 32),
                                    (int32_t)(uint32_t)ooff, (int32_t)(uint32_t)((uint64_t)ooff >> 32));
      run += 1ull << (16 * cls[u]);
    }
  }
  // positions past the live result (reserved capacity) count no products
#pragma unroll
  for (int u = 0; u < kClassPer; ++u) {
    const int32_t c = chunk * kClassChunk + threadIdx.x * kClassPer + u;
    if (c >= nnzc && c < nchunks * kClassChunk) cnp[c] = 0;
  }
  if (chunk == 0 && threadIdx.x <= 4) cls_start[threadIdx.x] = (int32_t)off[(int64_t)threadIdx.x * nchunks];
}

// Product descriptors in list order: for list entry e (a C block with np
// products from stack position p0), desc[qstart[e] + l] = {A value offset
// | k << 56, B value offset} of its l-th product.  A wave serves four
// entries at a time, 16 lanes each (a C block has about a dozen products).
// With every block of A and B of edge ue (> 0) the offsets are the block
// indices times ue^2, without gathering the offset tables.
__global__ __launch_bounds__(256) void k_class_desc(const int64_t* __restrict__ totals,
                                                    const int4* __restrict__ list,
                                                    const int64_t* __restrict__ qstart,
                                                    const int2* __restrict__ prod,
                                                    const int64_t* __restrict__ Aoff,
                                                    const int64_t* __restrict__ Boff, int32_t ue,
                                                    int4* __restrict__ desc) {
  const int32_t nnzc = live_nnzc(totals);
  const int lane = threadIdx.x & 63, g = lane >> 4, l0 = lane & 15;
  const int32_t nwaves = gridDim.x * 4;
  for (int32_t e0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4; e0 < nnzc; e0 += nwaves * 4) {
    const int32_t e = e0 + g;
    if (e >= nnzc) continue;
    const int4 ent = list[2 * (int64_t)e];
    const uint32_t m = (uint32_t)(ent.x & 255);
    // k = (m*k) / m without a division per product: for m*k <= 256 and
    // m <= 16, k = floor(m*k * ceil(2^16/m) / 2^16) exactly (the excess is at
    // most 256 / 2^16 < 1)
    const uint32_t inv = (65536u + m - 1u) / m;
    const int64_t q = qstart[e];
    for (int32_t l = l0; l < ent.z; l += 16) {
      const int64_t p = (int64_t)ent.y + l;
      const int2 ab = prod[p];
      const int32_t a = ab.x, b = ab.y;
      int64_t ao, bo;
      int32_t k;
      if (ue) {
        ao = (int64_t)a * (ue * ue);
        bo = (int64_t)b * (ue * ue);
        k = ue;
      } else {
        ao = Aoff[a];
        k = (int32_t)(((uint32_t)(Aoff[a + 1] - ao) * inv) >> 16);
        bo = Boff[b];
      }
      desc[q + l] = make_int4((int32_t)(uint32_t)ao, (int32_t)((uint32_t)(ao >> 32) | ((uint32_t)k << 24)),
                              (int32_t)(uint32_t)bo, (int32_t)(uint32_t)(bo >> 32));
    }
  }
}

// ------------------------------------------------------------ numeric

constexpr int kOperand = 256;  // doubles of one staged operand (a block of at most 16 x 16)
constexpr int kStage = 2 * kOperand;  // A then B, each stored exactly as in memory

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
  const int64_t* qstart;
  const int4* desc;
  double* Cv;
  double alpha, beta;
};

// Take ownership of a batch that was loaded a batch earlier: the empty asm
// reads the registers, so the compiler waits for their load here, once per
// batch; afterwards they are plain values and the per-product readlanes need
// no wait (the wait count the compiler would otherwise derive at each
// readlane assumes the batch load may be the most recent one).
__device__ __forceinline__ void settle(int4& v) {
  asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
}

__device__ __forceinline__ int64_t make64(int32_t lo, int32_t hi) {
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// One class: C blocks list[L0, L1) padded to MP x NP, D products in flight.
//
// Each wave takes a contiguous run of the class list (the chunks the XCD's
// round robin gives it), so its list entries and product descriptors (stored
// in list order) are contiguous.  The wave walks them as one stream of slots:
// one slot per product, and one empty slot for a C block without products.
//
// The product loop is kept short, since at a few hundred bytes per product
// the kernel is bound by instructions issued, not by memory:
//   - list entries and descriptors arrive in 64-wide vector batches read back
//     with readlane, each loaded one batch ahead, and the loop issues no
//     scalar memory loads (whose completion every LDS wait would also await);
//   - every product issues the same RA + RB operand loads from the block start
//     with immediate offsets (the value slack after every matrix covers the
//     overrun), so the compiler's wait counts are exact;
//   - a slot carries one packed word (m, n, k, valid, last); the finishing data
//     of each C block goes into a lane-indexed queue when its entry starts and
//     is read back when the block is finished;
//   - B rows k .. 4*ceil(k/4)-1 are written as zeros, so the four K slices run
//     the same number of steps with no lane masks.
template <int MP, int NP, int D>
__device__ __forceinline__ void small_class(const SmallOps& P, double* __restrict__ wl, int32_t L0, int32_t L1,
                                            int32_t xcd, int32_t wpx, int32_t wix, int lane) {
  constexpr int RM = MP / 4, RN = NP / 4, V = RM * RN;
  constexpr int RA = MP * 16 / 64, RB = 16 * NP / 64;  // element rows of the largest A and B blocks (k = 16)
  static_assert(V % 4 == 0 && D % 2 == 0, "tile shape");
  const int s = lane >> 4, rho = (lane >> 2) & 3, gam = lane & 3;

  // This wave's run of the list: [E0, E1), products [Q0, Q0 + NQ) in list order.
  const int64_t L = L1 - L0;
  const int64_t X0 = L0 + L * xcd / kXcds, X1 = L0 + L * (xcd + 1) / kXcds;
  const int32_t E0 = (int32_t)(X0 + wave_base(X1 - X0, wpx, wix));
  const int32_t E1 = (int32_t)(X0 + wave_base(X1 - X0, wpx, wix + 1));
  if (E0 >= E1) return;
  const int64_t Q0 = P.qstart[E0];
  const int32_t NQ = (int32_t)(P.qstart[E1] - Q0);
  const int4* __restrict__ dq = P.desc + Q0;

  // ---- entry batches: lane u holds entry eb + u (current) and eb + 64 + u (next)
  int32_t eb = E0, ei = E0;
  int4 ca, cb, na, nb;
  auto load_entries = [&](int32_t base, int4& x, int4& y) {
    const int64_t e = base + lane < E1 ? base + lane : E1 - 1;
    x = P.list[2 * e];
    y = P.list[2 * e + 1];
  };
  load_entries(eb, ca, cb);
  settle(ca);
  settle(cb);
  load_entries(eb + 64, na, nb);
  // ---- descriptor batches: lane u holds descriptor qb + u (current) and qb + 64 + u (next)
  int32_t qb = 0, qi = 0;
  int4 cd, nd;
  auto load_desc = [&](int32_t base, int4& x) {
    const int32_t q = base + lane < NQ ? base + lane : (NQ > 0 ? NQ - 1 : 0);
    x = dq[q];
  };
  load_desc(qb, cd);
  settle(cd);
  load_desc(qb + 64, nd);

  // ---- finishing data of the C blocks between fetch and finish: a queue in
  // lanes (entry w at lane w mod 64; at most D+1 blocks are open at a time)
  int32_t fifo_mn = 0, fifo_co0 = 0, fifo_co1 = 0, fifo_oo0 = 0, fifo_oo1 = 0;
  int32_t fw = 0, fr = 0;

  // ---- fetch cursor: current entry (m, n, products left)
  bool fok = true;
  int32_t fm = 0, fn = 0, frem = 0;
  auto take_entry = [&]() {
    const int u = ei - eb;
    const int32_t mn = __builtin_amdgcn_readlane(ca.x, u);
    fm = mn & 255;
    fn = mn >> 8;
    frem = __builtin_amdgcn_readlane(ca.z, u);
    const bool mine = lane == (fw & 63);
    fifo_mn = mine ? mn : fifo_mn;
    fifo_co0 = mine ? __builtin_amdgcn_readlane(cb.x, u) : fifo_co0;
    fifo_co1 = mine ? __builtin_amdgcn_readlane(cb.y, u) : fifo_co1;
    fifo_oo0 = mine ? __builtin_amdgcn_readlane(cb.z, u) : fifo_oo0;
    fifo_oo1 = mine ? __builtin_amdgcn_readlane(cb.w, u) : fifo_oo1;
    ++fw;
  };
  auto next_entry = [&]() {
    ++ei;
    if (ei >= E1) {
      fok = false;
      return;
    }
    if (ei - eb == 64) {
      eb += 64;
      ca = na;
      cb = nb;
      settle(ca);
      settle(cb);
      load_entries(eb + 64, na, nb);
    }
    take_entry();
  };
  take_entry();

  // ---- slots: product X lives in slot X % D from its fetch to its stage write.
  // Packed word: m | n << 5 | k << 10 | valid << 15 | last << 16.
  double sa[D][RA], sb[D][RB];
  int32_t sw[D];
  // masked-off lanes keep their previous values: start from zeros so that
  // every stale value is finite (inner steps past k multiply them by zero)
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int j = 0; j < RA; ++j) sa[d][j] = 0.0;
#pragma unroll
    for (int j = 0; j < RB; ++j) sb[d][j] = 0.0;
  }
  auto fetch = [&](auto slot) {
    constexpr int d = decltype(slot)::value;
    int64_t ao = 0, bo = 0;
    int32_t k = 0;
    if (fok && frem > 0) {
      const int u = qi - qb;
      const int32_t dy = __builtin_amdgcn_readlane(cd.y, u);
      ao = make64(__builtin_amdgcn_readlane(cd.x, u), dy & 0xffffff);
      k = (int32_t)((uint32_t)dy >> 24);
      bo = make64(__builtin_amdgcn_readlane(cd.z, u), __builtin_amdgcn_readlane(cd.w, u));
      --frem;
      ++qi;
      if (qi - qb == 64) {
        qb += 64;
        cd = nd;
        settle(cd);
        load_desc(qb + 64, nd);
      }
    }
    sw[d] = fm | (fn << 5) | (k << 10) | ((int32_t)fok << 15) | ((int32_t)(frem == 0) << 16);
    const int32_t mk = fm * k, kn = k * fn;  // before the cursor moves to the next C block
    if (fok && frem == 0) next_entry();
    // RA + RB loads from the block starts, always issued; lanes past the
    // block are masked off (no traffic) and keep stale values, which never
    // reach a stored output
    const double* pa = P.Av + ao + lane;
    const double* pb = P.Bv + bo + lane;
#pragma unroll
    for (int j = 0; j < RA; ++j)
      if (lane + 64 * j < mk) sa[d][j] = pa[64 * j];
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (lane + 64 * j < kn) sb[d][j] = pb[64 * j];
  };

  // what each LDS stage holds (the packed word of its slot)
  int32_t stw[2] = {0, 0};
  auto stage_write = [&](auto slot, auto stage) {
    constexpr int d = decltype(slot)::value;
    constexpr int st = decltype(stage)::value;
    const int32_t w = sw[d];
    stw[st] = w;
    const int32_t n = (w >> 5) & 31, k = (w >> 10) & 31;
    if (k == 0) return;
    // A and B are copied as they are stored (row-major, dense); B's values
    // past the block are written as zeros, so the rows k .. 4*ceil(k/4)-1 that
    // the K slices reach contribute nothing
    double* As = wl + st * kStage;
    double* Bs = As + kOperand;
    const int32_t kn = k * n;
#pragma unroll
    for (int j = 0; j < RA; ++j) As[lane + 64 * j] = sa[d][j];
#pragma unroll
    for (int j = 0; j < RB; ++j) Bs[lane + 64 * j] = lane + 64 * j < kn ? sb[d][j] : 0.0;
  };

  double acc[V];
#pragma unroll
  for (int x = 0; x < V; ++x) acc[x] = 0.0;
  // Lane (s, rho, gam), inner index t = s + 4j: A(rho*RM + i, t) = As[(rho*RM + i)*k + t]
  // and B(t, gam*RN + jj) = Bs[t*n + gam*RN + jj].  Rows and columns past the
  // block, and inner indices past k (where B is zero), only reach padded
  // outputs or add zeros.
  // The inner steps go in groups of G whose LDS reads are issued together
  // (reads past 4*ceil(k/4) stay inside the stage and are not used).
  auto compute = [&](auto stage) {
    constexpr int st = decltype(stage)::value;
    constexpr int G = RM + RN <= 4 ? 2 : 1;
    const int32_t w = stw[st];
    const int32_t n = (w >> 5) & 31, k = (w >> 10) & 31;
    const double* As = wl + st * kStage + rho * RM * k + s;
    const double* Bs = wl + st * kStage + kOperand + s * n + gam * RN;
#pragma unroll
    for (int j0 = 0; j0 < 4; j0 += G) {
      if (4 * j0 < k) {
        double a[G][RM], b[G][RN];
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
          for (int i = 0; i < RM; ++i) a[g][i] = As[i * k + 4 * (j0 + g)];
#pragma unroll
          for (int jj = 0; jj < RN; ++jj) b[g][jj] = Bs[4 * (j0 + g) * n + jj];
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
          if (4 * (j0 + g) < k) {
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
              for (int jj = 0; jj < RN; ++jj) acc[i * RN + jj] = fma(a[g][i], b[g][jj], acc[i * RN + jj]);
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
    const int r = fr & 63;
    ++fr;
    const int32_t mn = __builtin_amdgcn_readlane(fifo_mn, r);
    const int32_t m = mn & 255, n = mn >> 8;
    const int64_t coff = make64(__builtin_amdgcn_readlane(fifo_co0, r), __builtin_amdgcn_readlane(fifo_co1, r));
    const int64_t oo = make64(__builtin_amdgcn_readlane(fifo_oo0, r), __builtin_amdgcn_readlane(fifo_oo1, r));
    // this lane's outputs are tile slots y = (V/4)*s + x
#pragma unroll
    for (int x = 0; x < V / 4; ++x) {
      const int y = (V / 4) * s + x;
      const int R = rho * RM + y / RN, Cc = gam * RN + y % RN;
      if (R < m && Cc < n) tile[R * n + Cc] = P.alpha * acc[x];
    }
    wave_sync();
    const int32_t mnv = m * n;
    double* out = P.Cv + coff;
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

  // Step i (slot n = i mod D, in stage n & 1): multiply slot n, write slot
  // n+1 into the other stage and refill its register slot with slot n+1+D,
  // then wait for the stage writes (the next step reads them); if slot n ends
  // its C block, finish the block in its stage.
  wave_sync();
  bool more = true;
  while (more) {
    static_for<0, D>([&](auto idx) {
      constexpr int i = decltype(idx)::value;
      constexpr int nx = (i + 1) % D;
      constexpr int st = i & 1;
      if (!more) return;
      const int32_t w = stw[st];
      if (!((w >> 15) & 1)) {
        more = false;
        return;
      }
      compute(std::integral_constant<int, st>());
      stage_write(std::integral_constant<int, nx>(), std::integral_constant<int, st ^ 1>());
      fetch(std::integral_constant<int, nx>());
      wave_sync();
      if ((w >> 16) & 1) finish(std::integral_constant<int, st>());
    });
  }
}

// Several products of one C block per step: PG products, one per group of
// 64/PG lanes, each over 4/PG K slices (PG = 4 for the 8x8 class: one
// product per 16 lanes over every inner index; PG = 2 for 8x16 and 16x8).
// Lane l keeps the layout of the one-product form: quarter s = l >> 4 owns
// K slice s mod (4/PG) of the product of group s / (4/PG), and rows and
// columns by (rho, gam); the four quarters' sums are added at the end of the
// C block exactly as the K slices are.  A step holds the next one to PG
// products of the current C block (a C block's last step may leave groups
// without a product: their k is 0 and their B block is all zeros).  Against
// one product per step this divides the per-product instructions, which
// bound the small-block kernel, by up to PG.
//
// One LDS stage (each group: A then B; the tile of a finished block is
// parked there too) and D register slots of PG products.
// KM bounds the inner size k (16 in general; 8 lets two steps of the 8x8
// class fit in registers when every block edge is at most 8).
template <int MP, int NP, int PG, int D, int KM = 16>
__device__ __forceinline__ void small_multi(const SmallOps& P, double* __restrict__ wl, int32_t L0, int32_t L1,
                                            int32_t xcd, int32_t wpx, int32_t wix, int lane) {
  constexpr int RM = MP / 4, RN = NP / 4, V = RM * RN;
  constexpr int GL = 64 / PG;                      // lanes per group
  constexpr int KS = 4 / PG;                       // K slices per product
  constexpr int kA = MP * KM, kB = KM * NP;        // largest A and B blocks
  constexpr int QA = kA / GL, QB = kB / GL;        // loads per lane of a group
  constexpr int kGroup = kA + kB;                  // LDS doubles per group: A, then B
  static_assert(PG * kGroup <= 2 * kStage, "one stage of PG groups fits the wave's LDS");
  static_assert(kA % GL == 0 && kB % GL == 0 && V % 4 == 0, "tile shape");
  const int s = lane >> 4, rho = (lane >> 2) & 3, gam = lane & 3;
  const int grp = lane / GL, ks = s % KS, li = lane % GL;

  // This wave's run of the list: [E0, E1), products [Q0, Q0 + NQ) in list order.
  const int64_t L = L1 - L0;
  const int64_t X0 = L0 + L * xcd / kXcds, X1 = L0 + L * (xcd + 1) / kXcds;
  const int32_t E0 = (int32_t)(X0 + wave_base(X1 - X0, wpx, wix));
  const int32_t E1 = (int32_t)(X0 + wave_base(X1 - X0, wpx, wix + 1));
  if (E0 >= E1) return;
  const int64_t Q0 = P.qstart[E0];
  const int32_t NQ = (int32_t)(P.qstart[E1] - Q0);
  const int4* __restrict__ dq = P.desc + Q0;

  // ---- entry batches: lane u holds entry eb + u (current) and eb + 64 + u (next)
  int32_t eb = E0, ei = E0;
  int4 ca, cb, na, nb;
  auto load_entries = [&](int32_t base, int4& x, int4& y) {
    const int64_t e = base + lane < E1 ? base + lane : E1 - 1;
    x = P.list[2 * e];
    y = P.list[2 * e + 1];
  };
  load_entries(eb, ca, cb);
  settle(ca);
  settle(cb);
  load_entries(eb + 64, na, nb);
  // ---- descriptor batches: lane u holds descriptor qb + u (current) and qb + 64 + u (next)
  int32_t qb = 0, qi = 0;
  int4 cd, nd;
  auto load_desc = [&](int32_t base, int4& x) {
    const int32_t q = base + lane < NQ ? base + lane : (NQ > 0 ? NQ - 1 : 0);
    x = dq[q];
  };
  load_desc(qb, cd);
  settle(cd);
  load_desc(qb + 64, nd);

  // ---- finishing data of the C blocks between fetch and finish: a queue in
  // lanes (entry w at lane w mod 64; at most D+1 blocks are open at a time)
  int32_t fifo_mn = 0, fifo_co0 = 0, fifo_co1 = 0, fifo_oo0 = 0, fifo_oo1 = 0;
  int32_t fw = 0, fr = 0;

  // ---- fetch cursor: current entry (m, n, products left)
  bool fok = true;
  int32_t fm = 0, fn = 0, frem = 0;
  auto take_entry = [&]() {
    const int u = ei - eb;
    const int32_t mn = __builtin_amdgcn_readlane(ca.x, u);
    fm = mn & 255;
    fn = mn >> 8;
    frem = __builtin_amdgcn_readlane(ca.z, u);
    const bool mine = lane == (fw & 63);
    fifo_mn = mine ? mn : fifo_mn;
    fifo_co0 = mine ? __builtin_amdgcn_readlane(cb.x, u) : fifo_co0;
    fifo_co1 = mine ? __builtin_amdgcn_readlane(cb.y, u) : fifo_co1;
    fifo_oo0 = mine ? __builtin_amdgcn_readlane(cb.z, u) : fifo_oo0;
    fifo_oo1 = mine ? __builtin_amdgcn_readlane(cb.w, u) : fifo_oo1;
    ++fw;
  };
  auto next_entry = [&]() {
    ++ei;
    if (ei >= E1) {
      fok = false;
      return;
    }
    if (ei - eb == 64) {
      eb += 64;
      ca = na;
      cb = nb;
      settle(ca);
      settle(cb);
      load_entries(eb + 64, na, nb);
    }
    take_entry();
  };
  take_entry();

  // ---- slots: step X lives in slot X % D from its fetch to its stage write.
  // Packed word: m | n << 5 | kmax << 10 | valid << 15 | last << 16, where
  // kmax is the largest inner size of the step's products; sk holds the
  // inner size of the lane's group's product (0: none).
  double sa[D][QA], sb[D][QB];
  int32_t sw[D], sk[D];
  // masked-off lanes keep their previous values: start from zeros so that
  // every stale value is finite (inner steps past k multiply them by zero)
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int j = 0; j < QA; ++j) sa[d][j] = 0.0;
#pragma unroll
    for (int j = 0; j < QB; ++j) sb[d][j] = 0.0;
  }
  auto fetch = [&](auto slot) {
    constexpr int d = decltype(slot)::value;
    int64_t ao = 0, bo = 0;
    int32_t k = 0, kmax = 0;
    if (fok && frem > 0) {
      const int32_t cnt = frem < PG ? frem : PG;
      const int u0 = qi - qb;
      // descriptors u0 .. u0+cnt-1 of the current batch; past 63 they are
      // the first ones of the next batch
      static_for<0, PG>([&](auto gi) {
        constexpr int G = decltype(gi)::value;
        if (G < cnt) {
          const int u = u0 + G;
          const bool cur = u < 64;
          const int uu = cur ? u : u - 64;
          const int32_t dx = __builtin_amdgcn_readlane(cur ? cd.x : nd.x, uu);
          const int32_t dy = __builtin_amdgcn_readlane(cur ? cd.y : nd.y, uu);
          const int32_t dz = __builtin_amdgcn_readlane(cur ? cd.z : nd.z, uu);
          const int32_t dw = __builtin_amdgcn_readlane(cur ? cd.w : nd.w, uu);
          const int32_t kg = (int32_t)((uint32_t)dy >> 24);
          kmax = kg > kmax ? kg : kmax;
          const bool mine = grp == G;
          ao = mine ? make64(dx, dy & 0xffffff) : ao;
          bo = mine ? make64(dz, dw) : bo;
          k = mine ? kg : k;
        }
      });
      frem -= cnt;
      qi += cnt;
      if (qi - qb >= 64) {
        qb += 64;
        cd = nd;
        settle(cd);
        load_desc(qb + 64, nd);
      }
    }
    sw[d] = fm | (fn << 5) | (kmax << 10) | ((int32_t)fok << 15) | ((int32_t)(frem == 0) << 16);
    sk[d] = k;
    const int32_t mk = fm * k, kn = k * fn;  // before the cursor moves to the next C block
    if (fok && frem == 0) next_entry();
    // QA + QB loads per lane from the group's block starts, always issued;
    // lanes past the block are masked off and keep stale values
    const double* pa = P.Av + ao + li;
    const double* pb = P.Bv + bo + li;
#pragma unroll
    for (int j = 0; j < QA; ++j)
      if (li + GL * j < mk) sa[d][j] = pa[GL * j];
#pragma unroll
    for (int j = 0; j < QB; ++j)
      if (li + GL * j < kn) sb[d][j] = pb[GL * j];
  };

  // the step in the stage: its packed word and the lane's group's inner size
  int32_t stw = 0, stk = 0;
  double* const As = wl + grp * kGroup;
  double* const Bs = As + kA;
  auto stage_write = [&](auto slot) {
    constexpr int d = decltype(slot)::value;
    stw = sw[d];
    stk = sk[d];
    const int32_t n = (stw >> 5) & 31;
    // A as stored; B as stored with zeros past the block, so inner indices
    // past the group's k (up to the step's largest) add nothing
    const int32_t kn = stk * n;
#pragma unroll
    for (int j = 0; j < QA; ++j) As[li + GL * j] = sa[d][j];
#pragma unroll
    for (int j = 0; j < QB; ++j) Bs[li + GL * j] = li + GL * j < kn ? sb[d][j] : 0.0;
  };

  double acc[V];
#pragma unroll
  for (int x = 0; x < V; ++x) acc[x] = 0.0;
  // Lane (s, rho, gam), inner index t = ks + KS*j: A(rho*RM + i, t) =
  // As[(rho*RM + i)*k + t], B(t, gam*RN + jj) = Bs[t*n + gam*RN + jj] of its
  // group's product.  Inner indices past the group's k (up to the step's
  // largest, rounded up to KS) meet zero B rows.
  auto compute = [&]() {
    const int32_t n = (stw >> 5) & 31, kmax = (stw >> 10) & 31;
    const double* Ar = As + rho * RM * stk + ks;
    const double* Bc = Bs + ks * n + gam * RN;
    const int32_t steps = (kmax + KS - 1) / KS;
#pragma unroll 2
    for (int32_t j = 0; j < steps; ++j) {
      double a[RM], b[RN];
#pragma unroll
      for (int i = 0; i < RM; ++i) a[i] = Ar[i * stk + KS * j];
#pragma unroll
      for (int jj = 0; jj < RN; ++jj) b[jj] = Bc[KS * j * n + jj];
#pragma unroll
      for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int jj = 0; jj < RN; ++jj) acc[i * RN + jj] = fma(a[i], b[jj], acc[i * RN + jj]);
    }
  };

  // Finish the C block of the step just multiplied: sum the groups, park
  // alpha*acc row-major in the stage (free once multiplied), add beta*C_in
  // and store coalesced.
  auto finish = [&]() {
    double* const tile = wl;
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
    const int r = fr & 63;
    ++fr;
    const int32_t mn = __builtin_amdgcn_readlane(fifo_mn, r);
    const int32_t m = mn & 255, n = mn >> 8;
    const int64_t coff = make64(__builtin_amdgcn_readlane(fifo_co0, r), __builtin_amdgcn_readlane(fifo_co1, r));
    const int64_t oo = make64(__builtin_amdgcn_readlane(fifo_oo0, r), __builtin_amdgcn_readlane(fifo_oo1, r));
    wave_sync();  // every group has read the stage
    // this lane's outputs are tile slots y = (V/4)*s + x
#pragma unroll
    for (int x = 0; x < V / 4; ++x) {
      const int y = (V / 4) * s + x;
      const int R = rho * RM + y / RN, Cc = gam * RN + y % RN;
      if (R < m && Cc < n) tile[R * n + Cc] = P.alpha * acc[x];
    }
    wave_sync();
    const int32_t mnv = m * n;
    double* out = P.Cv + coff;
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
#pragma unroll
    for (int x = 0; x < V; ++x) acc[x] = 0.0;
  };

  // Prime: slots 0..D-1.  Step i (slot i mod D): write the slot into the
  // stage, refill it with step i+D, multiply; finish the C block if the step
  // ends it.
  static_for<0, D>([&](auto d) { fetch(d); });
  bool more = true;
  while (more) {
    static_for<0, D>([&](auto idx) {
      if (!more) return;
      if (!((sw[decltype(idx)::value] >> 15) & 1)) {
        more = false;
        return;
      }
      wave_sync();
      stage_write(idx);
      fetch(idx);
      wave_sync();
      compute();
      if ((stw >> 16) & 1) finish();
    });
  }
}

// FP64 matrix-core form: one product per step on v_mfma_f64_4x4x4_4b (four
// independent 4x4x4 products per instruction).  The padded MP x NP C block is
// a grid of 4x4 tiles, four per instruction (G = MP*NP/64 instructions per K
// step): tile tau = 4g + b of instruction group g sits at tile row tau / (NP/4)
// and tile column tau % (NP/4).  Lane 16kk + 4b + i holds A_b[i][kk] and
// B_b[kk][i]; the result lane 16i + 4b + j holds D_b[i][j].  The inner index
// runs in pairs so that one 16-byte LDS read gives a lane the operands of two
// instructions (slot kk: t = 8kp + 2kk and t + 1), so k is padded to 8 or 16.
// A product is staged in one LDS stage per wave: A as rows of stride kMmaS
// doubles, B transposed (row c holds B(:, c)) with the same stride, and the
// inner-index pads k .. kpad-1 of both written as zeros.  Rows past m and
// columns past n stay stale: they only reach outputs that are never stored.
// The C block is accumulated in G registers per lane and stored directly.
constexpr int kMmaS = 18;  // even (16-byte pairs), and eight rows of one read fall on distinct banks
// ceil(2^16 / x) for x = 1..16: (e * kInv16[x]) >> 16 = e / x for e < 256
__constant__ uint32_t kInv16[17] = {0,    65536, 32768, 21846, 16384, 13108, 10923, 9363, 8192,
                                    7282, 6554,  5958,  5462,  5042,  4682,  4370,  4096};

template <int MP, int NP, int D>
__device__ __forceinline__ void small_mfma(const SmallOps& P, double* __restrict__ wl, int32_t L0, int32_t L1,
                                           int32_t xcd, int32_t wpx, int32_t wix, int lane) {
  constexpr int TN = NP / 4, G = MP * NP / 64;
  constexpr int QA = MP * 16 / 64, QB = 16 * NP / 64;  // element loads per lane of the largest A and B (k = 16)
  static_assert((MP + NP) * kMmaS <= 2 * kStage, "the stage fits the wave's LDS");
  double* const As = wl;
  double* const Bs = wl + MP * kMmaS;
  const int kk = lane >> 4, bq = (lane >> 2) & 3, iq = lane & 3;

  // This wave's run of the list: [E0, E1), products [Q0, Q0 + NQ) in list order.
  const int64_t L = L1 - L0;
  const int64_t X0 = L0 + L * xcd / kXcds, X1 = L0 + L * (xcd + 1) / kXcds;
  const int32_t E0 = (int32_t)(X0 + wave_base(X1 - X0, wpx, wix));
  const int32_t E1 = (int32_t)(X0 + wave_base(X1 - X0, wpx, wix + 1));
  if (E0 >= E1) return;
  const int64_t Q0 = P.qstart[E0];
  const int32_t NQ = (int32_t)(P.qstart[E1] - Q0);
  const int4* __restrict__ dq = P.desc + Q0;

  // ---- entry batches: lane u holds entry eb + u (current) and eb + 64 + u (next)
  int32_t eb = E0, ei = E0;
  int4 ca, cb, na, nb;
  auto load_entries = [&](int32_t base, int4& x, int4& y) {
    const int64_t e = base + lane < E1 ? base + lane : E1 - 1;
    x = P.list[2 * e];
    y = P.list[2 * e + 1];
  };
  load_entries(eb, ca, cb);
  settle(ca);
  settle(cb);
  load_entries(eb + 64, na, nb);
  // ---- descriptor batches: lane u holds descriptor qb + u (current) and qb + 64 + u (next)
  int32_t qb = 0, qi = 0;
  int4 cd, nd;
  auto load_desc = [&](int32_t base, int4& x) {
    const int32_t q = base + lane < NQ ? base + lane : (NQ > 0 ? NQ - 1 : 0);
    x = dq[q];
  };
  load_desc(qb, cd);
  settle(cd);
  load_desc(qb + 64, nd);

  // ---- finishing data of the C blocks between fetch and finish: a queue in
  // lanes (entry w at lane w mod 64; at most D+1 blocks are open at a time)
  int32_t fifo_mn = 0, fifo_co0 = 0, fifo_co1 = 0, fifo_oo0 = 0, fifo_oo1 = 0;
  int32_t fw = 0, fr = 0;

  // ---- fetch cursor: current entry (m, n, products left)
  bool fok = true;
  int32_t fm = 0, fn = 0, frem = 0;
  auto take_entry = [&]() {
    const int u = ei - eb;
    const int32_t mn = __builtin_amdgcn_readlane(ca.x, u);
    fm = mn & 255;
    fn = mn >> 8;
    frem = __builtin_amdgcn_readlane(ca.z, u);
    const bool mine = lane == (fw & 63);
    fifo_mn = mine ? mn : fifo_mn;
    fifo_co0 = mine ? __builtin_amdgcn_readlane(cb.x, u) : fifo_co0;
    fifo_co1 = mine ? __builtin_amdgcn_readlane(cb.y, u) : fifo_co1;
    fifo_oo0 = mine ? __builtin_amdgcn_readlane(cb.z, u) : fifo_oo0;
    fifo_oo1 = mine ? __builtin_amdgcn_readlane(cb.w, u) : fifo_oo1;
    ++fw;
  };
  auto next_entry = [&]() {
    ++ei;
    if (ei >= E1) {
      fok = false;
      return;
    }
    if (ei - eb == 64) {
      eb += 64;
      ca = na;
      cb = nb;
      settle(ca);
      settle(cb);
      load_entries(eb + 64, na, nb);
    }
    take_entry();
  };
  take_entry();

  // ---- slots: product X lives in slot X % D from its fetch to its stage write.
  // Packed word: m | n << 5 | k << 10 | valid << 15 | last << 16.
  double sa[D][QA], sb[D][QB];
  int32_t sw[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int j = 0; j < QA; ++j) sa[d][j] = 0.0;
#pragma unroll
    for (int j = 0; j < QB; ++j) sb[d][j] = 0.0;
  }
  auto fetch = [&](auto slot) {
    constexpr int d = decltype(slot)::value;
    int64_t ao = 0, bo = 0;
    int32_t k = 0;
    if (fok && frem > 0) {
      const int u = qi - qb;
      const int32_t dy = __builtin_amdgcn_readlane(cd.y, u);
      ao = make64(__builtin_amdgcn_readlane(cd.x, u), dy & 0xffffff);
      k = (int32_t)((uint32_t)dy >> 24);
      bo = make64(__builtin_amdgcn_readlane(cd.z, u), __builtin_amdgcn_readlane(cd.w, u));
      --frem;
      ++qi;
      if (qi - qb == 64) {
        qb += 64;
        cd = nd;
        settle(cd);
        load_desc(qb + 64, nd);
      }
    }
    sw[d] = fm | (fn << 5) | (k << 10) | ((int32_t)fok << 15) | ((int32_t)(frem == 0) << 16);
    const int32_t mk = fm * k, kn = k * fn;  // before the cursor moves to the next C block
    if (fok && frem == 0) next_entry();
    const double* pa = P.Av + ao + lane;
    const double* pb = P.Bv + bo + lane;
#pragma unroll
    for (int j = 0; j < QA; ++j)
      if (lane + 64 * j < mk) sa[d][j] = pa[64 * j];
#pragma unroll
    for (int j = 0; j < QB; ++j)
      if (lane + 64 * j < kn) sb[d][j] = pb[64 * j];
  };

  // the product in the stage: its packed word
  int32_t stw = 0;
  auto stage_write = [&](auto slot) {
    constexpr int d = decltype(slot)::value;
    stw = sw[d];
    const int32_t m = stw & 31, n = (stw >> 5) & 31, k = (stw >> 10) & 31;
    if (k == 0) return;
    const int32_t kpad = (k + 7) & ~7;
    // element e of A (row-major m x k) is (e / k, e % k), of B (k x n) is
    // (e / n, e % n): for e < 256 and divisors up to 16 the quotient is
    // (e * ceil(2^16 / x)) >> 16 exactly
    const uint32_t ik = kInv16[k], in = kInv16[n];
    const int32_t mk = m * k, kn = k * n;
#pragma unroll
    for (int j = 0; j < QA; ++j) {
      const int32_t e = lane + 64 * j;
      if (e < mk) {
        const int32_t r = (int32_t)(((uint32_t)e * ik) >> 16);
        As[r * kMmaS + (e - r * k)] = sa[d][j];
      }
    }
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      const int32_t e = lane + 64 * j;
      if (e < kn) {
        const int32_t t = (int32_t)(((uint32_t)e * in) >> 16);
        Bs[(e - t * n) * kMmaS + t] = sb[d][j];
      }
    }
    // zero pads k .. kpad-1 of every A row and every B^T row (at most 7 each)
#pragma unroll
    for (int j = 0; j < (MP * 8 + 63) / 64; ++j) {
      const int32_t q = lane + 64 * j, r = q >> 3, t = k + (q & 7);
      if (r < MP && t < kpad) As[r * kMmaS + t] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < (NP * 8 + 63) / 64; ++j) {
      const int32_t q = lane + 64 * j, c = q >> 3, t = k + (q & 7);
      if (c < NP && t < kpad) Bs[c * kMmaS + t] = 0.0;
    }
  };

  double acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = 0.0;
  auto compute = [&]() {
    const int32_t k = (stw >> 10) & 31;
    const int32_t npair = (k + 7) >> 3;  // 0, 1 or 2
    // the B tile column of a lane is the same in every group (4g + b mod TN = b mod TN)
    const double* const bp = Bs + (4 * (bq % TN) + iq) * kMmaS + 2 * kk;
    for (int32_t kp = 0; kp < npair; ++kp) {
      const double2 bv = *reinterpret_cast<const double2*>(bp + 8 * kp);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int bi = (4 * g + bq) / TN;
        const double2 av = *reinterpret_cast<const double2*>(As + (4 * bi + iq) * kMmaS + 8 * kp + 2 * kk);
        acc[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(av.x, bv.x, acc[g], 0, 0, 0);
        acc[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(av.y, bv.y, acc[g], 0, 0, 0);
      }
    }
  };

  // Finish the C block of the product just multiplied: item g of lane
  // 16i + 4b + j is C(4 bi + i, 4 bj + j) of tile 4g + b.
  auto finish = [&]() {
    const int r = fr & 63;
    ++fr;
    const int32_t mn = __builtin_amdgcn_readlane(fifo_mn, r);
    const int32_t m = mn & 255, n = mn >> 8;
    const int64_t coff = make64(__builtin_amdgcn_readlane(fifo_co0, r), __builtin_amdgcn_readlane(fifo_co1, r));
    const int64_t oo = make64(__builtin_amdgcn_readlane(fifo_oo0, r), __builtin_amdgcn_readlane(fifo_oo1, r));
    double* const out = P.Cv + coff;
    const double* const ov = P.Ov + (oo >= 0 ? oo : 0);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int tau = 4 * g + bq;
      const int R = 4 * (tau / TN) + kk, Cc = 4 * (tau % TN) + iq;
      if (R < m && Cc < n) {
        double v = P.alpha * acc[g];
        if (oo >= 0) v += P.beta * ov[R * n + Cc];
        out[R * n + Cc] = v;
      }
      acc[g] = 0.0;
    }
  };

  // Prime: slots 0..D-1.  Step i (slot i mod D): write the slot into the
  // stage, refill it with product i+D, multiply; finish the C block if the
  // product ends it.
  static_for<0, D>([&](auto d) { fetch(d); });
  bool more = true;
  while (more) {
    static_for<0, D>([&](auto idx) {
      if (!more) return;
      if (!((sw[decltype(idx)::value] >> 15) & 1)) {
        more = false;
        return;
      }
      wave_sync();
      stage_write(idx);
      fetch(idx);
      wave_sync();
      compute();
      if ((stw >> 16) & 1) finish();
    });
  }
}

// The same launch with every class in the matrix-core form, D products in flight.
template <int D>
__global__ __launch_bounds__(256, 4) void k_numeric_small_mma(const double* __restrict__ Av,
                                                            const double* __restrict__ Bv,
                                                            const double* __restrict__ Ov,
                                                            const int4* __restrict__ list,
                                                            const int32_t* __restrict__ cls_start,
                                                            const int64_t* __restrict__ qstart,
                                                            const int4* __restrict__ desc, double* __restrict__ Cv,
                                                            double alpha, double beta, int32_t mask) {
  __shared__ __align__(16) double lds[4][2 * kStage];
  const SmallOps P{Av, Bv, Ov, list, qstart, desc, Cv, alpha, beta};
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t xcd = blockIdx.x % kXcds;
  const int32_t wpx = (int32_t)(gridDim.x / kXcds) * 4;
  const int32_t wix = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x / kXcds) * 4 + wv);
  double* wl = &lds[wv][0];
  for (int x = lane; x < 2 * kStage; x += 64) wl[x] = 0.0;  // stale rows stay finite
  wave_sync();
  int32_t b[5];
#pragma unroll
  for (int x = 0; x < 5; ++x) b[x] = cls_start[x];
  if (mask & 1) small_mfma<8, 8, D>(P, wl, b[0], b[1], xcd, wpx, wix, lane);
  if (mask & 2) small_mfma<8, 16, D>(P, wl, b[1], b[2], xcd, wpx, wix, lane);
  if (mask & 4) small_mfma<16, 8, D>(P, wl, b[2], b[3], xcd, wpx, wix, lane);
  if (mask & 8) small_mfma<16, 16, D>(P, wl, b[3], b[4], xcd, wpx, wix, lane);
}

// One persistent launch over every class: each wave runs its share of the
// classes selected by `mask` (bit c = class c) in turn.  D0, D1, D2 are the
// products in flight of the 8x8, 8x16 and 16x8 classes (16x16 always holds 2:
// four 16x16 slots do not fit beside its accumulators); 1 selects the form
// with several products per step (four for 8x8, two for 8x16 and 16x8), and
// D0 = 8 two steps of four 8x8 products for block edges of at most 8.
template <int D0, int D1, int D2>
__global__ __launch_bounds__(256, 4) void k_numeric_small(const double* __restrict__ Av, const double* __restrict__ Bv,
                                                       const double* __restrict__ Ov, const int4* __restrict__ list,
                                                       const int32_t* __restrict__ cls_start,
                                                       const int64_t* __restrict__ qstart,
                                                       const int4* __restrict__ desc, double* __restrict__ Cv,
                                                       double alpha, double beta, int32_t mask) {
  __shared__ __align__(16) double lds[4][2 * kStage];
  const SmallOps P{Av, Bv, Ov, list, qstart, desc, Cv, alpha, beta};
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t xcd = blockIdx.x % kXcds;
  const int32_t wpx = (int32_t)(gridDim.x / kXcds) * 4;
  const int32_t wix = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x / kXcds) * 4 + wv);
  double* wl = &lds[wv][0];
  int32_t b[5];
#pragma unroll
  for (int x = 0; x < 5; ++x) b[x] = cls_start[x];
  if (mask & 1) {
    if constexpr (D0 == 1)
      small_multi<8, 8, 4, 1>(P, wl, b[0], b[1], xcd, wpx, wix, lane);
    else if constexpr (D0 == 8)
      small_multi<8, 8, 4, 2, 8>(P, wl, b[0], b[1], xcd, wpx, wix, lane);
    else
      small_class<8, 8, D0>(P, wl, b[0], b[1], xcd, wpx, wix, lane);
  }
  if (mask & 2) {
    if constexpr (D1 == 1)
      small_multi<8, 16, 2, 1>(P, wl, b[1], b[2], xcd, wpx, wix, lane);
    else
      small_class<8, 16, D1>(P, wl, b[1], b[2], xcd, wpx, wix, lane);
  }
  if (mask & 4) {
    if constexpr (D2 == 1)
      small_multi<16, 8, 2, 1>(P, wl, b[2], b[3], xcd, wpx, wix, lane);
    else
      small_class<16, 8, D2>(P, wl, b[2], b[3], xcd, wpx, wix, lane);
  }
  if (mask & 8) small_class<16, 16, 2>(P, wl, b[3], b[4], xcd, wpx, wix, lane);
}


}  // namespace

// Grid of the numeric kernel: four workgroups of 4 waves per CU, a multiple
// of the XCD count; the list layout depends on its waves per XCD.
int32_t small_grid() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return ((cus * 4 + kXcds - 1) / kXcds) * kXcds;
}

int32_t small_waves_per_xcd() { return small_grid() / kXcds * 4; }

int64_t class_entries(int64_t nnzc_bound) {
  return (nnzc_bound + kClassChunk - 1) / kClassChunk * kClassChunk;
}

int64_t class_list_tmp_elems(int64_t nnzc_bound) {
  const int64_t nchunks = (nnzc_bound + kClassChunk - 1) / kClassChunk;
  return 4 * nchunks + 1;
}

hipError_t launch_class_lists(const NumArgs& a, int64_t* cnt, int64_t* cnt_pre, int64_t* tmp, int4* list,
                              int32_t* cls_start, int64_t* cnp, int64_t* qstart, int4* desc, hipStream_t s) {
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
                     a.use_old, cnt_pre, list, cls_start, cnp, small_waves_per_xcd());
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive(cnp, (int64_t)nchunks * kClassChunk, qstart, tmp, s);
  if (e != hipSuccess) return e;
  int64_t blocks = (a.nnzc_bound + 15) / 16;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_class_desc, dim3((uint32_t)blocks), dim3(256), 0, s, a.totals, list, qstart, a.prod, a.A.blk_off, a.B.blk_off, (int32_t)a.uniform, desc);
  return hipGetLastError();
}

// Compiled pipeline variants, indexed by the tuner's variant number.
using SmallKernel = void (*)(const double*, const double*, const double*, const int4*, const int32_t*,
                            const int64_t*, const int4*, double*, double, double, int32_t);
constexpr SmallKernel kSmallKernels[] = {k_numeric_small<1, 1, 1>, k_numeric_small<1, 2, 2>, k_numeric_small<4, 2, 2>,
                                         k_numeric_small<1, 1, 2>, k_numeric_small<1, 2, 1>, k_numeric_small<8, 2, 2>,
                                         k_numeric_small_mma<2>,   k_numeric_small_mma<3>};

constexpr int kSmallDepths[][4] = {{1, 1, 1, 2}, {1, 2, 2, 2}, {4, 2, 2, 2}, {1, 1, 2, 2},
                                   {1, 2, 1, 2}, {8, 2, 2, 2}, {18, 18, 18, 18}, {19, 19, 19, 19}};
static_assert(sizeof(kSmallKernels) / sizeof(kSmallKernels[0]) == kSmallVariants, "variant table");
static_assert(sizeof(kSmallDepths) / sizeof(kSmallDepths[0]) == kSmallVariants, "variant table");

int32_t small_variant_max_edge(int32_t v) { return v >= 0 && v < kSmallVariants && kSmallDepths[v][0] == 8 ? 8 : 16; }

void small_variant_depths(int32_t v, int32_t* depths) {
  for (int c = 0; c < 4; ++c) depths[c] = (v >= 0 && v < kSmallVariants) ? kSmallDepths[v][c] : 0;
}

hipError_t launch_numeric_small(const NumArgs& a, const int4* list, const int32_t* cls_start, const int64_t* qstart,
                                const int4* desc, int32_t variant, int32_t mask, hipStream_t s) {
  if (a.nnzc_bound <= 0) return hipSuccess;
  if (variant < 0 || variant >= kSmallVariants) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kSmallKernels[variant], dim3(small_grid()), dim3(256), 0, s, a.A.values, a.B.values,
                     a.use_old ? a.Cin.values : a.c_values, list, cls_start, qstart, desc, a.c_values, a.alpha,
                     a.beta, mask & kSmallAllClasses);
  return hipGetLastError();
}

}  // namespace bsmm
