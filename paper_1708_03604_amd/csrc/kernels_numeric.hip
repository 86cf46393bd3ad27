// Numeric phase: for every C block (i,j), acc = sum over its kept products
// A(i,k) * B(k,j) (in stack order, i.e. ascending k), then
// C(i,j) = alpha*acc + beta*C_in(i,j) (Section 2 of the paper: the local
// multiply is a sum of pairwise products of (m x k) and (k x n) blocks).
//
// Each C block is owned by exactly one wave, so no floating-point atomics are
// used and the result does not depend on the schedule.
#include <type_traits>

#include "bsmm_internal.h"

namespace bsmm {

// ---------------------------------------------------------------------------
// Any block sizes (the path for blocks that are neither all <= 16 nor all
// 23x23): one wave per C block at a time.  The C block is cut into square
// sub-tiles of edge T (32, or 16 where the tile policy asks for it) and every
// product into K chunks of at most 32; a sub-tile is accumulated in registers
// over all chunks of all products of its C block.
//
// C_in prefetch (g.mid_cpre, also chosen by the autotuner): the C_in values of
// a sub-tile are loaded before its last chunk is multiplied (faster where C
// blocks have few products, slower where the loop's registers matter more).
//
// Tile policy (g.mid_t16, chosen by the autotuner per set of block edges):
// 0 = every C block in 32x32 sub-tiles; 1 = a C block with both edges <= 16
// (e.g. 9x9 beside 22- and 32-edge blocks) is one 16x16 sub-tile, in the
// vector form, lane 8*ty + tx owning rows 2ty, 2ty+1 and columns 2tx, 2tx+1,
// with half the operand loads per chunk and a quarter of the FMAs.  (Cutting
// larger blocks into 16x16 sub-tiles too, wherever that pads less, measured
// slower: every extra sub-tile walks the block's products again.)  Both sizes
// sum every output over the same inner indices in the same order with the
// same FMAs, so the vector form gives the same bits with either.
//
// A chunk is staged through wave-private LDS with a row stride of kMidStride
// doubles, zeros past the block and the chunk; the loads of the next chunk
// are issued before the current chunk is multiplied.  Two forms multiply a
// staged chunk, chosen per C block; both keep the sub-tile's 16 values per
// lane in the same registers:
//   - C blocks with both edges >= 16, in multiplies whose inner block edges
//     are all >= 16: FP64 matrix cores, v_mfma_f64_4x4x4_4b
//     as in the 23x23 kernel (lane 16k + 4b + i holds A_b[i][k] and B_b[k][i],
//     result lane 16i + 4b + j holds D_b[i][j]).  The sub-tile is a 4x4 grid of
//     8x8 super-tiles, each the 2x2 tiles of one instruction, one accumulator
//     per super-tile; the inner index runs in pairs (slot k: t = 8p + 2k and
//     t + 1), so A is staged as stored and B transposed and one 16-byte read
//     gives a lane the operands of two instructions: per 8 inner indices,
//     eight reads and 32 instructions.
//     (The inner index is padded to a multiple of 8 there, while the vector
//     form runs exactly k steps: with narrow inner blocks it is the faster.)
//   - otherwise FP64 vector FMA, A staged transposed (row t holds A(r, k0+t))
//     and B as is: lane l = 8*ty + tx owns sub-tile rows 4ty..4ty+3 and
//     columns 4tx..4tx+3 and reads its 4 A values and 4 B values of inner
//     index t with two 16-byte loads each.
// ---------------------------------------------------------------------------
constexpr int kMid = 32;
constexpr int kMidStride = 34;  // doubles per LDS row: 16-byte aligned rows, 2-way write conflicts at most
constexpr int kMidOperand = kMid * kMidStride;

// Position of a wave in its chunk sequence: C block c, sub-tile (ti, tj),
// product x in [x0, x1), K chunk k0 of the product's inner size k.
struct MidCursor {
  int32_t c, m, n, t, ti, tj, nti, ntj, k, k0;
  int64_t x, x0, x1, aoff, boff;
  bool valid;
};

__device__ __forceinline__ void mid_product(const NumArgs& g, MidCursor& u) {
  if (u.x < u.x1) {
    const int2 ab = g.prod[u.x];
    const int32_t a = ab.x;
    const int64_t a0 = g.A.blk_off[a], a1 = g.A.blk_off[a + 1];
    u.aoff = a0;
    u.boff = g.B.blk_off[ab.y];
    u.k = (int32_t)((uint32_t)(a1 - a0) / (uint32_t)u.m);
  } else {
    u.k = 0;  // C block without products: one empty chunk finishes each sub-tile
  }
  u.k0 = 0;
}

__device__ __forceinline__ void mid_block(const NumArgs& g, MidCursor& u, int32_t nnzc) {
  u.valid = u.c < nnzc;
  if (!u.valid) return;
  const int64_t off = g.c_blk_off[u.c];
  u.n = g.c_col_sizes[g.c_col_idx[u.c]];
  u.m = (int32_t)((uint32_t)(g.c_blk_off[u.c + 1] - off) / (uint32_t)u.n);
  u.t = (g.mid_t16 && u.m <= 16 && u.n <= 16) ? 16 : kMid;
  u.nti = (u.m + u.t - 1) / u.t;
  u.ntj = (u.n + u.t - 1) / u.t;
  u.ti = 0;
  u.tj = 0;
  u.x0 = g.prod_ptr[u.c];
  u.x1 = g.prod_ptr[u.c + 1];
  u.x = u.x0;
  mid_product(g, u);
}

// Advance to the next chunk; returns true if the chunk just left was the
// last one of its sub-tile.
__device__ __forceinline__ bool mid_next(const NumArgs& g, MidCursor& u, int32_t nnzc, int32_t nwaves) {
  u.k0 += kMid;
  if (u.k0 < u.k) return false;
  if (u.x < u.x1) ++u.x;
  if (u.x < u.x1) {
    mid_product(g, u);
    return false;
  }
  if (++u.tj == u.ntj) {
    u.tj = 0;
    ++u.ti;
  }
  if (u.ti < u.nti) {
    u.x = u.x0;
    mid_product(g, u);
    return true;
  }
  u.c += nwaves;
  mid_block(g, u, nnzc);
  return true;
}

// WIDE: every inner block edge is >= 16 (the matrix-core form may run); the
// other instantiation is the vector form alone.
template <bool WIDE, bool CPRE>
__global__ __launch_bounds__(256, 2) void k_numeric_mid(NumArgs g) {
  __shared__ __align__(16) double lds[4][2 * kMidOperand];  // per wave: A^T, then B
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ty = lane >> 3, tx = lane & 7;
  const int lc = lane & 31, lr = lane >> 5;  // staging: column lc of rows lr, lr+2, ..., lr+30
  double* const As = &lds[wv][0];
  double* const Bs = &lds[wv][kMidOperand];
  const int32_t nnzc = live_nnzc(g.totals);
  const int32_t nwaves = gridDim.x * 4;

  MidCursor f;  // fetch cursor, one chunk ahead of the compute cursor
  f.c = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);
  mid_block(g, f, nnzc);
  if (!f.valid) return;

  // Operand registers of the chunk in flight, zero outside the block and the
  // chunk: with 32x32 sub-tiles A(32ti + lr + 2v, k0 + lc) and
  // B(k0 + lr + 2v, 32tj + lc), v < 16; with 16x16 sub-tiles
  // A(16ti + lr + 2v, k0 + lc) and B(k0 + br + 4v, 16tj + bc), v < 8.
  double ra[16], rb[16];
  const int bc = lane & 15, br = lane >> 4;
  auto fetch = [&](const MidCursor& u) {
    const int kk = min(kMid, u.k - u.k0);
    const int mm = min(u.t, u.m - u.t * u.ti), nn = min(u.t, u.n - u.t * u.tj);
    if (u.t == 16) {
      const double* ap = g.A.values + u.aoff + (int64_t)(16 * u.ti + lr) * u.k + u.k0 + lc;
      const double* bp = g.B.values + u.boff + (int64_t)(u.k0 + br) * u.n + 16 * u.tj + bc;
      const bool acol = lc < kk, bcol = bc < nn;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int r = lr + 2 * v;
        ra[v] = (acol && r < mm) ? ap[(int64_t)2 * v * u.k] : 0.0;
        rb[v] = (bcol && br + 4 * v < kk) ? bp[(int64_t)4 * v * u.n] : 0.0;
      }
      return;
    }
    const double* ap = g.A.values + u.aoff + (int64_t)(u.t * u.ti + lr) * u.k + u.k0 + lc;
    const double* bp = g.B.values + u.boff + (int64_t)(u.k0 + lr) * u.n + u.t * u.tj + lc;
    const bool acol = lc < kk, bcol = lc < nn;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = lr + 2 * v;
      ra[v] = (acol && r < mm) ? ap[(int64_t)2 * v * u.k] : 0.0;
      rb[v] = (bcol && r < kk) ? bp[(int64_t)2 * v * u.n] : 0.0;
    }
  };
  auto stage = [&](bool mma, bool t16) {
    if (t16) {
      // B first: were the A stores (the vector form's first eight) first,
      // the compiler would merge the two loops into one of run-time length
      // and keep ra in scratch memory
#pragma unroll
      for (int v = 0; v < 8; ++v) Bs[(br + 4 * v) * kMidStride + bc] = rb[v];
#pragma unroll
      for (int v = 0; v < 8; ++v) As[lc * kMidStride + lr + 2 * v] = ra[v];
    } else if (mma) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        As[(lr + 2 * v) * kMidStride + lc] = ra[v];
        Bs[lc * kMidStride + lr + 2 * v] = rb[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        As[lc * kMidStride + lr + 2 * v] = ra[v];
        Bs[(lr + 2 * v) * kMidStride + lc] = rb[v];
      }
    }
  };
  auto sync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  fetch(f);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (;;) {
    // the chunk to multiply now is the one the fetch cursor points at
    const MidCursor cur = f;
    const bool mma = WIDE && cur.t == kMid && cur.m >= 16 && cur.n >= 16;  // uniform over the wave
    const bool t16 = cur.t == 16;
    sync();
    stage(mma, t16);
    sync();
    const bool last = mid_next(g, f, nnzc, nwaves);
    // CPRE: the sub-tile ends with this chunk, so load its C_in values now,
    // before the next chunk's operand loads: they arrive during the multiply,
    // and waiting for them at the finish does not wait for the operand loads
    // (the form without it keeps fewer registers live through the loop).
    double cin[4][4];
    if (CPRE && last) {
      const int32_t o = g.use_old ? g.c_old_idx[cur.c] : -1;
      const double* ov = o >= 0 ? g.Cin.values + g.Cin.blk_off[o] : nullptr;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // matrix-core form: lane 16k + 4b + i' holds row 8I + 4(b >> 1) + k,
          // column 8J + 4(b & 1) + i' of super-tile (I, J) = (i, j)
          const int r = cur.t * cur.ti + (mma ? 8 * i + 4 * ((lane >> 3) & 1) + (lane >> 4) : t16 ? 2 * ty + i : 4 * ty + i);
          const int cc = cur.t * cur.tj + (mma ? 8 * j + 4 * ((lane >> 2) & 1) + (lane & 3) : t16 ? 2 * tx + j : 4 * tx + j);
          const bool in = (!t16 || (i < 2 && j < 2)) && r < cur.m && cc < cur.n;
          cin[i][j] = (ov && in) ? ov[(int64_t)r * cur.n + cc] : 0.0;
        }
    }
    if (f.valid) fetch(f);
    const int kk = max(0, min(kMid, cur.k - cur.k0));
    if (mma) {
      // acc[I][J]: super-tile (I, J); fragment lane roles as in the 23x23 kernel
      const int fk = lane >> 4, fb = (lane >> 2) & 3, fi = lane & 3;
      const double* ap = As + (4 * (fb >> 1) + fi) * kMidStride + 2 * fk;
      const double* bp = Bs + (4 * (fb & 1) + fi) * kMidStride + 2 * fk;
      for (int kp = 0; kp < (kk + 7) >> 3; ++kp) {
        double2 a[4], b[4];
#pragma unroll
        for (int I = 0; I < 4; ++I) a[I] = *reinterpret_cast<const double2*>(ap + 8 * I * kMidStride + 8 * kp);
#pragma unroll
        for (int J = 0; J < 4; ++J) b[J] = *reinterpret_cast<const double2*>(bp + 8 * J * kMidStride + 8 * kp);
#pragma unroll
        for (int I = 0; I < 4; ++I)
#pragma unroll
          for (int J = 0; J < 4; ++J) acc[I][J] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[I].x, b[J].x, acc[I][J], 0, 0, 0);
#pragma unroll
        for (int I = 0; I < 4; ++I)
#pragma unroll
          for (int J = 0; J < 4; ++J) acc[I][J] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[I].y, b[J].y, acc[I][J], 0, 0, 0);
      }
    } else if (t16) {
      // 16x16 sub-tile: acc[i][j] for i, j < 2 (rows 2ty + i, columns 2tx + j)
      const double* ap = As + 2 * ty;
      const double* bp = Bs + 2 * tx;
#pragma unroll 4
      for (int t = 0; t < kk; ++t) {
        const double2 a = *reinterpret_cast<const double2*>(ap + t * kMidStride);
        const double2 b = *reinterpret_cast<const double2*>(bp + t * kMidStride);
        acc[0][0] = fma(a.x, b.x, acc[0][0]);
        acc[0][1] = fma(a.x, b.y, acc[0][1]);
        acc[1][0] = fma(a.y, b.x, acc[1][0]);
        acc[1][1] = fma(a.y, b.y, acc[1][1]);
      }
    } else {
      const double* ap = As + 4 * ty;
      const double* bp = Bs + 4 * tx;
#pragma unroll 4
      for (int t = 0; t < kk; ++t) {
        const double2 a01 = *reinterpret_cast<const double2*>(ap + t * kMidStride);
        const double2 a23 = *reinterpret_cast<const double2*>(ap + t * kMidStride + 2);
        const double2 b01 = *reinterpret_cast<const double2*>(bp + t * kMidStride);
        const double2 b23 = *reinterpret_cast<const double2*>(bp + t * kMidStride + 2);
        const double a[4] = {a01.x, a01.y, a23.x, a23.y};
        const double b[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
      }
    }
    if (last) {
      // alpha * acc + beta * C_in, then store the lane's 16 outputs
      const int64_t off = g.c_blk_off[cur.c];
      const int32_t o = g.use_old ? g.c_old_idx[cur.c] : -1;
      const double* ov = o >= 0 ? g.Cin.values + g.Cin.blk_off[o] : nullptr;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = cur.t * cur.ti + (mma ? 8 * i + 4 * ((lane >> 3) & 1) + (lane >> 4) : t16 ? 2 * ty + i : 4 * ty + i);
          const int cc = cur.t * cur.tj + (mma ? 8 * j + 4 * ((lane >> 2) & 1) + (lane & 3) : t16 ? 2 * tx + j : 4 * tx + j);
          if ((!t16 || (i < 2 && j < 2)) && r < cur.m && cc < cur.n) {
            const int64_t e = (int64_t)r * cur.n + cc;
            double v = g.alpha * acc[i][j];
            if (ov) v = v + g.beta * (CPRE ? cin[i][j] : ov[e]);
            g.c_values[off + e] = v;
          }
          acc[i][j] = 0.0;
        }
      }
    }
    if (!f.valid) break;
  }
}

// ---------------------------------------------------------------------------
// Square blocks of edge S in [17, 24] (the 23x23 molecule blocks), padded to
// a 24x24 tile.
// ---------------------------------------------------------------------------
constexpr int kTileEdge = 24;

// For each of three targets t, the first c in [lo, hi] with prod_ptr[c] >= t
// (prod_ptr is non-decreasing), hi if there is none: a branchless search
// whose step count depends only on hi - lo, so the three loads of each step
// are in flight together (the schedule pass is bound by these dependent
// loads, not by arithmetic).
__device__ __forceinline__ void lower_bound_c3(const int64_t* __restrict__ prod_ptr, int32_t lo, int32_t hi,
                                               const int64_t (&t)[3], int32_t (&r)[3]) {
  int32_t b[3] = {lo, lo, lo};
  if (hi > lo) {
    int32_t n = hi - lo;
    while (n > 1) {  // invariant: the answer lies in [b, b + n]
      const int32_t half = n >> 1;
      int64_t v[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) v[s] = prod_ptr[b[s] + half];
#pragma unroll
      for (int s = 0; s < 3; ++s) b[s] = v[s] < t[s] ? b[s] + half : b[s];
      n -= half;
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) b[s] += prod_ptr[b[s]] < t[s] ? 1 : 0;
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) r[s] = b[s];
}

// Schedule of the 23x23 kernels: the C blocks [c0, c1) of the panel (all
// blocks without panels) are cut into 8 XCD parts of equal product counts
// (XCD x: products [P x / 8, P (x+1) / 8) of the panel's P), and each part
// into ns slices of equal product counts, cut at C block boundaries:
// bounds[x (ns+1) + j] is the first C block of slice j of part x.  Waves
// take every wpx-th slice of their XCD's part, so each wave gets about the
// same number of products while an XCD still works on nearby block rows.
// The panel's first stack position follows the bounds (slices_pbase).
constexpr int kKernelXcds = kSliceParts;
constexpr int kSlicesPerWave = 16;  // measured: 8 1.63 ms, 16 1.60, 32 1.65, 64 1.76 (molecules)
__global__ void k_product_slices(const int64_t* __restrict__ prod_ptr, const int64_t* __restrict__ totals,
                                 const int32_t* __restrict__ c_row_ptr, const int32_t* __restrict__ panel, int32_t ns,
                                 int32_t* __restrict__ bounds) {
  const int32_t nnzc = live_nnzc(totals);
  int32_t c0 = 0, c1 = nnzc;
  if (panel && nnzc > 0) {
    c0 = c_row_ptr[panel[0]];
    c1 = c_row_ptr[panel[1]];
  }
  const int64_t pb = nnzc > 0 ? prod_ptr[c0] : 0;
  const int64_t P = nnzc > 0 ? prod_ptr[c1] - pb : 0;
  const int32_t per = ns + 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) *reinterpret_cast<int64_t*>(bounds + kKernelXcds * per) = pb;
  for (int32_t t = blockIdx.x * 256 + threadIdx.x; t < kKernelXcds * per; t += gridDim.x * 256) {
    const int32_t x = t / per, j = t - x * per;
    const int64_t p0 = pb + P * x / kKernelXcds, p1 = pb + P * (x + 1) / kKernelXcds;
    const int64_t tg[3] = {p0, p1, p0 + (p1 - p0) * j / ns};
    int32_t r[3];
    lower_bound_c3(prod_ptr, c0, c1, tg, r);
    const int32_t X0 = x == 0 ? c0 : r[0];
    const int32_t X1 = x == kKernelXcds - 1 ? c1 : r[1];
    int32_t b;
    if (j == 0) b = X0;
    else if (j == ns) b = X1;
    else b = min(X1, max(X0, r[2]));
    bounds[t] = b;
  }
}

// ---------------------------------------------------------------------------
// Square blocks of edge S in [17, 24] on the FP64 matrix cores
// (v_mfma_f64_4x4x4_4b: four independent 4x4x4 products per instruction, which
// pad a 23-edge only to 24).  One wave per C block at a time; the product
// stack is one flat array ordered by C block: each XCD (workgroup b runs on
// XCD b mod 8) owns a contiguous run of C blocks with 1/8 of the products, cut
// into slices of equal product counts (k_product_slices); its waves take every
// wpx-th slice and walk their products as one stream (operands of the next
// product in registers, two LDS stages).
//
// Instruction layout (measured on the device): lane 16k + 4b + i holds
// A_b[i][k] and B_b[k][i'] with i' = i, and the result lane 16i + 4b + j holds
// D_b[i][j].  The 24x24 C block is a 3x3 grid of 8x8 super-tiles, each the
// 2x2 tiles b = 2*bi + bj of one instruction, so a lane keeps one FP64
// accumulator per super-tile (9 in all).  The inner index runs in pairs: the
// two instructions of K step kp use t = 8kp + 2k and t = 8kp + 2k + 1 in slot
// k, so one 16-byte LDS read gives a lane both: A is staged as stored and B
// transposed, both with row stride 26 doubles (16-byte aligned rows, and the
// eight rows one read touches fall on distinct banks).  Pads (row/column 23,
// inner index 23) stay zero.  54 instructions per product.
// ---------------------------------------------------------------------------
constexpr int kMfmaStride = 26;
constexpr int kMfmaOperand = kTileEdge * kMfmaStride;

template <int S>
__global__ __launch_bounds__(256, 2) void k_numeric_mfma24(
    const double* __restrict__ Av, const double* __restrict__ Bv, const double* __restrict__ Ov,
    const int64_t* __restrict__ prod_ptr, const int2* __restrict__ prod,
    const int32_t* __restrict__ c_old_idx, double* __restrict__ Cv, const int64_t* __restrict__ totals, int use_old,
    double alpha, double beta, const int32_t* __restrict__ bounds, int32_t ns) {
  static_assert(S >= 17 && S <= kTileEdge, "matrix-core kernel covers edges 17..24");
  constexpr int NE = S * S;
  constexpr int PER = (NE + 63) / 64;
  constexpr int LAST = NE - 64 * (PER - 1);
  // per wave: two stages, each A then B^T
  __shared__ __align__(16) double lds[4][2][2 * kMfmaOperand];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int x = lane; x < 4 * kMfmaOperand; x += 64) (&lds[wv][0][0])[x] = 0.0;

  // LDS offset (doubles, within a stage) of element e = lane + 64u of a
  // product: A as stored, B transposed
  int offA[PER], offB[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (u < PER - 1 || lane < LAST) ? lane + 64 * u : 0;
    const int r = e / S, c = e - r * S;
    offA[u] = r * kMfmaStride + c;
    offB[u] = kMfmaOperand + c * kMfmaStride + r;
  }
  const bool tail = lane < LAST;
  // fragment reads: slot k = lane >> 4, tile b = (lane >> 2) & 3, row/column
  // i = lane & 3 of the tile; super-tile (I, J) and K step kp add constants
  const int fk = lane >> 4, fb = (lane >> 2) & 3, fi = lane & 3;
  const int afrag = (4 * (fb >> 1) + fi) * kMfmaStride + 2 * fk;
  const int bfrag = kMfmaOperand + (4 * (fb & 1) + fi) * kMfmaStride + 2 * fk;

  const int32_t xcd = blockIdx.x % kKernelXcds;
  const int32_t wpx = (int32_t)(gridDim.x / kKernelXcds) * 4;  // waves per XCD
  const int32_t wix = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x / kKernelXcds) * 4 + wv);
  const int32_t nnzc = live_nnzc(totals);
  if (nnzc == 0) return;
  const int32_t* const bnd = bounds + xcd * (ns + 1);
  const int64_t pbase = slices_pbase(bounds, ns);  // stack position of prod[0]

  // fetch cursor: slice iq, products [ip, ip_end)
  int32_t iq = wix;
  int64_t ip = 0, ip_end = 0;
  if (iq < ns) {
    ip = prod_ptr[bnd[iq]];
    ip_end = prod_ptr[bnd[iq + 1]];
  }
  auto next_index = [&]() -> int64_t {
    while (ip >= ip_end) {
      iq += wpx;
      if (iq >= ns) return -1;
      ip = prod_ptr[bnd[iq]];
      ip_end = prod_ptr[bnd[iq + 1]];
    }
    return ip++;
  };
  int32_t qa0 = -1, qb0 = -1, qa1 = -1, qb1 = -1;
  {
    const int64_t n0 = next_index();
    if (n0 >= 0) {
      const int2 e0 = prod[n0 - pbase];
      qa0 = e0.x;
      qb0 = e0.y;
    }
    const int64_t n1 = next_index();
    if (n1 >= 0) {
      const int2 e1 = prod[n1 - pbase];
      qa1 = e1.x;
      qb1 = e1.y;
    }
  }
  double opa[PER], opb[PER];
  auto fetch_next = [&]() {
    if (qa0 >= 0) {
      const double* Ab = Av + (int64_t)qa0 * NE + lane;
      const double* Bb = Bv + (int64_t)qb0 * NE + lane;
#pragma unroll
      for (int u = 0; u < PER - 1; ++u) {
        opa[u] = Ab[64 * u];
        opb[u] = Bb[64 * u];
      }
      opa[PER - 1] = tail ? Ab[64 * (PER - 1)] : 0.0;
      opb[PER - 1] = tail ? Bb[64 * (PER - 1)] : 0.0;
    }
    qa0 = qa1;
    qb0 = qb1;
    const int64_t n = next_index();
    const int2 e = n >= 0 ? prod[n - pbase] : make_int2(-1, -1);
    qa1 = e.x;
    qb1 = e.y;
  };
  auto stage_write = [&](const int st) {
    double* base = &lds[wv][st][0];
#pragma unroll
    for (int u = 0; u < PER - 1; ++u) {
      base[offA[u]] = opa[u];
      base[offB[u]] = opb[u];
    }
    if (tail) {
      base[offA[PER - 1]] = opa[PER - 1];
      base[offB[PER - 1]] = opb[PER - 1];
    }
  };

  const bool any = qa0 >= 0;
  if (any) {
    fetch_next();
    stage_write(0);
    fetch_next();
  }
  double acc[3][3];
  auto step = [&](auto stage) {
    constexpr int st = decltype(stage)::value;
    // the staging and the next loads at raised issue priority, so that they
    // go out while the other wave on the SIMD runs its matrix instructions
    // (measured: 1.597 -> 1.583 ms; raising it around the MFMAs instead was
    // slower)
    __builtin_amdgcn_s_setprio(1);
    stage_write(st ^ 1);
    fetch_next();
    __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double* base = &lds[wv][st][0];
#pragma unroll
    for (int kp = 0; kp < 3; ++kp) {
      double2 a[3], b[3];
#pragma unroll
      for (int I = 0; I < 3; ++I) a[I] = *reinterpret_cast<const double2*>(base + afrag + 8 * I * kMfmaStride + 8 * kp);
#pragma unroll
      for (int J = 0; J < 3; ++J) b[J] = *reinterpret_cast<const double2*>(base + bfrag + 8 * J * kMfmaStride + 8 * kp);
#pragma unroll
      for (int I = 0; I < 3; ++I)
#pragma unroll
        for (int J = 0; J < 3; ++J) acc[I][J] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[I].x, b[J].x, acc[I][J], 0, 0, 0);
#pragma unroll
      for (int I = 0; I < 3; ++I)
#pragma unroll
        for (int J = 0; J < 3; ++J) acc[I][J] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[I].y, b[J].y, acc[I][J], 0, 0, 0);
    }
  };

  // compute cursor: slice cq, C blocks [c, c1), products [p, pe) of block c
  int32_t cq = wix;
  int32_t c = 0, c1 = 0;
  int64_t p = 0, pe = 0;
  while (cq < ns && bnd[cq] == bnd[cq + 1]) cq += wpx;
  if (cq >= ns) return;
  c = bnd[cq];
  c1 = bnd[cq + 1];
  p = prod_ptr[c];
  pe = prod_ptr[c + 1];
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int J = 0; J < 3; ++J) acc[I][J] = 0.0;

  // this lane's result element of super-tile (I, J): row 8I + orow, column 8J + ocol
  const int orow = 4 * (fb >> 1) + fk, ocol = 4 * (fb & 1) + fi;
  // Finish every C block that ends at p: apply alpha, park the block
  // row-major in the free LDS stage, then add beta*C_in and store it with
  // contiguous accesses.  Returns false when the wave has no products left.
  auto advance = [&](auto freestage) -> bool {
    constexpr int fs = decltype(freestage)::value;
    double* const tile = &lds[wv][fs][0];
    while (p == pe) {
#pragma unroll
      for (int I = 0; I < 3; ++I)
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const int R = 8 * I + orow, Cc = 8 * J + ocol;
          if (R < S && Cc < S) tile[R * S + Cc] = alpha * acc[I][J];
        }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int32_t o = use_old ? c_old_idx[c] : -1;
      double* out = Cv + (int64_t)c * NE + lane;
      const double* tl = tile + lane;
      if (o >= 0) {
        const double* ov = Ov + (int64_t)o * NE + lane;
        double ol[PER];
#pragma unroll
        for (int u = 0; u < PER - 1; ++u) ol[u] = ov[64 * u];
        ol[PER - 1] = tail ? ov[64 * (PER - 1)] : 0.0;
#pragma unroll
        for (int u = 0; u < PER - 1; ++u) out[64 * u] = tl[64 * u] + beta * ol[u];
        if (tail) out[64 * (PER - 1)] = tl[64 * (PER - 1)] + beta * ol[PER - 1];
      } else {
#pragma unroll
        for (int u = 0; u < PER - 1; ++u) out[64 * u] = tl[64 * u];
        if (tail) out[64 * (PER - 1)] = tl[64 * (PER - 1)];
      }
      // the parked block overwrote some inner-index pads of the stage's A
      // operand (positions r*26 + t, t >= S, below S*S): restore their zeros
      // once every lane has read the parked block
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < kTileEdge) {
#pragma unroll
        for (int t = S; t < kTileEdge; ++t)
          if (lane * kMfmaStride + t < NE) tile[lane * kMfmaStride + t] = 0.0;
      }
#pragma unroll
      for (int I = 0; I < 3; ++I)
#pragma unroll
        for (int J = 0; J < 3; ++J) acc[I][J] = 0.0;
      ++c;
      if (c == c1) {
        do {
          cq += wpx;
          if (cq >= ns) return false;
        } while (bnd[cq] == bnd[cq + 1]);
        c = bnd[cq];
        c1 = bnd[cq + 1];
        p = prod_ptr[c];
      }
      pe = prod_ptr[c + 1];
    }
    return true;
  };

  for (;;) {
    if (p == pe && !advance(std::integral_constant<int, 1>())) break;
    step(std::integral_constant<int, 0>());
    ++p;
    if (p == pe && !advance(std::integral_constant<int, 0>())) break;
    step(std::integral_constant<int, 1>());
    ++p;
  }
}

// Grid of the 23x23 kernel: two workgroups of 4 waves per CU, a multiple of 8 (XCDs).
static int32_t tile23_grid() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return ((cus * 2 + kKernelXcds - 1) / kKernelXcds) * kKernelXcds;
}

int64_t numeric_work_elems() {
  const int64_t ns = (int64_t)tile23_grid() / kKernelXcds * 4 * kSlicesPerWave;
  return kKernelXcds * (ns + 1) + 2;  // bounds, then the int64 stack base (at byte 32 (ns + 1): aligned)
}

int32_t launch_product_slices(const int64_t* prod_ptr, const int64_t* totals, const int32_t* c_row_ptr,
                              const int32_t* panel, int32_t* work, hipStream_t s) {
  const int32_t ns = tile23_grid() / kKernelXcds * 4 * kSlicesPerWave;
  const int32_t n = kKernelXcds * (ns + 1);
  hipLaunchKernelGGL(k_product_slices, dim3((n + 255) / 256), dim3(256), 0, s, prod_ptr, totals, c_row_ptr, panel,
                     ns, work);
  return ns;
}

int32_t tile23_workgroups() { return tile23_grid(); }

hipError_t launch_numeric(const NumArgs& a, int uniform_size, int32_t* work, hipStream_t s) {
  if (a.nnzc_bound <= 0) return hipSuccess;
  if (uniform_size == 23) {
    const int32_t blocks = tile23_grid();
    const int32_t ns = launch_product_slices(a.prod_ptr, a.totals, a.c_row_ptr, a.panel, work, s);
    hipLaunchKernelGGL(k_numeric_mfma24<23>, dim3(blocks), dim3(256), 0, s, a.A.values, a.B.values,
                       a.use_old ? a.Cin.values : a.A.values, a.prod_ptr, a.prod, a.c_old_idx,
                       a.c_values, a.totals, a.use_old, a.alpha, a.beta, work, ns);
    return hipGetLastError();
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int64_t blocks = (a.nnzc_bound + 3) / 4;  // every wave owns at least one C block at the start
  if (blocks > 2 * cus) blocks = 2 * cus;   // two workgroups of 4 waves per CU stay resident
  if (a.wide_inner) {
    if (a.mid_cpre)
      hipLaunchKernelGGL((k_numeric_mid<true, true>), dim3((uint32_t)blocks), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_numeric_mid<true, false>), dim3((uint32_t)blocks), dim3(256), 0, s, a);
  } else {
    if (a.mid_cpre)
      hipLaunchKernelGGL((k_numeric_mid<false, true>), dim3((uint32_t)blocks), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_numeric_mid<false, false>), dim3((uint32_t)blocks), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace bsmm
