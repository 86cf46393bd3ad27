// Exact-slice (Ozaki-style) block products of 23x23 blocks on INT8 matrix
// cores, the accuracy-preserving alternative to the BF16 split.
//
// Scaling.  Every row r of block row i of A gets one power of two 2^ea(i,r)
// above the largest |A| in that row over all blocks of the block row; every
// column q of block column j of B gets 2^eb(j,q) the same way (the frexp
// exponent: max < 2^e <= 2*max).
//
// Slices.  A value x of such a row becomes y = x 2^-e in (-1, 1) and seven
// signed digits, taken by rounding to nearest: d1 = rint(64 y), then
// d(s+1) = rint(128 * remainder(s)), so that
//     y = sum_s d_s 2^-w_s + rho,  w_s = 6 + 7(s-1),  |d_s| <= 64,  |rho| <= 2^-49.
// Every step is exact in FP64.
//
// Products.  A block product keeps the slice products (s, t) with s + t <= 8:
// for each degree g = s + t the INT8 matrix core adds sum_c dA_s dB_t exactly
// into an INT32 accumulator I_g, over all products of the C block (the scales
// are shared by every product of a C block, so no conversion per product).
// At the end of the C block
//     C(r,q) = alpha * 2^(ea(i,r) + eb(j,q)) * sum_g I_g 2^-(12 + 7(g-2)) + beta * C_in(r,q),
// in FP64.  The dropped slice products and the remainders bound the error
// per C element by 2^-39 |alpha| n M_A(i,r) M_B(j,q) (n performed block
// products, M the row and column maxima above), plus FP64 rounding.
//
// Storage of the slices (per block, 3872 bytes, 16-byte aligned): 23 rows of
// 7 slices x 24 bytes (23 digits and a zero).  A is stored as is (row r holds
// A(r, :)), slices in the order 1..7; B transposed (row q holds B(:, q)),
// slices in the order 7..1.  In LDS each slice takes 32 bytes (bytes 24..31
// zero), so that K chunk m of A holds slice m+1 and K chunk p of B slice 7-p:
// the product of A chunk m and B chunk p belongs to degree 8 + m - p, and the
// pairs p >= m are exactly those with s + t <= 8.
#include <climits>
#include <algorithm>
#include <type_traits>

#include "bsmm_internal.h"

namespace bsmm {

namespace {

constexpr int kE = 23;
constexpr int kNE = kE * kE;
constexpr int kSlices = 7;
constexpr int kDegrees = 7;                        // g = 2..8
constexpr int kSliceBytes = 24;
constexpr int kRowBytes = kSlices * kSliceBytes;   // 168
constexpr int kBlockBytes = 3872;                  // 23 * 168 = 3864, padded to 16
constexpr int kChunks = kBlockBytes / 16;          // 242
constexpr int kHalves = kE * kRowBytes / 8;        // 483 eight-byte pieces with data
constexpr int kPer = (kChunks + 63) / 64;          // 4
constexpr int kLast = kChunks - 64 * (kPer - 1);   // lanes with a 4th chunk: 50
constexpr int kLdsRow = 240;                       // bytes per LDS row: 7 x 32 + 16 (bank stagger)
constexpr int kLdsOperand = 32 * kLdsRow;          // 32 rows (23..31 zero)
constexpr int kLdsStage = 2 * kLdsOperand;         // A then B^T: 15360 bytes
static_assert(kE * kRowBytes <= kBlockBytes && kBlockBytes % 16 == 0, "slice block layout");

// Exactness of the INT32 accumulators: a C block takes at most kMaxRowA
// products, each adding at most 7 * 23 * 64 * 64 to a degree.
static_assert((int64_t)kMaxRowA * 7 * 23 * 64 * 64 < INT32_MAX, "INT32 slice accumulators could overflow");

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) p[t] = v;
}

// rowof[b] = block row of block b (one thread per block row).
__global__ void k_block_rows(const int32_t* __restrict__ row_ptr, int32_t nbrows, int32_t* __restrict__ rowof) {
  for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < nbrows; i += gridDim.x * 256)
    for (int32_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b) rowof[b] = i;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Scale exponents: one wave per block.  The lanes read the block's values
// contiguously and put each value's frexp exponent (INT_MIN for zero) in the
// wave's LDS table; lane R < 23 then takes the largest over row R (A) or
// column R (B, transpose = 1) -- the exponent of the largest magnitude -- and
// raises exps[grp[b]*23 + R] with it.
template <int TRANSPOSE>
__global__ __launch_bounds__(256) void k_slice_exponents(const double* __restrict__ values,
                                                         const int64_t* __restrict__ d_nnzb,
                                                         const int32_t* __restrict__ grp, int32_t* __restrict__ exps) {
  __shared__ int32_t ext[4][kNE];
  const int64_t nnzb = *d_nnzb;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t b = (int64_t)blockIdx.x * 4 + wv; b < nnzb; b += (int64_t)gridDim.x * 4) {
    const double* v = values + b * kNE;
#pragma unroll
    for (int u = 0; u < (kNE + 63) / 64; ++u) {
      const int e = lane + 64 * u;
      if (e < kNE) {
        const double x = v[e];
        int ex = INT_MIN;
        if (x != 0.0) (void)frexp(x, &ex);
        ext[wv][e] = ex;
      }
    }
    wave_sync();
    if (lane < kE) {
      int32_t m = INT_MIN;
#pragma unroll
      for (int c = 0; c < kE; ++c) m = max(m, ext[wv][TRANSPOSE ? c * kE + lane : lane * kE + c]);
      if (m != INT_MIN) atomicMax(&exps[(int64_t)grp[b] * kE + lane], m);
    }
    wave_sync();
  }
}

// Digits of every value: one wave per block.  The lanes read the block's
// values contiguously, write the seven digits of each into the block's
// 3872-byte layout in LDS (pad bytes zeroed once, never written), and store
// the block as 16-byte pieces.
template <int TRANSPOSE>
__global__ __launch_bounds__(256) void k_slice_int8(const double* __restrict__ values, const int64_t* __restrict__ d_nnzb,
                                                    const int32_t* __restrict__ grp, const int32_t* __restrict__ exps,
                                                    uint8_t* __restrict__ out) {
  __shared__ __align__(16) int8_t buf[4][kBlockBytes];
  const int64_t nnzb = *d_nnzb;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int8_t* const t = buf[wv];
  for (int x = lane; x < kChunks; x += 64) reinterpret_cast<uint4*>(t)[x] = make_uint4(0, 0, 0, 0);
  wave_sync();
  for (int64_t b = (int64_t)blockIdx.x * 4 + wv; b < nnzb; b += (int64_t)gridDim.x * 4) {
    const int32_t gb = grp[b];
    const double* v = values + b * kNE;
#pragma unroll
    for (int u = 0; u < (kNE + 63) / 64; ++u) {
      const int e = lane + 64 * u;
      if (e < kNE) {
        const int r = e / kE, c = e - r * kE;                    // stored position
        const int R = TRANSPOSE ? c : r, C = TRANSPOSE ? r : c;  // slice row, position in the slice
        const int32_t ex = exps[(int64_t)gb * kE + R];
        const double y = ex == INT_MIN ? 0.0 : ldexp(v[e], -ex);
        double w = 64.0 * y;
#pragma unroll
        for (int sl = 0; sl < kSlices; ++sl) {
          const double d = rint(w);
          const int pos = TRANSPOSE ? kSlices - 1 - sl : sl;
          t[R * kRowBytes + pos * kSliceBytes + C] = (int8_t)(int)d;
          w = 128.0 * (w - d);
        }
      }
    }
    wave_sync();
    uint4* const o = reinterpret_cast<uint4*>(out + b * kBlockBytes);
    for (int x = lane; x < kChunks; x += 64) o[x] = reinterpret_cast<const uint4*>(t)[x];
    wave_sync();
  }
}

// block row of C block c: the last i with row_ptr[i] <= c
__device__ __forceinline__ int32_t row_of(const int32_t* row_ptr, int32_t nbrows, int32_t c) {
  int32_t lo = 0, hi = nbrows;
  while (hi - lo > 1) {
    const int32_t mid = __builtin_amdgcn_readfirstlane((lo + hi) >> 1);
    if (row_ptr[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Schedule as in the FP64 and BF16 23x23 kernels: each XCD owns a contiguous
// run of C blocks holding 1/8 of the products, cut into slices of equal
// product counts, and its waves take every wpx-th slice; products are fetched
// two ahead into two register slots and written to the wave's LDS stage one
// at a time.
// v_mfma_i32_32x32x32_i8 operands: lane l holds row (column) l % 32 and the
// 16 inner indices 16 (l / 32) .. +15 of a 32-wide chunk; result item x of
// lane l is row 8 (x / 4) + 4 (l / 32) + x % 4, column l % 32.
__global__ __launch_bounds__(256, 2) void k_numeric_slice23(
    const uint8_t* __restrict__ As, const uint8_t* __restrict__ Bs, const int32_t* __restrict__ ea,
    const int32_t* __restrict__ eb, const int32_t* __restrict__ c_row_ptr, int32_t nbrows,
    const int32_t* __restrict__ c_col_idx, const double* __restrict__ Ov, const int64_t* __restrict__ prod_ptr,
    const int2* __restrict__ prod, const int32_t* __restrict__ c_old_idx,
    double* __restrict__ Cv, const int64_t* __restrict__ totals, int use_old, double alpha, double beta,
    const int32_t* __restrict__ bounds, int32_t ns) {
  __shared__ __align__(16) unsigned char lds[4][kLdsStage];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned char* stage = &lds[wv][0];
  for (int x = lane; x < kLdsStage / 16; x += 64) reinterpret_cast<uint4*>(stage)[x] = make_uint4(0, 0, 0, 0);
  const bool tail = lane < kLast;
  // LDS byte offsets of the two 8-byte halves of chunk u*64 + lane: half h
  // is row h / 21, slice (h % 21) / 3, part h % 3 (-1: the block's padding)
  int off[kPer][2];
#pragma unroll
  for (int u = 0; u < kPer; ++u)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int h = 2 * (lane + 64 * u) + q;
      const int r = h / 21, w = h - 21 * r;
      off[u][q] = h < kHalves ? r * kLdsRow + (w / 3) * 32 + (w % 3) * 8 : -1;
    }
  const int opnd = (lane & 31) * kLdsRow + (lane >> 5) * 16;

  const int32_t nnzc = live_nnzc(totals);
  if (nnzc == 0) return;
  constexpr int kXcds = kSliceParts;
  const int32_t xcd = blockIdx.x % kXcds;
  const int32_t wpx = (int32_t)(gridDim.x / kXcds) * 4;
  const int32_t wix = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x / kXcds) * 4 + wv);
  const int32_t* const bnd = bounds + xcd * (ns + 1);
  const int64_t pbase = slices_pbase(bounds, ns);  // stack position of prod[0]

  // fetch cursor: slice iq of the XCD's part, products [ip, ip_end)
  int32_t iq = wix;
  int64_t ip = 0, ip_end = 0;
  if (iq < ns) {
    ip = prod_ptr[bnd[iq]];
    ip_end = prod_ptr[bnd[iq + 1]];
  }
  auto next_index = [&]() __attribute__((always_inline)) -> int64_t {
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
  u32x4 opa0[kPer], opb0[kPer], opa1[kPer], opb1[kPer];
  // the next product's slice blocks into a slot (a past-the-end product
  // rereads block 0, so every fetch issues the same loads)
  auto fetch_next = [&](u32x4(&opa)[kPer], u32x4(&opb)[kPer]) __attribute__((always_inline)) {
    {
      const int64_t ia = qa0 >= 0 ? qa0 : 0, ib = qa0 >= 0 ? qb0 : 0;
      const u32x4* Ab = reinterpret_cast<const u32x4*>(As + ia * kBlockBytes) + lane;
      const u32x4* Bb = reinterpret_cast<const u32x4*>(Bs + ib * kBlockBytes) + lane;
#pragma unroll
      for (int u = 0; u < kPer - 1; ++u) {
        opa[u] = Ab[64 * u];
        opb[u] = Bb[64 * u];
      }
      opa[kPer - 1] = Ab[tail ? 64 * (kPer - 1) : 0];
      opb[kPer - 1] = Bb[tail ? 64 * (kPer - 1) : 0];
    }
    qa0 = qa1;
    qb0 = qb1;
    const int64_t n = next_index();
    const int2 e = n >= 0 ? prod[n - pbase] : make_int2(-1, -1);
    qa1 = e.x;
    qb1 = e.y;
  };
  auto stage_write = [&](const u32x4(&opa)[kPer], const u32x4(&opb)[kPer]) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (u == kPer - 1 && !tail) continue;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (off[u][q] < 0) continue;
        const uint2 va = q ? make_uint2(opa[u][2], opa[u][3]) : make_uint2(opa[u][0], opa[u][1]);
        const uint2 vb = q ? make_uint2(opb[u][2], opb[u][3]) : make_uint2(opb[u][0], opb[u][1]);
        *reinterpret_cast<uint2*>(stage + off[u][q]) = va;
        *reinterpret_cast<uint2*>(stage + kLdsOperand + off[u][q]) = vb;
      }
    }
  };

  v16i acc[kDegrees];  // acc[g - 2]: degree g
  auto multiply_stage = [&]() __attribute__((always_inline)) {
    v4i bf[kSlices];
#pragma unroll
    for (int p = 0; p < kSlices; ++p) bf[p] = *reinterpret_cast<const v4i*>(stage + kLdsOperand + 32 * p + opnd);
#pragma unroll
    for (int m = 0; m < kSlices; ++m) {
      const v4i af = *reinterpret_cast<const v4i*>(stage + 32 * m + opnd);
#pragma unroll
      for (int p = m; p < kSlices; ++p)
        acc[6 + m - p] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af, bf[p], acc[6 + m - p], 0, 0, 0);
    }
  };

  // compute cursor: slice cq, C blocks [c, c1), products [p, pe) of block c
  int32_t cq = wix, c = 0, c1 = 0;
  int64_t p = 0, pe = 0;
  while (cq < ns && bnd[cq] == bnd[cq + 1]) cq += wpx;
  if (cq >= ns) return;
  c = bnd[cq];
  c1 = bnd[cq + 1];
  p = prod_ptr[c];
  pe = prod_ptr[c + 1];
#pragma unroll
  for (int g = 0; g < kDegrees; ++g) acc[g] = v16i{};

  const int Q = lane & 31;
  // Finish every C block that ends at p: combine the degrees in FP64, scale,
  // add beta*C_in and store (rows of 23 consecutive doubles per item).
  auto advance = [&]() __attribute__((always_inline)) -> bool {
    while (p == pe) {
      const int32_t i = row_of(c_row_ptr, nbrows, c);
      const int32_t j = c_col_idx[c];
      const int32_t o = use_old ? c_old_idx[c] : -1;
      int32_t ebq = Q < kE ? eb[(int64_t)j * kE + Q] : 0;
      if (ebq == INT_MIN) ebq = 0;
      double* const out = Cv + (int64_t)c * kNE;
      const double* const ov = Ov + (int64_t)(o >= 0 ? o : 0) * kNE;
#pragma unroll
      for (int x = 0; x < 16; ++x) {
        const int R = 8 * (x >> 2) + 4 * (lane >> 5) + (x & 3);
        if (R < kE && Q < kE) {
          double v = 0.0;
#pragma unroll
          for (int g = kDegrees - 1; g >= 0; --g) v += ldexp((double)acc[g][x], -(12 + 7 * g));
          int32_t ear = ea[(int64_t)i * kE + R];
          if (ear == INT_MIN) ear = 0;
          double res = alpha * ldexp(v, ear + ebq);
          if (o >= 0) res += beta * ov[R * kE + Q];
          out[R * kE + Q] = res;
        }
      }
#pragma unroll
      for (int g = 0; g < kDegrees; ++g) acc[g] = v16i{};
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

  fetch_next(opa0, opb0);
  fetch_next(opa1, opb1);
  // (the two halves carry distinct markers so that the compiler keeps the
  // slots as separate registers)
  for (;;) {
    if (p == pe && !advance()) break;
    asm volatile("; slot 0");
    wsync();
    stage_write(opa0, opb0);
    fetch_next(opa0, opb0);
    wsync();
    multiply_stage();
    ++p;
    if (p == pe && !advance()) break;
    asm volatile("; slot 1");
    wsync();
    stage_write(opa1, opb1);
    fetch_next(opa1, opb1);
    wsync();
    multiply_stage();
    ++p;
  }
}

}  // namespace

int64_t slice_bytes(int64_t nblocks) { return nblocks * kBlockBytes; }

hipError_t launch_slice_int8x7(const double* values, const int64_t* d_nnzb, int64_t bound, int transpose,
                               const int32_t* row_ptr, int32_t nbrows, const int32_t* col_idx, int32_t ngroups,
                               int32_t* rowof, int32_t* exps, uint8_t* out, hipStream_t s) {
  const int64_t nexp = (int64_t)ngroups * kE;
  if (nexp > 0) {
    const int64_t g = std::min<int64_t>((nexp + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3((uint32_t)g), dim3(256), 0, s, exps, nexp, (int32_t)INT_MIN);
  }
  if (bound <= 0) return hipGetLastError();
  const int32_t* grp = col_idx;
  if (!transpose) {
    const int32_t g = std::max<int32_t>(1, std::min<int32_t>((nbrows + 255) / 256, 4096));
    hipLaunchKernelGGL(k_block_rows, dim3(g), dim3(256), 0, s, row_ptr, nbrows, rowof);
    grp = rowof;
  }
  const int64_t ge = std::min<int64_t>((bound + 3) / 4, 16384);  // one wave per block
  const int64_t gs = ge;
  if (transpose) {
    hipLaunchKernelGGL(k_slice_exponents<1>, dim3((uint32_t)ge), dim3(256), 0, s, values, d_nnzb, grp, exps);
    hipLaunchKernelGGL(k_slice_int8<1>, dim3((uint32_t)gs), dim3(256), 0, s, values, d_nnzb, grp, exps, out);
  } else {
    hipLaunchKernelGGL(k_slice_exponents<0>, dim3((uint32_t)ge), dim3(256), 0, s, values, d_nnzb, grp, exps);
    hipLaunchKernelGGL(k_slice_int8<0>, dim3((uint32_t)gs), dim3(256), 0, s, values, d_nnzb, grp, exps, out);
  }
  return hipGetLastError();
}

hipError_t launch_numeric_slice23(const NumArgs& a, const int32_t* c_row_ptr, int32_t nbrows, const uint8_t* As,
                                  const uint8_t* Bs, const int32_t* ea, const int32_t* eb, int32_t* work,
                                  hipStream_t s) {
  if (a.nnzc_bound <= 0) return hipSuccess;
  const int32_t ns = launch_product_slices(a.prod_ptr, a.totals, a.c_row_ptr, a.panel, work, s);
  hipLaunchKernelGGL(k_numeric_slice23, dim3(tile23_workgroups()), dim3(256), 0, s, As, Bs, ea, eb, c_row_ptr,
                     nbrows, a.c_col_idx, a.use_old ? a.Cin.values : a.c_values, a.prod_ptr, a.prod,
                     a.c_old_idx, a.c_values, a.totals, a.use_old, a.alpha, a.beta, work, ns);
  return hipGetLastError();
}

}  // namespace bsmm
