// Split-precision block products for 23x23 blocks on BF16 matrix cores.
//
// Every FP64 operand value x is split once per multiply into three BF16
// terms, x ~ s0 + s1 + s2 with s0 = bf16(x), s1 = bf16(x - s0),
// s2 = bf16(x - s0 - s1) (round to nearest even; the residuals are exact in
// FP64).  A block product keeps the six term products s_i(a) s_j(b) with
// i + j <= 2, on v_mfma_f32_16x16x32_bf16 with FP32 accumulation; the FP32
// result of each block product is added to an FP64 accumulator, and the C
// block is finished in FP64 (alpha, beta, C_in).  Norms, the filter and the
// symbolic phase stay FP64 (they run before this kernel, unchanged).
//
// Storage of the split terms (per block, 16-byte aligned): three slices of
// 23 rows x 24 BF16 (the 24th column zero), 3312 bytes instead of the 4232
// bytes of the FP64 block.  A is stored as is (row i holds A(i, :)), B
// transposed (row j holds B(:, j)), so both MFMA operands read 8 consecutive
// inner indices with one 16-byte LDS load.
#include <type_traits>

#include "bsmm_internal.h"

namespace bsmm {

namespace {

constexpr int kE = 23;                     // block edge
constexpr int kRowPad = 24;                // BF16 per stored row
constexpr int kSlice = kE * kRowPad;       // 552 BF16 per slice
constexpr int kSplitBlock = 3 * kSlice;    // 1656 BF16 = 3312 bytes per block
constexpr int kChunks = kSplitBlock * 2 / 16;  // 207 16-byte chunks per block
constexpr int kChunksPerSlice = kSlice * 2 / 16;  // 69
constexpr int kLdsRow = 80;                // bytes per LDS row (32 BF16 + pad)
constexpr int kLdsSlice = 32 * kLdsRow;    // 2560 bytes: 32 rows, rows 23..31 zero
constexpr int kLdsOperand = 3 * kLdsSlice; // 7680 bytes
constexpr int kLdsStage = 2 * kLdsOperand; // 15360 bytes: A slices then B^T slices
constexpr int kPer = (kChunks + 63) / 64;  // 4 chunk loads per lane and operand
constexpr int kLast = kChunks - 64 * (kPer - 1);  // lanes with a 4th chunk: 15

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // 16 bytes, a plain vector value

// float -> bf16 bits, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ double bf16_value(uint16_t h) { return (double)__uint_as_float((uint32_t)h << 16); }

// One wave per block: the 529 values are read with coalesced loads, split in
// registers, placed in LDS in the stored layout (three slices of 23 rows x
// 24 BF16, B transposed, the 24th column zero) and written out as 16-byte
// chunks, so both the reads and the writes are contiguous.
__global__ __launch_bounds__(256) void k_split_bf16x3(const double* __restrict__ values,
                                                      const int64_t* __restrict__ d_nnzb, int transpose,
                                                      uint16_t* __restrict__ out) {
  __shared__ __align__(16) uint16_t tile[4][kSplitBlock];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint16_t* const t = tile[wv];
  const int64_t nnzb = *d_nnzb;
  // the pad column (stored column 23 of every row of every slice) is never
  // written below: zero it once
  for (int x = lane; x < 3 * kE; x += 64) t[(x / kE) * kSlice + (x % kE) * kRowPad + kE] = 0;
  for (int64_t b = (int64_t)blockIdx.x * 4 + wv; b < nnzb; b += (int64_t)gridDim.x * 4) {
    const double* v = values + b * (kE * kE);
#pragma unroll
    for (int u = 0; u < (kE * kE + 63) / 64; ++u) {
      const int e = lane + 64 * u;
      if (e < kE * kE) {
        const double x = v[e];
        const int r = e / kE, c = e - r * kE;  // the block's row r, column c
        const int pos = transpose ? c * kRowPad + r : r * kRowPad + c;
        const uint16_t h0 = bf16_bits((float)x);
        const double r1 = x - bf16_value(h0);
        const uint16_t h1 = bf16_bits((float)r1);
        const double r2 = r1 - bf16_value(h1);
        t[pos] = h0;
        t[kSlice + pos] = h1;
        t[2 * kSlice + pos] = bf16_bits((float)r2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    u32x4* const o = reinterpret_cast<u32x4*>(out + b * kSplitBlock);
    const u32x4* const src = reinterpret_cast<const u32x4*>(t);
    for (int x = lane; x < kChunks; x += 64) o[x] = src[x];
    // every lane has read the tile before the next block overwrites it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Schedule as in the FP64 23x23 kernel: each XCD owns a contiguous run of C
// blocks holding 1/8 of the products, cut into slices of equal product
// counts (launch_product_slices); its waves take every wpx-th slice.
// Products are fetched two steps ahead into two register slots; one LDS
// stage per wave, written after the previous product has been read.
__global__ __launch_bounds__(256, 2) void k_numeric_split23(
    const uint16_t* __restrict__ As, const uint16_t* __restrict__ Bs, const double* __restrict__ Ov,
    const int64_t* __restrict__ prod_ptr, const int2* __restrict__ prod,
    const int32_t* __restrict__ c_old_idx, double* __restrict__ Cv, const int64_t* __restrict__ totals,
    int use_old, double alpha, double beta, const int32_t* __restrict__ bounds, int32_t ns) {
  constexpr int NE = kE * kE;
  constexpr int PER_C = (NE + 63) / 64;
  constexpr int LAST_C = NE - 64 * (PER_C - 1);
  __shared__ __align__(16) unsigned char lds[4][kLdsStage];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned char* stage = &lds[wv][0];
  for (int x = lane; x < kLdsStage / 16; x += 64) reinterpret_cast<uint4*>(stage)[x] = make_uint4(0, 0, 0, 0);

  // LDS byte offset of chunk u*64 + lane of a stored split block
  int off[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int c = (u < kPer - 1 || lane < kLast) ? lane + 64 * u : 0;
    const int s = c / kChunksPerSlice, w = c - s * kChunksPerSlice;
    off[u] = s * kLdsSlice + (w / 3) * kLdsRow + (w % 3) * 16;
  }
  const bool tail = lane < kLast;
  // MFMA operand address (bytes) of this lane within a slice, tile row/col 0
  const int opnd = (lane & 15) * kLdsRow + (lane >> 4) * 16;

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
  // two register slots, as separately named arrays (kept in registers)
  u32x4 opa0[kPer], opb0[kPer], opa1[kPer], opb1[kPer];
  // the next product's split blocks into a slot (a past-the-end product
  // rereads block 0, so every fetch issues the same loads)
  auto fetch_next = [&](u32x4(&opa)[kPer], u32x4(&opb)[kPer]) __attribute__((always_inline)) {
    {
      const int64_t ia = qa0 >= 0 ? qa0 : 0, ib = qa0 >= 0 ? qb0 : 0;
      const u32x4* Ab = reinterpret_cast<const u32x4*>(As + ia * kSplitBlock) + lane;
      const u32x4* Bb = reinterpret_cast<const u32x4*>(Bs + ib * kSplitBlock) + lane;
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
    for (int u = 0; u < kPer - 1; ++u) {
      *reinterpret_cast<u32x4*>(stage + off[u]) = opa[u];
      *reinterpret_cast<u32x4*>(stage + kLdsOperand + off[u]) = opb[u];
    }
    if (tail) {
      *reinterpret_cast<u32x4*>(stage + off[kPer - 1]) = opa[kPer - 1];
      *reinterpret_cast<u32x4*>(stage + kLdsOperand + off[kPer - 1]) = opb[kPer - 1];
    }
  };

  double acc[16];  // C tile (mt, nt) item i at acc[4*(2*mt+nt) + i]
  auto multiply_stage = [&]() {
    bf16x8 a[3][2], b[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[s][t] = *reinterpret_cast<const bf16x8*>(stage + s * kLdsSlice + t * 16 * kLdsRow + opnd);
        b[s][t] = *reinterpret_cast<const bf16x8*>(stage + kLdsOperand + s * kLdsSlice + t * 16 * kLdsRow + opnd);
      }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        // term products, smallest first: (0,2) (1,1) (2,0) (0,1) (1,0) (0,0)
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][mt], b[2][nt], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][mt], b[1][nt], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][mt], b[0][nt], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][mt], b[1][nt], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][mt], b[0][nt], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][mt], b[0][nt], c, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[4 * (2 * mt + nt) + i] += (double)c[i];
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
  for (int x = 0; x < 16; ++x) acc[x] = 0.0;

  // Finish every C block that ends at p: park alpha*acc in the stage (free:
  // the next product is written afterwards), add beta*C_in, store coalesced.
  auto advance = [&]() -> bool {
    double* const tile = reinterpret_cast<double*>(stage);
    const bool tl = lane < LAST_C;
    while (p == pe) {
      wsync();
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int R = 16 * mt + 4 * (lane >> 4) + i, Cc = 16 * nt + (lane & 15);
            if (R < kE && Cc < kE) tile[R * kE + Cc] = alpha * acc[4 * (2 * mt + nt) + i];
          }
      wsync();
      const int32_t o = use_old ? c_old_idx[c] : -1;
      double* out = Cv + (int64_t)c * NE + lane;
      const double* tp = tile + lane;
      if (o >= 0) {
        const double* ov = Ov + (int64_t)o * NE + lane;
        double ol[PER_C];
#pragma unroll
        for (int u = 0; u < PER_C - 1; ++u) ol[u] = ov[64 * u];
        ol[PER_C - 1] = tl ? ov[64 * (PER_C - 1)] : 0.0;
#pragma unroll
        for (int u = 0; u < PER_C - 1; ++u) out[64 * u] = tp[64 * u] + beta * ol[u];
        if (tl) out[64 * (PER_C - 1)] = tp[64 * (PER_C - 1)] + beta * ol[PER_C - 1];
      } else {
#pragma unroll
        for (int u = 0; u < PER_C - 1; ++u) out[64 * u] = tp[64 * u];
        if (tl) out[64 * (PER_C - 1)] = tp[64 * (PER_C - 1)];
      }
      wsync();
      // the parked tile overwrote stage bytes that must read as zero padding
      for (int x = lane; x < (NE * 8 + 15) / 16; x += 64)
        reinterpret_cast<uint4*>(stage)[x] = make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int x = 0; x < 16; ++x) acc[x] = 0.0;
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

  // Pipeline: product n is fetched into slot n % 2 at step n-2, written to
  // the stage at the start of step n (after product n-1 has been read) and
  // multiplied; its slot then takes product n+2.
  fetch_next(opa0, opb0);
  fetch_next(opa1, opb1);
  // (the two halves carry distinct markers so that the compiler does not
  // merge them into one body indexing the slots at run time, which would put
  // the slots in scratch memory)
  for (;;) {
    if (p == pe && !advance()) break;
    asm volatile("; slot 0");
    wsync();
    __builtin_amdgcn_s_setprio(1);  // as in the FP64 kernel: staging and loads first
    stage_write(opa0, opb0);
    fetch_next(opa0, opb0);
    __builtin_amdgcn_s_setprio(0);
    wsync();
    multiply_stage();
    ++p;
    if (p == pe && !advance()) break;
    asm volatile("; slot 1");
    wsync();
    __builtin_amdgcn_s_setprio(1);  // as in the FP64 kernel: staging and loads first
    stage_write(opa1, opb1);
    fetch_next(opa1, opb1);
    __builtin_amdgcn_s_setprio(0);
    wsync();
    multiply_stage();
    ++p;
  }
}

}  // namespace

int64_t split_elems(int64_t nblocks) { return nblocks * kSplitBlock; }

hipError_t launch_split_bf16x3(const double* values, const int64_t* d_nnzb, int64_t bound, int transpose,
                               uint16_t* out, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  int64_t blocks = (bound + 3) / 4;  // one wave per block
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_split_bf16x3, dim3((uint32_t)blocks), dim3(256), 0, s, values, d_nnzb, transpose, out);
  return hipGetLastError();
}

hipError_t launch_numeric_split23(const NumArgs& a, const uint16_t* As, const uint16_t* Bs, int32_t* work,
                                  hipStream_t s) {
  if (a.nnzc_bound <= 0) return hipSuccess;
  const int32_t ns = launch_product_slices(a.prod_ptr, a.totals, a.c_row_ptr, a.panel, work, s);
  hipLaunchKernelGGL(k_numeric_split23, dim3(tile23_workgroups()), dim3(256), 0, s, As, Bs,
                     a.use_old ? a.Cin.values : a.c_values, a.prod_ptr, a.prod, a.c_old_idx,
                     a.c_values, a.totals, a.use_old, a.alpha, a.beta, work, ns);
  return hipGetLastError();
}

}  // namespace bsmm
