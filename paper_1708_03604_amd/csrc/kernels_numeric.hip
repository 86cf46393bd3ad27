// Numeric phase: for every C block (i,j), acc = sum over its kept products
// A(i,k) * B(k,j) (in stack order, i.e. ascending k), then
// C(i,j) = alpha*acc + beta*C_in(i,j) (Section 2 of the paper: the local
// multiply is a sum of pairwise products of (m x k) and (k x n) blocks).
//
// Each C block is owned by exactly one wave, so no floating-point atomics are
// used and the result does not depend on the schedule.
#include "bsmm_internal.h"

namespace bsmm {

// Any block sizes: lanes own output elements, operands read from global memory.
__global__ __launch_bounds__(256) void k_numeric_generic(NumArgs g) {
  const int lane = threadIdx.x & 63;
  const int32_t nwaves = gridDim.x * 4;
  for (int32_t c = blockIdx.x * 4 + (threadIdx.x >> 6); c < g.nnzc; c += nwaves) {
    const int32_t n = g.c_col_sizes[g.c_col_idx[c]];
    const int64_t off = g.c_blk_off[c];
    const int64_t mn = g.c_blk_off[c + 1] - off;
    const int32_t m = (int32_t)(mn / n);
    const int64_t p0 = g.prod_ptr[c], p1 = g.prod_ptr[c + 1];
    const int32_t old = g.use_old ? g.c_old_idx[c] : -1;
    const double* oldv = old >= 0 ? g.Cin.values + g.Cin.blk_off[old] : nullptr;
    for (int64_t e0 = 0; e0 < mn; e0 += 64) {
      const int64_t e = e0 + lane;
      const bool active = e < mn;
      const int32_t r = active ? (int32_t)(e / n) : 0;
      const int32_t s = active ? (int32_t)(e % n) : 0;
      double acc = 0.0;
      for (int64_t x = p0; x < p1; ++x) {
        const int32_t a = g.prod_a[x];
        const int32_t b = g.prod_b[x];
        const int64_t ao = g.A.blk_off[a];
        const int32_t k = (int32_t)((g.A.blk_off[a + 1] - ao) / m);
        const double* av = g.A.values + ao + (int64_t)r * k;
        const double* bv = g.B.values + g.B.blk_off[b] + s;
        if (active)
          for (int32_t t = 0; t < k; ++t) acc = fma(av[t], bv[(int64_t)t * n], acc);
      }
      if (active) {
        double v = g.alpha * acc;
        if (oldv) v = v + g.beta * oldv[e];
        g.c_values[off + e] = v;
      }
    }
  }
}

hipError_t launch_numeric(const NumArgs& a, int uniform_size, hipStream_t s) {
  (void)uniform_size;
  if (a.nnzc <= 0) return hipSuccess;
  int32_t blocks = (a.nnzc + 3) / 4;
  if (blocks > 32768) blocks = 32768;
  hipLaunchKernelGGL(k_numeric_generic, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace bsmm
