/*
 * Plain CPU FP64 oracle for the node-local DBCSR block-sparse multiply.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or load
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Bethune et al., "Porting of the DBCSR library for Sparse
 * Matrix-Matrix Multiplications to Intel Xeon Phi systems", 2017):
 *   - matrices are stored in blocked CSR form (Section 2, storage paragraph);
 *   - the local multiply is C = C + A*B built from pairwise products of an
 *     (m x k) A block with a (k x n) B block (Section 2, local computation);
 *     generalised here to C = alpha*A*B + beta*C;
 *   - the traversal runs over A block rows and, inside each, over B blocks,
 *     i.e. row-wise Gustavson SpGEMM (Section 1.1 and Section 2);
 *   - a block product is performed only if the product of the two block norms
 *     exceeds a threshold: the on-the-fly filter (Section 2).
 *
 * Readings where the paper is silent:
 *   - the block norm is the Frobenius norm;
 *   - its sum of squares runs in a fixed order so that the filter decision is
 *     reproducible bit for bit: 64 interleaved partial sums (element e goes to
 *     partial e mod 64, ascending e, each step a fused multiply-add), then a
 *     pairwise tree (partial l += partial l+d for d = 32,16,...,1), then the
 *     correctly rounded square root;
 *   - a product is kept iff eps <= 0 or fl(normA * normB) > eps (strict);
 *     alpha does not enter the decision;
 *   - the result pattern is every (i,j) with at least one kept product, plus
 *     the pattern of the old C when beta != 0; blocks stay even if their
 *     values are zero; with beta == 0 the old C is never read;
 *   - values: acc_ij = sum over kept k (ascending) and t (ascending) of
 *     a_rt * b_ts, separate multiply and add; C_ij = alpha*acc + beta*Cold_ij;
 *   - filter(M, eps) keeps a block iff eps <= 0 or its norm > eps;
 *   - blocks are stored row-major, blocks contiguous in CSR order.
 *
 * Compiled with -ffp-contract=off: the only fused operations are the fma()
 * calls written below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG 1
#define OR_E_SHAPE 2
#define OR_E_PATTERN 3
#define OR_E_NOMEM 5
#define OR_E_CAPACITY 6

typedef struct {
  int32_t nbrows;
  int32_t nbcols;
  const int32_t* row_sizes; /* [nbrows] */
  const int32_t* col_sizes; /* [nbcols] */
  int32_t nnzb;
  const int32_t* row_ptr; /* [nbrows+1] */
  const int32_t* col_idx; /* [nnzb] */
  const double* values;   /* sum of block sizes, CSR block order, row-major */
} oracle_mat;

/* Blocked CSR well-formedness (Section 2 storage format). */
int oracle_check(const oracle_mat* M) {
  if (M->nbrows < 0 || M->nbcols < 0 || M->nnzb < 0) return OR_E_ARG;
  for (int32_t i = 0; i < M->nbrows; ++i)
    if (M->row_sizes[i] < 1) return OR_E_ARG;
  for (int32_t j = 0; j < M->nbcols; ++j)
    if (M->col_sizes[j] < 1) return OR_E_ARG;
  if (M->row_ptr[0] != 0 || M->row_ptr[M->nbrows] != M->nnzb) return OR_E_PATTERN;
  for (int32_t i = 0; i < M->nbrows; ++i) {
    if (M->row_ptr[i + 1] < M->row_ptr[i]) return OR_E_PATTERN;
    for (int32_t b = M->row_ptr[i]; b < M->row_ptr[i + 1]; ++b) {
      if (M->col_idx[b] < 0 || M->col_idx[b] >= M->nbcols) return OR_E_PATTERN;
      if (b > M->row_ptr[i] && M->col_idx[b] <= M->col_idx[b - 1]) return OR_E_PATTERN;
    }
  }
  return OR_OK;
}

/* Offset (in doubles) of every block of M; off[nnzb] is the value count. */
static int64_t* block_offsets(const oracle_mat* M) {
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)M->nnzb + 1));
  if (!off) return NULL;
  off[0] = 0;
  for (int32_t i = 0; i < M->nbrows; ++i)
    for (int32_t b = M->row_ptr[i]; b < M->row_ptr[i + 1]; ++b)
      off[b + 1] = off[b] + (int64_t)M->row_sizes[i] * M->col_sizes[M->col_idx[b]];
  return off;
}

int64_t oracle_value_count(const oracle_mat* M) {
  int64_t n = 0;
  for (int32_t i = 0; i < M->nbrows; ++i)
    for (int32_t b = M->row_ptr[i]; b < M->row_ptr[i + 1]; ++b)
      n += (int64_t)M->row_sizes[i] * M->col_sizes[M->col_idx[b]];
  return n;
}

/* Frobenius norm of one block of n elements in the fixed order described above. */
static double block_norm(const double* x, int64_t n) {
  double part[64];
  for (int l = 0; l < 64; ++l) part[l] = 0.0;
  for (int64_t e = 0; e < n; ++e) part[e % 64] = fma(x[e], x[e], part[e % 64]);
  for (int d = 32; d >= 1; d /= 2)
    for (int l = 0; l < d; ++l) part[l] = part[l] + part[l + d];
  return sqrt(part[0]);
}

/* Norm of every stored block (the quantity the on-the-fly filter uses, Section 2). */
int oracle_norms(const oracle_mat* M, double* out) {
  int64_t* off = block_offsets(M);
  if (!off) return OR_E_NOMEM;
  for (int32_t b = 0; b < M->nnzb; ++b) out[b] = block_norm(M->values + off[b], off[b + 1] - off[b]);
  free(off);
  return OR_OK;
}

static int kept(const double* nA, const double* nB, int32_t p, int32_t q, double eps) {
  if (eps <= 0.0) return 1;
  double prod = nA[p] * nB[q];
  return prod > eps;
}

/* Position of column j in block row i of M, or -1. */
static int32_t find_block(const oracle_mat* M, int32_t i, int32_t j) {
  int32_t lo = M->row_ptr[i], hi = M->row_ptr[i + 1] - 1;
  while (lo <= hi) {
    int32_t mid = lo + (hi - lo) / 2;
    if (M->col_idx[mid] == j) return mid;
    if (M->col_idx[mid] < j) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Sorted result columns of block row i and its kept-product count.
 * mark[] (nbcols bytes) is all-zero on entry and on exit. */
static int32_t row_columns(const oracle_mat* A, const oracle_mat* B, const oracle_mat* Cold, int use_old,
                           const double* nA, const double* nB, double eps, int32_t i, unsigned char* mark,
                           int32_t* cols, int64_t* nprod) {
  int32_t n = 0;
  int64_t np = 0;
  for (int32_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; ++p) {
    int32_t k = A->col_idx[p];
    for (int32_t q = B->row_ptr[k]; q < B->row_ptr[k + 1]; ++q) {
      if (!kept(nA, nB, p, q, eps)) continue;
      ++np;
      int32_t j = B->col_idx[q];
      if (!mark[j]) {
        mark[j] = 1;
        cols[n++] = j;
      }
    }
  }
  if (use_old) {
    for (int32_t q = Cold->row_ptr[i]; q < Cold->row_ptr[i + 1]; ++q) {
      int32_t j = Cold->col_idx[q];
      if (!mark[j]) {
        mark[j] = 1;
        cols[n++] = j;
      }
    }
  }
  qsort(cols, (size_t)n, sizeof(int32_t), cmp_i32);
  for (int32_t x = 0; x < n; ++x) mark[cols[x]] = 0;
  *nprod = np;
  return n;
}

/*
 * C = alpha*A*B + beta*Cold with on-the-fly filter eps.
 * Cold may be NULL when beta == 0 (it is not read then).
 * Outputs: c_row_ptr[nbrows+1], c_col_idx[cap_nnzb], c_values[cap_nvals] and the
 * product stack (st_c, st_a, st_b)[cap_nprod]: one entry per kept block product,
 * giving the C block, A block and B block index, sorted by C block and then
 * by inner block index k.  counts[0..2] = result nnzb, value count, product count.
 * If a capacity is too small, counts are set, nothing else is written and
 * OR_E_CAPACITY is returned.
 */
int oracle_multiply(double alpha, const oracle_mat* A, const oracle_mat* B, double beta, const oracle_mat* Cold,
                    double eps, int64_t cap_nnzb, int64_t cap_nvals, int64_t cap_nprod, int32_t* c_row_ptr,
                    int32_t* c_col_idx, double* c_values, int32_t* st_c, int32_t* st_a, int32_t* st_b,
                    int64_t* counts) {
  int rc;
  if (isnan(eps) || isinf(eps) || isnan(alpha) || isinf(alpha) || isnan(beta) || isinf(beta)) return OR_E_ARG;
  if ((rc = oracle_check(A)) != OR_OK) return rc;
  if ((rc = oracle_check(B)) != OR_OK) return rc;
  if (A->nbcols != B->nbrows) return OR_E_SHAPE;
  for (int32_t k = 0; k < A->nbcols; ++k)
    if (A->col_sizes[k] != B->row_sizes[k]) return OR_E_SHAPE;
  const int use_old = (beta != 0.0) && Cold != NULL;
  if (use_old) {
    if ((rc = oracle_check(Cold)) != OR_OK) return rc;
    if (Cold->nbrows != A->nbrows || Cold->nbcols != B->nbcols) return OR_E_SHAPE;
    for (int32_t i = 0; i < A->nbrows; ++i)
      if (Cold->row_sizes[i] != A->row_sizes[i]) return OR_E_SHAPE;
    for (int32_t j = 0; j < B->nbcols; ++j)
      if (Cold->col_sizes[j] != B->col_sizes[j]) return OR_E_SHAPE;
  }
  const int32_t nbrows = A->nbrows, nbcols = B->nbcols;

  double* nA = (double*)malloc(sizeof(double) * ((size_t)A->nnzb + 1));
  double* nB = (double*)malloc(sizeof(double) * ((size_t)B->nnzb + 1));
  int64_t* offA = block_offsets(A);
  int64_t* offB = block_offsets(B);
  int64_t* offO = use_old ? block_offsets(Cold) : NULL;
  int32_t* rowC = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nbrows + 1));
  int64_t* rowP = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nbrows + 1));
  int64_t* rowV = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nbrows + 1));
  if (!nA || !nB || !offA || !offB || (use_old && !offO) || !rowC || !rowP || !rowV) {
    rc = OR_E_NOMEM;
    goto done;
  }
  if (eps > 0.0) {
    oracle_norms(A, nA);
    oracle_norms(B, nB);
  }

  /* Pass 1: per block row, the number of result blocks, products and values. */
  rc = OR_OK;
#pragma omp parallel
  {
    unsigned char* mark = (unsigned char*)calloc((size_t)nbcols + 1, 1);
    int32_t* cols = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nbcols + 1));
    if (!mark || !cols) {
#pragma omp critical
      rc = OR_E_NOMEM;
    } else {
#pragma omp for schedule(static)
      for (int32_t i = 0; i < nbrows; ++i) {
        int64_t np;
        int32_t n = row_columns(A, B, Cold, use_old, nA, nB, eps, i, mark, cols, &np);
        int64_t nv = 0;
        for (int32_t x = 0; x < n; ++x) nv += (int64_t)A->row_sizes[i] * B->col_sizes[cols[x]];
        rowC[i + 1] = n;
        rowP[i + 1] = np;
        rowV[i + 1] = nv;
      }
    }
    free(mark);
    free(cols);
  }
  if (rc != OR_OK) goto done;
  rowC[0] = 0;
  rowP[0] = 0;
  rowV[0] = 0;
  for (int32_t i = 0; i < nbrows; ++i) {
    if ((int64_t)rowC[i] + rowC[i + 1] > INT32_MAX) {
      rc = OR_E_CAPACITY;
      goto done;
    }
    rowC[i + 1] += rowC[i];
    rowP[i + 1] += rowP[i];
    rowV[i + 1] += rowV[i];
  }
  counts[0] = rowC[nbrows];
  counts[1] = rowV[nbrows];
  counts[2] = rowP[nbrows];
  if (counts[0] > cap_nnzb || counts[1] > cap_nvals || counts[2] > cap_nprod) {
    rc = OR_E_CAPACITY;
    goto done;
  }
  for (int32_t i = 0; i <= nbrows; ++i) c_row_ptr[i] = rowC[i];

  /* Pass 2: pattern, product stack and values, one block row per thread. */
#pragma omp parallel
  {
    unsigned char* mark = (unsigned char*)calloc((size_t)nbcols + 1, 1);
    int32_t* cols = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nbcols + 1));
    if (!mark || !cols) {
#pragma omp critical
      rc = OR_E_NOMEM;
    } else {
#pragma omp for schedule(static)
      for (int32_t i = 0; i < nbrows; ++i) {
        int64_t np;
        int32_t n = row_columns(A, B, Cold, use_old, nA, nB, eps, i, mark, cols, &np);
        const int32_t m = A->row_sizes[i];
        int64_t prod_pos = rowP[i];
        int64_t val_pos = rowV[i];
        for (int32_t x = 0; x < n; ++x) {
          const int32_t j = cols[x];
          const int32_t nn = B->col_sizes[j];
          const int32_t c = rowC[i] + x;
          double* acc = c_values + val_pos;
          c_col_idx[c] = j;
          for (int64_t e = 0; e < (int64_t)m * nn; ++e) acc[e] = 0.0;
          for (int32_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; ++p) {
            const int32_t k = A->col_idx[p];
            const int32_t q = find_block(B, k, j);
            if (q < 0 || !kept(nA, nB, p, q, eps)) continue;
            st_c[prod_pos] = c;
            st_a[prod_pos] = p;
            st_b[prod_pos] = q;
            ++prod_pos;
            const int32_t kk = A->col_sizes[k];
            const double* a = A->values + offA[p];
            const double* b = B->values + offB[q];
            for (int32_t r = 0; r < m; ++r)
              for (int32_t s = 0; s < nn; ++s) {
                double sum = acc[(int64_t)r * nn + s];
                for (int32_t t = 0; t < kk; ++t) sum = sum + a[(int64_t)r * kk + t] * b[(int64_t)t * nn + s];
                acc[(int64_t)r * nn + s] = sum;
              }
          }
          const int32_t o = use_old ? find_block(Cold, i, j) : -1;
          const double* old = (o >= 0) ? Cold->values + offO[o] : NULL;
          for (int64_t e = 0; e < (int64_t)m * nn; ++e) {
            double v = alpha * acc[e];
            if (old) v = v + beta * old[e];
            acc[e] = v;
          }
          val_pos += (int64_t)m * nn;
        }
      }
    }
    free(mark);
    free(cols);
  }

done:
  free(nA);
  free(nB);
  free(offA);
  free(offB);
  free(offO);
  free(rowC);
  free(rowP);
  free(rowV);
  return rc;
}

/*
 * filter(M, eps): keep a block iff eps <= 0 or its norm > eps ("increases
 * sparsity", Section 2).  Outputs the compacted pattern and values;
 * counts[0..1] = kept blocks, kept values.  Capacity handling as in multiply.
 */
int oracle_filter(const oracle_mat* M, double eps, int64_t cap_nnzb, int64_t cap_nvals, int32_t* o_row_ptr,
                  int32_t* o_col_idx, double* o_values, int64_t* counts) {
  int rc = oracle_check(M);
  if (rc != OR_OK) return rc;
  if (isnan(eps) || isinf(eps)) return OR_E_ARG;
  double* nrm = (double*)malloc(sizeof(double) * ((size_t)M->nnzb + 1));
  int64_t* off = block_offsets(M);
  if (!nrm || !off) {
    free(nrm);
    free(off);
    return OR_E_NOMEM;
  }
  oracle_norms(M, nrm);
  int64_t nb = 0, nv = 0;
  for (int32_t b = 0; b < M->nnzb; ++b)
    if (eps <= 0.0 || nrm[b] > eps) {
      ++nb;
      nv += off[b + 1] - off[b];
    }
  counts[0] = nb;
  counts[1] = nv;
  if (nb > cap_nnzb || nv > cap_nvals) {
    free(nrm);
    free(off);
    return OR_E_CAPACITY;
  }
  int64_t ob = 0, ov = 0;
  o_row_ptr[0] = 0;
  for (int32_t i = 0; i < M->nbrows; ++i) {
    for (int32_t b = M->row_ptr[i]; b < M->row_ptr[i + 1]; ++b) {
      if (!(eps <= 0.0 || nrm[b] > eps)) continue;
      o_col_idx[ob++] = M->col_idx[b];
      for (int64_t e = off[b]; e < off[b + 1]; ++e) o_values[ov++] = M->values[e];
    }
    o_row_ptr[i + 1] = (int32_t)ob;
  }
  free(nrm);
  free(off);
  return OR_OK;
}

/* Frobenius norm of a whole matrix: plain sum of squares over all stored
 * values in storage order, then the square root (sign-iteration residual). */
double oracle_frobenius(const oracle_mat* M) {
  int64_t n = oracle_value_count(M);
  double s = 0.0;
  for (int64_t e = 0; e < n; ++e) s = s + M->values[e] * M->values[e];
  return sqrt(s);
}
