"""The split-precision scheme, emulated on the CPU, against the assertions of
the GPU split tests (tests/test_gpu_split.py): leaving out any one of the six
BF16 term products must make those assertions fail, so the GPU tests can
detect such a regression.

The emulation restates the scheme from its definition (FP64 value -> three
BF16 terms by repeated round-to-nearest-even of the residual; a block product
keeps the term products s_i(a) s_j(b) with i + j <= 2) in numpy; each term
product is multiplied with the FP64 oracle, so the only error left is the
split's own.  Nothing here runs on or imports the GPU library.
"""
import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import workloads as W

KEPT = [(0, 2), (1, 1), (2, 0), (0, 1), (1, 0), (0, 0)]


def bf16(x):
    """Round FP64 values to BF16 (through FP32, nearest even), as FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def split3(x):
    s0 = bf16(x)
    s1 = bf16(x - s0)
    s2 = bf16(x - s0 - s1)
    return [s0, s1, s2]


def emulate(A, B, terms):
    """sum over (i, j) in terms of S_i(A) S_j(B), each product by the oracle."""
    SA, SB = split3(A.values), split3(B.values)
    out = None
    for i, j in terms:
        Ai = W.with_pattern(A.row_sizes, A.col_sizes, A.row_ptr, A.col_idx, SA[i])
        Bj = W.with_pattern(B.row_sizes, B.col_sizes, B.row_ptr, B.col_idx, SB[j])
        r = oracle.multiply(1.0, Ai, Bj, 0.0, None, 0.0)
        out = r.values.copy() if out is None else out + r.values
    return out


def test_three_term_values_split_exactly():
    x, parts = W.three_term_values(np.random.default_rng(5), 10000)
    s = split3(x)
    for got, want in zip(s, parts):
        assert np.array_equal(got, want)
    assert np.array_equal(parts[0] + parts[1] + parts[2], x)


def test_three_term_case_rejects_each_dropped_term():
    # the exact-equality assertion of test_split_three_terms_exact
    A, B, Ap, Bp = W.three_term_pair(241, [23] * 12)

    def kept_sum(terms):
        out = None
        for i, j in terms:
            Ai = W.with_pattern(A.row_sizes, A.col_sizes, A.row_ptr, A.col_idx, Ap[i])
            Bj = W.with_pattern(B.row_sizes, B.col_sizes, B.row_ptr, B.col_idx, Bp[j])
            t = oracle.multiply(1.0, Ai, Bj, 0.0, None, 0.0).values
            out = t if out is None else out + t
        return out

    want = kept_sum(KEPT)
    assert np.array_equal(emulate(A, B, KEPT), want)
    for drop in KEPT:
        got = emulate(A, B, [t for t in KEPT if t != drop])
        assert not np.array_equal(got, want), f"dropping {drop} went unnoticed"


def test_random_case_rejects_each_dropped_term():
    # the statistical assertions of check_split (relative Frobenius <= 1e-7,
    # max-abs <= 1e-6 of max |C|) on random U[-1,1] 23x23 blocks
    sizes = [23] * 16
    A = W.random_matrix(201, sizes, sizes, 0.3)
    B = W.random_matrix(202, sizes, sizes, 0.3)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0).values
    scale = np.abs(ref).max()

    def passes(v):
        rel = np.linalg.norm(v - ref) / np.linalg.norm(ref)
        return rel <= 1e-7 and np.abs(v - ref).max() <= 1e-6 * scale

    full = emulate(A, B, KEPT)
    rel_full = np.linalg.norm(full - ref) / np.linalg.norm(ref)
    assert rel_full < 2e-8, rel_full   # the split alone, without FP32 accumulation
    assert passes(full)
    for drop in KEPT:
        got = emulate(A, B, [t for t in KEPT if t != drop])
        assert not passes(got), f"dropping {drop} went unnoticed"
