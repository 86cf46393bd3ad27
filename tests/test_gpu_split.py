"""Split-precision multiply (three BF16 terms per value on matrix cores)
against the FP64 oracle, through the C-ABI.

The symbolic phase, norms and filter decisions are FP64 in both modes, so the
pattern and the product stack must match the oracle bit for bit.  The values
carry the error of the split: per C element

    |c - c_ref| <= 2^-15 * |alpha| * (|A| |B|)_ij + 2^-50 * (|alpha| (|A||B|)_ij + |beta| |C_in|_ij)

where |A||B| is the oracle's product of the absolute values over the same
kept block products (absolute values have the same block norms, so the
filter keeps the same products).  The 2^-15 term covers the dropped term
products (about 2^-22) and FP32 accumulation of 6 x 32 terms per block
product (192 * 2^-24); the last term covers FP64 rounding.
"""
import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import bsmm
from paper_1708_03604_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def absm(M):
    return W.with_pattern(M.row_sizes, M.col_sizes, M.row_ptr, M.col_idx, np.abs(M.values))


def gpu_split(A, B, Co, alpha, beta, eps):
    dA = bsmm.Matrix.from_csr(A)
    dB = bsmm.Matrix.from_csr(B)
    dCin = bsmm.Matrix.from_csr(Co) if Co is not None else None
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(alpha, dA, dB, beta, dCin, dC, eps, prec=bsmm.BSMM_SPLIT_BF16X3)
    out = dC.to_host() + (dC.stack(),)
    for m in (dA, dB, dCin, dC):
        if m is not None:
            m.close()
    return out


def check_split(A, B, Co, alpha, beta, eps):
    rp, ci, v, st = gpu_split(A, B, Co, alpha, beta, eps)
    ref = oracle.multiply(alpha, A, B, beta, Co if beta else None, eps)
    assert np.array_equal(rp, ref.row_ptr)
    assert np.array_equal(ci, ref.col_idx)
    assert np.array_equal(st, ref.stack.reshape(-1, 3))
    use_c = bool(beta) and Co is not None
    mag = oracle.multiply(abs(alpha), absm(A), absm(B), abs(beta), absm(Co) if use_c else None, eps)
    # |alpha| |A||B| on the result pattern: C_in's pattern with zero values
    Z = W.with_pattern(Co.row_sizes, Co.col_sizes, Co.row_ptr, Co.col_idx, np.zeros(Co.nvals)) if use_c else None
    pm = oracle.multiply(abs(alpha), absm(A), absm(B), 1.0 if use_c else 0.0, Z, eps)
    assert np.array_equal(mag.col_idx, ref.col_idx) and np.array_equal(pm.col_idx, ref.col_idx)
    pmag = pm.values
    bound = 2.0 ** -15 * pmag + 2.0 ** -50 * mag.values
    err = np.abs(v - ref.values)
    assert np.all(err <= bound), f"max excess {np.max(err - bound)}"
    rel = np.linalg.norm(v - ref.values) / max(np.linalg.norm(ref.values), 1e-300)
    # statistical level of the scheme (measured about 3.5e-8 relative Frobenius
    # and 6e-8 of max |C| on random data): dropping any one of the six term
    # products gives at least about 1e-6 (tests/test_split_scheme.py)
    assert rel <= 1e-7, f"relative Frobenius error {rel:.3e}"
    if err.size:
        assert err.max() <= 1e-6 * max(np.abs(ref.values).max(), 1e-300), f"max-abs error {err.max():.3e}"
    return rel


@pytest.mark.parametrize("alpha,beta,filt", [(1.0, 0.0, 0.0), (-0.75, 1.25, 0.0), (1.0, 1.0, 1.0)])
def test_split_within_bound(alpha, beta, filt):
    sizes = [23] * 24
    A = W.random_matrix(201, sizes, sizes, 0.3)
    B = W.random_matrix(202, sizes, sizes, 0.3)
    Co = W.random_matrix(203, sizes, sizes, 0.2)
    check_split(A, B, Co if beta else None, alpha, beta, filt)


def test_split_scaled_values():
    # wide dynamic range inside blocks: the split terms follow each value's exponent
    sizes = [23] * 12
    A = W.random_matrix(211, sizes, sizes, 0.5)
    B = W.random_matrix(212, sizes, sizes, 0.5)
    rng = np.random.default_rng(7)
    A.values = A.values * np.exp2(rng.integers(-30, 30, size=A.values.size))
    B.values = B.values * np.exp2(rng.integers(-30, 30, size=B.values.size))
    check_split(A, B, None, 1.0, 0.0, 0.0)


def test_split_integers_exact():
    # small integers are exact in one BF16 term and their sums in FP32
    sizes = [23] * 10
    A = W.random_matrix(221, sizes, sizes, 0.5, kind="int")
    B = W.random_matrix(222, sizes, sizes, 0.5, kind="int")
    rp, ci, v, st = gpu_split(A, B, None, 1.0, 0.0, 0.0)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    assert np.array_equal(v, ref.values)


def test_split_three_terms_exact():
    # Values p + q 2^-9 + r 2^-18 (|p|, |q| in 5..7, |r| in 1..7) split into
    # exactly the BF16 terms p, q 2^-9 and r 2^-18, so all six kept term
    # products matter.  A blocks hold one nonzero per row, so every FP32
    # partial sum of a block product stays exact (a multiple of 2^-18 below
    # 2^6) and the result must equal the scheme's sum of the kept term
    # products, sum over i + j <= 2 of S_i(A) S_j(B), bit for bit (each term
    # product by the FP64 oracle, exact here).  Leaving out any one term
    # product changes it (shown on the CPU in tests/test_split_scheme.py).
    sizes = [23] * 12
    A, B, Ap, Bp = W.three_term_pair(241, sizes)
    rp, ci, v, st = gpu_split(A, B, None, 1.0, 0.0, 0.0)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    assert np.array_equal(ci, ref.col_idx)
    want = None
    for i, j in [(0, 2), (1, 1), (2, 0), (0, 1), (1, 0), (0, 0)]:
        Ai = W.with_pattern(A.row_sizes, A.col_sizes, A.row_ptr, A.col_idx, Ap[i])
        Bj = W.with_pattern(B.row_sizes, B.col_sizes, B.row_ptr, B.col_idx, Bp[j])
        t = oracle.multiply(1.0, Ai, Bj, 0.0, None, 0.0).values
        want = t if want is None else want + t
    assert np.array_equal(v, want), f"max abs difference {np.max(np.abs(v - want)):.3e}"
    # the dropped term products (orders 3 and 4, at most 2 * 7*2^-9 * 7*2^-18
    # + 49*2^-36 per product of two values of magnitude >= 5) stay below
    # 2^-24 of |A||B|
    mag = oracle.multiply(1.0, absm(A), absm(B), 0.0, None, 0.0).values
    assert np.all(np.abs(v - ref.values) <= 2.0 ** -24 * mag)


def test_split_rejected_leaves_output_unchanged():
    # a split multiply on 5/13 blocks is rejected before anything is written:
    # the previous result, its pattern and its product stack stay as they were
    A = bsmm.Matrix.from_csr(W.random_matrix(251, [5, 13] * 6, [5, 13] * 6, 0.2))
    B = bsmm.Matrix.from_csr(W.random_matrix(252, [5, 13] * 6, [5, 13] * 6, 0.2))
    Abig = bsmm.Matrix.from_csr(W.random_matrix(253, [5, 13] * 6, [5, 13] * 6, 0.9))
    C = bsmm.Matrix.empty([5, 13] * 6, [5, 13] * 6)
    bsmm.multiply(1.0, A, B, 0.0, None, C, 0.0)
    before = C.to_host() + (C.stack(),)
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.multiply(1.0, Abig, Abig, 0.0, None, C, 0.0, prec=bsmm.BSMM_SPLIT_BF16X3)
    assert e.value.status == "BSMM_E_UNSUPPORTED"
    after = C.to_host() + (C.stack(),)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    for m in (A, B, Abig, C):
        m.close()


def test_split_molecules_full_size():
    # the split-precision form of the benchmark workload at full size, every row
    w = W.molecules()
    rel = check_split(w.A, w.B, w.C_old, w.alpha, w.beta, w.eps)
    print(f"split rel Frobenius error, molecules: {rel:.3e}")
