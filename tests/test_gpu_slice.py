"""Exact-slice precision (BSMM_SLICE_INT8X7: seven INT8 digits per value on
INT8 matrix cores) through the C-ABI, against the FP64 oracle and against the
CPU model of the scheme (tests/slice_model.py).

The symbolic phase, norms and filter decisions are FP64 as in every mode, so
pattern and product stack must match the oracle bit for bit.  The digit sums
are exact integers and the kernel combines the degrees in a fixed FP64 order,
so with alpha = 1, beta = 0 and no filter the values must equal the CPU model
bit for bit; in every case they must lie within the stated bound of the
oracle, 2^-39 |alpha| n_ij MA(i,r) MB(j,q) per element plus FP64 rounding of
the update, and at the level the scheme reaches on random data (the model
gives about 5e-15 relative Frobenius error; the tests ask for 1e-13).
"""
import numpy as np
import pytest

import oracle
import slice_model as SM
from paper_1708_03604_amd import bsmm
from paper_1708_03604_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_LEVEL = 1e-13


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


def gpu_slice(A, B, Co, alpha, beta, eps):
    dA = bsmm.Matrix.from_csr(A)
    dB = bsmm.Matrix.from_csr(B)
    dCin = bsmm.Matrix.from_csr(Co) if Co is not None else None
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(alpha, dA, dB, beta, dCin, dC, eps, prec=bsmm.BSMM_SLICE_INT8X7)
    assert bsmm.bsmm_stats(dC.handle)["path"] == bsmm.BSMM_PATH_SLICE23
    out = dC.to_host() + (dC.stack(),)
    for m in (dA, dB, dCin, dC):
        if m is not None:
            m.close()
    return out


def check_slice(A, B, Co, alpha, beta, eps):
    rp, ci, v, st = gpu_slice(A, B, Co, alpha, beta, eps)
    ref = oracle.multiply(alpha, A, B, beta, Co if beta else None, eps)
    assert np.array_equal(rp, ref.row_ptr)
    assert np.array_equal(ci, ref.col_idx)
    assert np.array_equal(st, ref.stack.reshape(-1, 3))
    use_c = bool(beta) and Co is not None
    mag = oracle.multiply(abs(alpha), absm(A), absm(B), abs(beta), absm(Co) if use_c else None, eps)
    bound = SM.error_bound(A, B, ref, ref.stack, alpha) + 2.0 ** -50 * mag.values
    err = np.abs(v - ref.values)
    assert np.all(err <= bound), f"max excess {np.max(err - bound)}"
    rel = np.linalg.norm(v - ref.values) / max(np.linalg.norm(ref.values), 1e-300)
    assert rel <= REL_LEVEL, f"relative Frobenius error {rel:.3e}"
    if err.size:
        assert err.max() <= REL_LEVEL * max(np.abs(ref.values).max(), 1e-300), f"max-abs error {err.max():.3e}"
    return v, rel


@pytest.mark.parametrize("alpha,beta,filt", [(1.0, 0.0, 0.0), (-0.75, 1.25, 0.0), (1.0, 1.0, 1.0)])
def test_slice_within_bound(alpha, beta, filt):
    sizes = [23] * 24
    A = W.random_matrix(401, sizes, sizes, 0.3)
    B = W.random_matrix(402, sizes, sizes, 0.3)
    Co = W.random_matrix(403, sizes, sizes, 0.2)
    check_slice(A, B, Co if beta else None, alpha, beta, filt)


def test_slice_equals_cpu_model_bits():
    # several tiles of work with ragged rows: every C element bit for bit
    sizes = [23] * 40
    A = W.random_matrix(411, sizes, sizes, 0.25)
    B = W.random_matrix(412, sizes, sizes, 0.25)
    v, _ = check_slice(A, B, None, 1.0, 0.0, 0.0)
    want, _ = SM.emulate(A, B)
    assert np.array_equal(v, want), f"max abs difference {np.max(np.abs(v - want)):.3e}"


def test_slice_seven_digit_exact():
    # every value made of exactly seven digits (scale 1): the result must be
    # the model's sum of the 28 kept digit products bit for bit; leaving out
    # any one of them changes it (tests/test_slice_scheme.py)
    A, B, DA, DB = W.seven_digit_pair(421, [23] * 12)
    rp, ci, v, st = gpu_slice(A, B, None, 1.0, 0.0, 0.0)
    ref, sums = SM.degree_sums(A, B, DA, DB)
    assert np.array_equal(ci, ref.col_idx)
    want = SM.combine(sums)
    assert np.array_equal(v, want), f"max abs difference {np.max(np.abs(v - want)):.3e}"


def test_slice_scaled_rows_and_columns():
    # powers of two per row of A and per column of B are taken out exactly by
    # the scales: the result is the unscaled result, scaled
    sizes = [23] * 12
    A = W.random_matrix(431, sizes, sizes, 0.5)
    B = W.random_matrix(432, sizes, sizes, 0.5)
    rng = np.random.default_rng(9)
    fr = np.exp2(rng.integers(-60, 60, size=(len(sizes), 23)))
    fc = np.exp2(rng.integers(-60, 60, size=(len(sizes), 23)))
    rows, rr, cols, cc = SM._index(A)
    As = W.with_pattern(A.row_sizes, A.col_sizes, A.row_ptr, A.col_idx, A.values * fr[rows, rr])
    rows, rr, cols, cc = SM._index(B)
    Bs = W.with_pattern(B.row_sizes, B.col_sizes, B.row_ptr, B.col_idx, B.values * fc[cols, cc])
    v0, _ = check_slice(A, B, None, 1.0, 0.0, 0.0)
    v1, _ = check_slice(As, Bs, None, 1.0, 0.0, 0.0)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    rows, rr, cols, cc = SM._index(ref)
    assert np.array_equal(v1, v0 * fr[rows, rr] * fc[cols, cc])


def test_slice_wide_range_inside_rows():
    # magnitudes spread over 2^-30..2^30 inside rows: the bound still holds
    # (it is relative to the row and column maxima)
    sizes = [23] * 12
    A = W.random_matrix(441, sizes, sizes, 0.5)
    B = W.random_matrix(442, sizes, sizes, 0.5)
    rng = np.random.default_rng(11)
    A.values = A.values * np.exp2(rng.integers(-30, 30, size=A.values.size))
    B.values = B.values * np.exp2(rng.integers(-30, 30, size=B.values.size))
    rp, ci, v, st = gpu_slice(A, B, None, 1.0, 0.0, 0.0)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    assert np.array_equal(ci, ref.col_idx)
    bound = SM.error_bound(A, B, ref, ref.stack, 1.0)
    assert np.all(np.abs(v - ref.values) <= bound + 2.0 ** -52 * np.abs(ref.values))
    want, _ = SM.emulate(A, B)
    assert np.array_equal(v, want)


def test_slice_zero_rows_and_empty_result():
    sizes = [23] * 6
    A = W.random_matrix(451, sizes, sizes, 0.6)
    B = W.random_matrix(452, sizes, sizes, 0.6)
    A.values[: 23 * 23] = 0.0        # first block all zero
    B.values[23 * 5: 23 * 9] = 0.0   # rows 5..8 of B's first block
    check_slice(A, B, None, 1.0, 0.0, 0.0)
    # every product filtered out: empty result
    rp, ci, v, st = gpu_slice(A, B, None, 1.0, 0.0, 1e300)
    assert len(ci) == 0 and len(v) == 0


def test_slice_in_place_and_deterministic():
    sizes = [23] * 16
    A = W.random_matrix(461, sizes, sizes, 0.3)
    B = W.random_matrix(462, sizes, sizes, 0.3)
    Co = W.random_matrix(463, sizes, sizes, 0.3)
    ref = oracle.multiply(0.5, A, B, 2.0, Co, 0.0)
    outs = []
    for _ in range(2):
        dA, dB, dC = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B), bsmm.Matrix.from_csr(Co)
        bsmm.multiply(0.5, dA, dB, 2.0, dC, dC, 0.0, prec=bsmm.BSMM_SLICE_INT8X7)
        outs.append(dC.to_host())
        for m in (dA, dB, dC):
            m.close()
    assert np.array_equal(outs[0][1], ref.col_idx)
    assert np.array_equal(outs[0][2], outs[1][2])
    rel = np.linalg.norm(outs[0][2] - ref.values) / np.linalg.norm(ref.values)
    assert rel <= REL_LEVEL


def test_slice_rejected_leaves_output_unchanged():
    A = bsmm.Matrix.from_csr(W.random_matrix(471, [5, 13] * 6, [5, 13] * 6, 0.2))
    B = bsmm.Matrix.from_csr(W.random_matrix(472, [5, 13] * 6, [5, 13] * 6, 0.2))
    Abig = bsmm.Matrix.from_csr(W.random_matrix(473, [5, 13] * 6, [5, 13] * 6, 0.9))
    C = bsmm.Matrix.empty([5, 13] * 6, [5, 13] * 6)
    bsmm.multiply(1.0, A, B, 0.0, None, C, 0.0)
    before = C.to_host() + (C.stack(),)
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.multiply(1.0, Abig, Abig, 0.0, None, C, 0.0, prec=bsmm.BSMM_SLICE_INT8X7)
    assert e.value.status == "BSMM_E_UNSUPPORTED"
    after = C.to_host() + (C.stack(),)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    for m in (A, B, Abig, C):
        m.close()


def test_slice_molecules_full_size():
    # the benchmark workload at full size, every row
    w = W.molecules()
    v, rel = check_slice(w.A, w.B, w.C_old, w.alpha, w.beta, w.eps)
    print(f"slice rel Frobenius error, molecules: {rel:.3e}")
