"""The exact-slice precision, emulated on the CPU (tests/slice_model.py),
pinned against things other than itself: values built from known digits
slice back into exactly those digits, every value is rebuilt from its digits
within the stated remainder, the emulated product stays within the stated
error bound of the FP64 oracle, and the bit-exact assertion of the GPU
seven-digit test rejects the result with any one kept digit product left
out.  Nothing here runs on or imports the GPU library."""
import numpy as np
import pytest

import oracle
import slice_model as SM
from paper_1708_03604_amd import workloads as W


def test_seven_digit_values_slice_into_their_digits():
    A, B, DA, DB = W.seven_digit_pair(301, [23] * 6)
    assert np.all(SM.exponents(A, "row") == 0) and np.all(SM.exponents(B, "col") == 0)
    assert np.array_equal(SM.digits(A, "row"), DA)
    assert np.array_equal(SM.digits(B, "col"), DB)


def test_digits_rebuild_every_value():
    # wide dynamic range inside and across rows: the digits rebuild every
    # scaled value within the stated remainder |rho| <= 2^-49
    M = W.random_matrix(302, [23] * 8, [23] * 8, 0.6)
    rng = np.random.default_rng(3)
    M.values = M.values * np.exp2(rng.integers(-40, 40, size=M.values.size))
    M.values[::17] = 0.0
    for by in ("row", "col"):
        D = SM.digits(M, by)
        assert np.abs(D).max() <= 64
        e = SM.exponents(M, by)
        rows, rr, cols, cc = SM._index(M)
        ev = e[rows, rr] if by == "row" else e[cols, cc]
        y = np.ldexp(M.values, -ev)
        assert np.all(np.abs(y) < 1.0)
        rebuilt = np.zeros_like(y)
        for s in range(SM.SLICES - 1, -1, -1):
            rebuilt = rebuilt + np.ldexp(D[s].astype(np.float64), -SM.WEIGHTS[s])
        assert np.all(np.abs(y - rebuilt) <= 2.0 ** -49 * (1 + 2.0 ** -40))
        # the largest value of every nonzero group has |y| in [1/2, 1)
        gm = SM.group_max(M, by)
        assert np.all((gm == 0) | ((np.ldexp(gm, -e) >= 0.5) & (np.ldexp(gm, -e) < 1.0)))


def test_digits_of_special_values():
    # zero rows, a single nonzero, exact powers of two and their negatives
    sizes = [23] * 2
    M = W.random_matrix(303, sizes, sizes, 1.0)
    M.values[:] = 0.0
    M.values[5] = 1.0           # block 0, row 0: max 1 -> scale 2, y = 1/2 -> d1 = 32
    M.values[6] = -0.25         # y = -1/8 -> d1 = -8
    M.values[23 * 23 + 100] = 3.0  # block 1, row 4: y = 3/4 -> d1 = 48
    D = SM.digits(M, "row")
    assert D[0, 5] == 32 and D[0, 6] == -8 and D[0, 23 * 23 + 100] == 48
    assert np.count_nonzero(D[1:]) == 0
    assert np.count_nonzero(D[0]) == 3


@pytest.mark.parametrize("seed,scale", [(311, False), (312, True)])
def test_emulated_product_within_stated_bound(seed, scale):
    sizes = [23] * 12
    A = W.random_matrix(seed, sizes, sizes, 0.4)
    B = W.random_matrix(seed + 1, sizes, sizes, 0.4)
    if scale:
        rng = np.random.default_rng(seed)
        A.values = A.values * np.exp2(rng.integers(-20, 20, size=A.values.size))
        B.values = B.values * np.exp2(rng.integers(-20, 20, size=B.values.size))
    v, pat = SM.emulate(A, B)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    assert np.array_equal(pat.col_idx, ref.col_idx)
    bound = SM.error_bound(A, B, ref, ref.stack, 1.0)
    err = np.abs(v - ref.values)
    assert np.all(err <= bound + 2.0 ** -52 * np.abs(ref.values))
    # far inside the bound on random data; the GPU tests assert this level
    rel = np.linalg.norm(v - ref.values) / np.linalg.norm(ref.values)
    assert rel <= 1e-12


def test_stated_bound_is_reached_in_order_of_magnitude():
    # the bound is not vacuous: leaving out the digit products of degrees 7
    # and 8 (the two smallest kept ones) breaks it on random data
    sizes = [23] * 10
    A = W.random_matrix(321, sizes, sizes, 0.5)
    B = W.random_matrix(322, sizes, sizes, 0.5)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    bound = SM.error_bound(A, B, ref, ref.stack, 1.0)
    no7 = [p for p in SM.KEPT if p[0] + p[1] < 5]
    v7, _ = SM.emulate(A, B, no7)
    assert np.any(np.abs(v7 - ref.values) > bound)


def test_seven_digit_case_rejects_each_dropped_pair():
    # the GPU test compares bit for bit with the full emulation
    A, B, DA, DB = W.seven_digit_pair(331, [23] * 8)
    full, _ = SM.emulate(A, B)
    for p in SM.KEPT:
        partial, _ = SM.emulate(A, B, [q for q in SM.KEPT if q != p])
        assert not np.array_equal(partial, full), f"dropping digit pair {p} not detected"
