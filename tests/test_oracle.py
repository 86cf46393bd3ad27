"""Pins of the CPU oracle against things other than itself: hand-computed
worked examples, closed forms, dense brute force through numpy, integer
exactness, invariants (identity, permutation, transpose, linearity, block
splitting) and the filter rule (ties, monotonicity, error bound).

All of these run on the CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from helpers import (brute_products, dense, frob_norms_numpy, from_dense, mask, permute,
                     transpose)
from paper_1708_03604_amd.workloads import BlockCSR, identity_like, random_matrix, with_pattern

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mat(d):
    return BlockCSR(d["row_sizes"], d["col_sizes"], d["row_ptr"], d["col_idx"],
                    np.array(d["values"], dtype=np.float64))


# ------------------------------------------------------------------ golden

def test_hand_example():
    g = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    A, B, Cold = _mat(g["A"]), _mat(g["B"]), _mat(g["Cold"])
    for case in g["cases"]:
        C = oracle.multiply(case["alpha"], A, B, case["beta"], Cold if case["beta"] else None,
                            case["eps"])
        assert C.row_ptr.tolist() == case["row_ptr"]
        assert C.col_idx.tolist() == case["col_idx"]
        assert C.values.tolist() == [float(v) for v in case["values"]]
        assert C.stack.tolist() == case["stack"]


def test_norm_closed_forms():
    g = json.load(open(os.path.join(GOLDEN, "norm_cases.json")))
    for case in g["cases"]:
        m, n = case["shape"]
        if "fill_hex" in case:
            vals = np.full(m * n, float.fromhex(case["fill_hex"]))
        else:
            vals = np.array([float.fromhex(h) for h in case["values_hex"]])
        M = BlockCSR([m], [n], [0, 1], [0], vals)
        got = oracle.norms(M)[0]
        assert got == float.fromhex(case["norm_hex"]), case["name"]


def test_norms_match_numpy_within_ulps():
    rng_sizes = [1, 2, 5, 13, 23, 30]
    M = random_matrix(11, rng_sizes, rng_sizes[::-1], 0.8)
    got = oracle.norms(M)
    ref = frob_norms_numpy(M)
    np.testing.assert_allclose(got, ref, rtol=4e-16 * 8, atol=0)


# -------------------------------------------------------- dense brute force

SIZE_SETS = [
    ([23] * 4, [23] * 3, [23] * 5),
    ([5, 13, 13, 5], [13, 5, 5], [5, 13, 5, 13, 5]),
    ([1, 2, 3], [4, 1], [2, 2, 1]),
    ([6] * 6, [6] * 6, [6] * 6),
]


@pytest.mark.parametrize("sizes", SIZE_SETS)
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-0.5, 1.5), (2.0, 1.0)])
def test_unfiltered_equals_dense(sizes, alpha, beta):
    rs, ks, cs = sizes
    A = random_matrix(101, rs, ks, 0.5)
    B = random_matrix(102, ks, cs, 0.5)
    Co = random_matrix(103, rs, cs, 0.3)
    C = oracle.multiply(alpha, A, B, beta, Co if beta else None, 0.0)
    # pattern: boolean product of masks, union old pattern
    pm = (mask(A).astype(int) @ mask(B).astype(int)) > 0
    if beta:
        pm |= mask(Co)
    assert np.array_equal(mask(C), pm)
    ref = alpha * (dense(A) @ dense(B)) + (beta * dense(Co) if beta else 0.0)
    got = dense(C)
    scale = np.abs(dense(A)) @ np.abs(dense(B))
    assert np.all(np.abs(got - ref) <= 1e-13 * (abs(alpha) * scale + abs(beta) + 1e-300))


@pytest.mark.parametrize("sizes", SIZE_SETS)
def test_integer_inputs_bit_exact(sizes):
    rs, ks, cs = sizes
    A = random_matrix(201, rs, ks, 0.6, kind="int")
    B = random_matrix(202, ks, cs, 0.6, kind="int")
    Co = random_matrix(203, rs, cs, 0.4, kind="int")
    C = oracle.multiply(3.0, A, B, -2.0, Co, 0.0)
    ref = 3.0 * (dense(A) @ dense(B)) - 2.0 * dense(Co)
    assert np.array_equal(dense(C), ref)


def test_empty_operands():
    A = with_pattern([3, 4], [5], [0, 0, 0], [])
    B = random_matrix(5, [5], [2, 2], 1.0)
    C = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    assert C.nnzb == 0 and C.row_ptr.tolist() == [0, 0, 0] and len(C.stack) == 0
    # beta != 0 with empty product: the result is beta * Cold on Cold's pattern
    Co = random_matrix(6, [3, 4], [2, 2], 1.0)
    C = oracle.multiply(1.0, A, B, 0.5, Co, 0.0)
    assert np.array_equal(C.col_idx, Co.col_idx)
    assert np.array_equal(C.values, 0.5 * Co.values)


def test_beta_zero_never_reads_cold():
    A = random_matrix(7, [4, 4], [4, 4], 1.0)
    B = random_matrix(8, [4, 4], [4, 4], 1.0)
    Co = random_matrix(9, [4, 4], [4, 4], 1.0)
    Co.values[:] = np.nan
    C = oracle.multiply(1.0, A, B, 0.0, Co, 0.0)
    assert np.all(np.isfinite(C.values))


# --------------------------------------------------------------- the stack

@pytest.mark.parametrize("eps", [0.0, 0.5, 2.0])
def test_stack_equals_brute_force(eps):
    sizes = [5, 13, 5, 13, 5, 23]
    A = random_matrix(301, sizes, sizes, 0.5)
    B = random_matrix(302, sizes, sizes, 0.5)
    nA, nB = frob_norms_numpy(A), frob_norms_numpy(B)
    # keep clear of ties: numpy norms may differ from the oracle's in the last ulp
    prods = [nA[p] * nB[q] for i in range(A.nbrows) for p in range(A.row_ptr[i], A.row_ptr[i + 1])
             for q in range(B.row_ptr[A.col_idx[p]], B.row_ptr[A.col_idx[p] + 1])]
    assert all(abs(x - eps) > 1e-12 for x in prods)
    C = oracle.multiply(1.0, A, B, 0.0, None, eps)
    ref = brute_products(A, B, nA, nB, eps)
    ref.sort(key=lambda t: (t[0], t[2], t[1]))  # C row, C column, then k
    # map (i, j) to C block index
    cidx = {}
    for i in range(C.nbrows):
        for c in range(C.row_ptr[i], C.row_ptr[i + 1]):
            cidx[(i, C.col_idx[c])] = c
    expect = [(cidx[(i, j)], p, q) for (i, k, j, p, q) in ref]
    assert C.stack.tolist() == [list(t) for t in expect]
    # pattern is exactly the set of (i, j) with a kept product
    assert sorted(cidx) == sorted({(i, j) for (i, k, j, p, q) in ref})


# ------------------------------------------------------------- invariants

def test_identity_is_neutral_bit_exact():
    sizes = [23, 5, 13, 23]
    A = random_matrix(401, sizes, sizes, 0.5)
    I = identity_like(with_pattern(sizes, sizes, [0] * 5, []))
    C = oracle.multiply(1.0, A, I, 0.0, None, 0.0)
    assert np.array_equal(C.row_ptr, A.row_ptr)
    assert np.array_equal(C.col_idx, A.col_idx)
    assert np.array_equal(C.values, A.values)
    C = oracle.multiply(1.0, I, A, 0.0, None, 0.0)
    assert np.array_equal(C.values, A.values)


def test_permutation_invariance():
    sizes = np.array([23, 5, 13, 23, 5, 13])
    A = random_matrix(501, sizes, sizes, 0.5, kind="int")
    B = random_matrix(502, sizes, sizes, 0.5, kind="int")
    p = np.array([3, 0, 5, 1, 4, 2])
    C = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    Cp = oracle.multiply(1.0, permute(A, p), permute(B, p), 0.0, None, 0.0)
    PC = permute(C, p)
    assert np.array_equal(mask(Cp), mask(PC))
    assert np.array_equal(dense(Cp), dense(PC))


def test_transpose_identity():
    rs, ks, cs = [5, 13, 23], [13, 5], [23, 5, 5, 13]
    A = random_matrix(601, rs, ks, 0.6, kind="int")
    B = random_matrix(602, ks, cs, 0.6, kind="int")
    C = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    Ct = oracle.multiply(1.0, transpose(B), transpose(A), 0.0, None, 0.0)
    assert np.array_equal(mask(Ct), mask(C).T)
    assert np.array_equal(dense(Ct), dense(C).T)


def test_linearity_integer():
    sizes = [5, 13, 5]
    A = random_matrix(701, sizes, sizes, 0.7, kind="int")
    B = random_matrix(702, sizes, sizes, 0.7, kind="int")
    Co = random_matrix(703, sizes, sizes, 0.7, kind="int")
    C1 = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    C3 = oracle.multiply(3.0, A, B, 0.0, None, 0.0)
    assert np.array_equal(C3.values, 3.0 * C1.values)
    Cb = oracle.multiply(2.0, A, B, -4.0, Co, 0.0)
    assert np.array_equal(dense(Cb), 2.0 * dense(C1) - 4.0 * dense(Co))


def test_block_splitting_same_dense_result():
    # one 23-block split into 10 + 13 in every dimension gives the same dense product
    A = random_matrix(801, [23, 23], [23, 23, 23], 0.7, kind="int")
    B = random_matrix(802, [23, 23, 23], [23, 23], 0.7, kind="int")
    C = oracle.multiply(1.0, A, B, 0.0, None, 0.0)

    def split(M, split_rows, split_cols):
        rs = np.array([s for x in M.row_sizes for s in ((10, 13) if split_rows else (x,))])
        cs = np.array([s for x in M.col_sizes for s in ((10, 13) if split_cols else (x,))])
        mk = mask(M)
        if split_rows:
            mk = np.repeat(mk, 2, axis=0)
        if split_cols:
            mk = np.repeat(mk, 2, axis=1)
        return from_dense(dense(M), rs, cs, mk)

    Cs = oracle.multiply(1.0, split(A, True, True), split(B, True, True), 0.0, None, 0.0)
    assert np.array_equal(dense(Cs), dense(C))


# ------------------------------------------------------------ filter rule

def _single(value, m, n):
    return BlockCSR([m], [n], [0, 1], [0], np.array([value] + [0.0] * (m * n - 1)))


def test_filter_tie_is_dropped():
    # norms exactly 2 and 2: the norm product is exactly 4
    A = _single(2.0, 3, 4)
    B = _single(-2.0, 4, 5)
    C = oracle.multiply(1.0, A, B, 0.0, None, 4.0)
    assert C.nnzb == 0 and len(C.stack) == 0
    C = oracle.multiply(1.0, A, B, 0.0, None, np.nextafter(4.0, 0.0))
    assert C.nnzb == 1 and len(C.stack) == 1
    assert C.values[0] == -4.0


def test_filter_does_not_depend_on_alpha():
    A = _single(2.0, 2, 2)
    B = _single(2.0, 2, 2)
    for alpha in (1.0, 0.5, -1.0, 1e-300):
        assert oracle.multiply(alpha, A, B, 0.0, None, 3.9).nnzb == 1
        assert oracle.multiply(alpha, A, B, 0.0, None, 4.0).nnzb == 0


def test_filter_monotone_and_error_bound():
    sizes = [23] * 6
    A = random_matrix(901, sizes, sizes, 0.6)
    B = random_matrix(902, sizes, sizes, 0.6)
    nA, nB = frob_norms_numpy(A), frob_norms_numpy(B)
    C0 = oracle.multiply(1.5, A, B, 0.0, None, 0.0)
    prev = None
    for eps in [0.0, 10.0, 30.0, 60.0, 90.0, 1e9]:
        Ce = oracle.multiply(1.5, A, B, 0.0, None, eps)
        s_e = {tuple(t) for t in Ce.stack.tolist()}
        # map stack entries to (a, b) pairs (C index differs between patterns)
        ab_e = {(a, b) for (_, a, b) in s_e}
        if prev is not None:
            assert ab_e <= prev
            assert np.all(mask(Ce) <= prev_mask)
        prev, prev_mask = ab_e, mask(Ce)
        dropped = {(a, b) for (_, a, b) in C0.stack.tolist()} - ab_e
        bound = 1.5 * sum(nA[a] * nB[b] for (a, b) in dropped)
        diff = np.linalg.norm(dense(Ce) - dense(C0))
        assert diff <= bound * (1 + 1e-12) + 1e-12


def test_filter_function():
    sizes = [5, 13, 23]
    M = random_matrix(1001, sizes, sizes, 1.0)
    n = np.sort(frob_norms_numpy(M))
    eps = 0.5 * (n[len(n) // 2] + n[len(n) // 2 + 1])  # between two norms, far from a tie
    F = oracle.filter(M, eps)
    keep = frob_norms_numpy(M) > eps
    ref = from_dense(dense(M), M.row_sizes, M.col_sizes, _keepmask(M, keep))
    assert np.array_equal(F.row_ptr, ref.row_ptr)
    assert np.array_equal(F.col_idx, ref.col_idx)
    assert np.array_equal(F.values, ref.values)
    # eps <= 0 keeps everything (even all-zero blocks); any positive eps drops zero blocks
    Z = with_pattern([2, 2], [2, 2], [0, 1, 2], [1, 0])
    assert oracle.filter(Z, 0.0).nnzb == 2
    assert oracle.filter(Z, 1e-300).nnzb == 0


def _keepmask(M, keep):
    out = np.zeros((M.nbrows, M.nbcols), dtype=bool)
    rows = M.block_rows()
    out[rows[keep], M.col_idx[keep]] = True
    return out


def test_frobenius():
    M = BlockCSR([1, 1], [2], [0, 1, 2], [0, 0], np.array([3.0, 0.0, 0.0, 4.0]))
    assert oracle.frobenius(M) == 5.0
    M = random_matrix(1101, [23, 5], [13, 23], 1.0)
    assert math.isclose(oracle.frobenius(M), np.linalg.norm(dense(M)), rel_tol=1e-14)


# -------------------------------------------------------------- validation

def test_validation_codes():
    good = random_matrix(1201, [2, 3], [4, 1], 1.0)
    assert oracle.check(good) == oracle.OK
    bad = BlockCSR([2, 3], [4, 1], [0, 2, 1], [0, 1, 0], np.zeros(1))
    assert oracle.check(bad) == oracle.E_PATTERN  # row_ptr not monotone
    bad = BlockCSR([2, 3], [4, 1], [0, 2, 3], [1, 0, 0], np.zeros(1))
    assert oracle.check(bad) == oracle.E_PATTERN  # unsorted columns
    bad = BlockCSR([2, 3], [4, 1], [0, 2, 3], [0, 0, 0], np.zeros(1))
    assert oracle.check(bad) == oracle.E_PATTERN  # duplicate column
    bad = BlockCSR([2, 3], [4, 1], [0, 1, 2], [0, 2], np.zeros(1))
    assert oracle.check(bad) == oracle.E_PATTERN  # column out of range
    bad = BlockCSR([2, 0], [4, 1], [0, 1, 2], [0, 1], np.zeros(1))
    assert oracle.check(bad) == oracle.E_ARG  # zero block size
    A = random_matrix(1202, [2, 3], [4, 1], 1.0)
    B = random_matrix(1203, [4, 2], [3], 1.0)  # inner sizes 4,1 vs 4,2
    with pytest.raises(oracle.OracleError) as e:
        oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    assert e.value.code == oracle.E_SHAPE
    with pytest.raises(oracle.OracleError) as e:
        oracle.multiply(1.0, A, A, 0.0, None, float("nan"))
    assert e.value.code in (oracle.E_ARG, oracle.E_SHAPE)


def test_threads_do_not_change_results():
    import subprocess, sys
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(0, %r);"
            "import numpy as np, oracle;"
            "from paper_1708_03604_amd.workloads import random_matrix;"
            "s=[23]*12; A=random_matrix(1, s, s, .4); B=random_matrix(2, s, s, .4);"
            "C=oracle.multiply(1.0, A, B, 0.0, None, 30.0);"
            "sys.stdout.write(C.values.tobytes().hex()[:4000] + str(C.values.sum().hex()))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.check_output([sys.executable, "-c", code % (root, root)], env=env))
    assert outs[0] == outs[1]
