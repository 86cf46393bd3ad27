"""Randomised parity over every kernel path, through the C-ABI.

Each case draws block sizes (from the sets that select the small-block,
23x23, generic and split paths; the "wide" set, every edge at least 16, sends
the generic path's blocks to its matrix-core form), densities, alpha, beta and the filter
threshold from its seed, runs the multiply synchronously and with reserved
capacities, and compares both with the oracle: pattern and stack bit-exact,
FP64 values within 1e-12 relative Frobenius (split precision: within its
stated per-element bound), and the reserved run bit-identical to the
synchronous one.
"""
import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import bsmm
from paper_1708_03604_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZE_SETS = {
    "small": [1, 2, 3, 5, 6, 8, 9, 13, 15, 16],
    "b23": [23],
    "mixed": [4, 9, 17, 22, 23, 32, 40],
    "b5_13": [5, 13],
    "wide": [16, 17, 24, 31, 32, 33, 40, 48, 64],
}


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def draw(seed):
    rng = np.random.default_rng(seed)
    name = sorted(SIZE_SETS)[seed % len(SIZE_SETS)]
    pool = SIZE_SETS[name]
    nr, nk, nc = (int(x) for x in rng.integers(3, 24, 3))
    rs, ks, cs = (rng.choice(pool, n).astype(np.int32) for n in (nr, nk, nc))
    A = W.random_matrix(seed * 10 + 1, rs, ks, float(rng.uniform(0.05, 0.6)))
    B = W.random_matrix(seed * 10 + 2, ks, cs, float(rng.uniform(0.05, 0.6)))
    Co = W.random_matrix(seed * 10 + 3, rs, cs, float(rng.uniform(0.0, 0.5)))
    alpha = float(rng.choice([1.0, -0.5, 2.25]))
    beta = float(rng.choice([0.0, 1.0, -1.5]))
    # filter: off, or near the median norm product
    eps = 0.0
    if rng.random() < 0.5 and A.nnzb and B.nnzb:
        eps = float(np.median(oracle.norms(A))) * float(np.median(oracle.norms(B)))
    return name, A, B, Co, alpha, beta, eps


def run(A, B, Co, alpha, beta, eps, prec, reserve):
    dA, dB = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B)
    dCin = bsmm.Matrix.from_csr(Co)
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    if reserve:
        nb = A.nbrows * B.nbcols
        bsmm.bsmm_reserve(dC.handle, max(nb, 1), max(int(A.row_sizes.sum()) * int(B.col_sizes.sum()), 1),
                          max(A.nbrows * A.nbcols * B.nbcols, 1))
    bsmm.multiply(alpha, dA, dB, beta, dCin, dC, eps, prec=prec)
    out = dC.to_host() + (dC.stack(), bsmm.bsmm_stats(dC.handle))
    for m in (dA, dB, dCin, dC):
        m.close()
    return out


@pytest.mark.parametrize("seed", range(30))
def test_random_case(seed):
    name, A, B, Co, alpha, beta, eps = draw(seed)
    ref = oracle.multiply(alpha, A, B, beta, Co if beta != 0.0 else None, eps)
    sync = run(A, B, Co, alpha, beta, eps, bsmm.BSMM_FP64, False)
    rp, ci, v, st, stats = sync
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    assert np.array_equal(st, ref.stack.reshape(-1, 3))
    n = np.linalg.norm(ref.values)
    err = np.linalg.norm(v - ref.values)
    assert err <= 1e-12 * n if n > 0 else err == 0
    res = run(A, B, Co, alpha, beta, eps, bsmm.BSMM_FP64, True)
    for a, b in zip(sync[:4], res[:4]):
        assert np.array_equal(a, b)
    assert sync[4] == res[4]


@pytest.mark.parametrize("seed", range(6))
def test_random_split_case(seed):
    rng = np.random.default_rng(100 + seed)
    nr, nk, nc = (int(x) for x in rng.integers(3, 16, 3))
    A = W.random_matrix(1000 + seed, [23] * nr, [23] * nk, float(rng.uniform(0.1, 0.6)))
    B = W.random_matrix(2000 + seed, [23] * nk, [23] * nc, float(rng.uniform(0.1, 0.6)))
    Co = W.random_matrix(3000 + seed, [23] * nr, [23] * nc, 0.3)
    beta = float(rng.choice([0.0, 1.0]))
    ref = oracle.multiply(1.0, A, B, beta, Co if beta else None, 0.0)
    absm = lambda M: W.with_pattern(M.row_sizes, M.col_sizes, M.row_ptr, M.col_idx, np.abs(M.values))
    Z = W.with_pattern(Co.row_sizes, Co.col_sizes, Co.row_ptr, Co.col_idx, np.zeros(Co.nvals)) if beta else None
    mag = oracle.multiply(1.0, absm(A), absm(B), 1.0 if beta else 0.0, Z, 0.0)
    full = oracle.multiply(1.0, absm(A), absm(B), abs(beta), absm(Co) if beta else None, 0.0)
    got = run(A, B, Co, 1.0, beta, 0.0, bsmm.BSMM_SPLIT_BF16X3, bool(seed % 2))
    assert np.array_equal(got[0], ref.row_ptr) and np.array_equal(got[1], ref.col_idx)
    assert np.all(np.abs(got[2] - ref.values) <= 2.0 ** -15 * mag.values + 2.0 ** -50 * full.values)
