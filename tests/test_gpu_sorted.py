"""Filtered multiplies over long B rows, through the C-ABI.

When a multiply has a filter and its B operand averages at least 48 blocks
per block row, the symbolic pass walks, for each A entry, only the kept
prefix of its B row taken in descending norm order.  The norm product is
monotone in the B norm, so the filter keeps exactly such a prefix (Section 2,
the on-the-fly filter).  B rows of more than 2048 blocks keep their stored
order, and every product on them is tested.  Pattern, product stack and
product count must equal the oracle's exactly and values must agree within
the FP64 tolerance.  The reported candidates must still count every product
before the filter.
"""
import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import bsmm
from paper_1708_03604_amd import workloads as W
from test_gpu_parity import check, gpu_multiply

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def candidates(A, B):
    """Block products before the filter: every A entry times its B row."""
    blen = np.diff(np.asarray(B.row_ptr))
    return int(blen[np.asarray(A.col_idx)].sum())


def norm_quantile(A, B, q):
    """A filter threshold near quantile q of the candidates' norm products."""
    na, nb = oracle.norms(A), oracle.norms(B)
    rng = np.random.default_rng(7)
    prod = rng.choice(na, 4000) * rng.choice(nb, 4000)
    return float(np.quantile(prod, q))


@pytest.mark.parametrize("q", [0.0, 0.3, 0.8, 0.99])
@pytest.mark.parametrize("sizes", ["uniform2", "mixed"])
def test_kept_prefixes_match_oracle(q, sizes):
    nb = 160
    if sizes == "uniform2":
        rs = ks = cs = [2] * nb
    else:
        rs, ks, cs = [1, 3, 2, 5] * (nb // 4), [2, 1, 4] * (nb // 3) + [1], [3, 1, 2, 2] * (nb // 4)
    A = W.random_matrix(811, rs, ks, 0.4)
    B = W.random_matrix(812, ks, cs, 0.45)
    Co = W.random_matrix(813, rs, cs, 0.2)
    assert len(B.col_idx) >= 48 * len(ks)  # long B rows: the kept-prefix walk
    eps = norm_quantile(A, B, q) if q > 0 else 1e-300
    ref = oracle.multiply(0.5, A, B, -1.0, Co, eps)
    got = gpu_multiply(A, B, Co, 0.5, -1.0, eps)
    check(ref, got)
    assert got[4]["candidates"] == candidates(A, B)


def test_rows_beyond_the_sort_length():
    # B rows 0 and 1 hold 2500 blocks (stored order, every product tested),
    # rows 2 and 3 hold 60 (norm order); 1x1 blocks whose magnitude falls
    # with the column, so the filter keeps under 2048 columns per C row
    ncol = 2500
    rng = np.random.default_rng(821)
    cols = [np.arange(ncol), np.arange(ncol), np.sort(rng.choice(ncol, 60, replace=False)),
            np.sort(rng.choice(ncol, 60, replace=False))]
    rp = np.concatenate(([0], np.cumsum([len(c) for c in cols])))
    ci = np.concatenate(cols)
    vals = rng.uniform(0.5, 1.0, len(ci)) * np.exp(-ci / 400.0) * rng.choice([-1.0, 1.0], len(ci))
    B = W.with_pattern(np.ones(4, dtype=np.int32), np.ones(ncol, dtype=np.int32), rp, ci, vals)
    nA = 40
    A = W.with_pattern(np.ones(nA, dtype=np.int32), np.ones(4, dtype=np.int32),
                       np.arange(0, 4 * nA + 1, 4), np.tile(np.arange(4), nA),
                       rng.uniform(0.2, 1.0, 4 * nA))
    eps = 0.05
    ref = oracle.multiply(1.0, A, B, 0.0, None, eps)
    assert np.diff(np.asarray(ref.row_ptr)).max() <= 2048
    assert 0 < len(ref.stack) < candidates(A, B)
    got = gpu_multiply(A, B, None, 1.0, 0.0, eps)
    check(ref, got)
    assert got[4]["candidates"] == candidates(A, B)
