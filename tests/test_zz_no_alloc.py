"""bsmm_filter_noalloc, the entry point that allocates nothing, against
bsmm_filter through the C-ABI: the same pattern and values bit for bit (the
filter is exact: fixed-order norms, a comparison, copies), on two calls in a
row whose second matrix is smaller, for an unreserved and a reserved matrix.
Both calls share the library's one scratch array on this GPU."""
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


def _cases():
    big = W.random_matrix(901, [23] * 40 + [5, 13] * 20, [23] * 40 + [5, 13] * 20, 0.35)
    small = W.random_matrix(902, [23] * 12 + [13] * 6, [23] * 12 + [13] * 6, 0.3)
    out = []
    for M in (big, small):
        nb = oracle.norms(M)
        out.append((M, float(np.median(nb))))
    assert out[1][0].nnzb < out[0][0].nnzb and out[1][0].nvals < out[0][0].nvals
    return out


@pytest.mark.parametrize("reserve", [False, True])
def test_filter_noalloc_matches_filter(reserve):
    for M, eps in _cases():
        ref = bsmm.Matrix.from_csr(M)
        bsmm.bsmm_filter(ref.handle, eps)
        got = bsmm.Matrix.from_csr(M)
        if reserve:
            bsmm.bsmm_reserve(got.handle, M.nnzb, M.nvals, 1)
        else:
            # a keep-all filter gives the matrix its second storage at this size
            bsmm.bsmm_filter(got.handle, -1.0)
        bsmm.bsmm_filter_noalloc(got.handle, eps)
        rp0, ci0, v0 = ref.to_host()
        rp1, ci1, v1 = got.to_host()
        assert np.array_equal(rp0, rp1) and np.array_equal(ci0, ci1) and np.array_equal(v0, v1)
        want = oracle.filter(M, eps)
        assert np.array_equal(rp1, want.row_ptr) and np.array_equal(ci1, want.col_idx)
        assert np.array_equal(v1, want.values)
        assert 0 < len(ci1) < M.nnzb
        ref.close()
        got.close()


def test_filter_noalloc_rejects_without_storage():
    M = W.random_matrix(903, [23] * 8, [23] * 8, 0.5)
    m = bsmm.Matrix.from_csr(M)
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.bsmm_filter_noalloc(m.handle, 1.0)
    assert e.value.status == "BSMM_E_CAPACITY"
    rp, ci, v = m.to_host()
    assert np.array_equal(ci, M.col_idx) and np.array_equal(v, M.values)
    m.close()
