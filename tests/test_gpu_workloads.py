"""Second workloads against the oracle, through the C-ABI: the S-E-shaped
6x6 input (very sparse, large block count, filter on), the H2O-64-shaped
fully occupied input with mixed 9/22/32 blocks, and the streaming block
products of the size sweep (m = n = k from 4 to 78).  Same bar as the main
parity tests: pattern and stack bit-exact, FP64 values within 1e-12 relative
Frobenius."""
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


def test_semi_empirical_small_full():
    w = W.semi_empirical(nmol=3000)
    got = gpu_multiply(w.A, w.B, None, w.alpha, w.beta, w.eps)
    assert 0 < got[4]["products"] < got[4]["candidates"]
    assert got[4]["path"] == bsmm.BSMM_PATH_SMALL
    check(oracle.multiply(w.alpha, w.A, w.B, w.beta, None, w.eps), got)


def test_semi_empirical_full_size():
    # the S-E-shaped workload at full size, every row: 234 M products, the
    # oracle's share is about 13 s on 16 host threads
    w = W.semi_empirical()
    got = gpu_multiply(w.A, w.B, None, w.alpha, w.beta, w.eps)
    print(f"S-E: {got[4]['candidates']} candidates, {got[4]['products']} products, {got[4]['nnzb']} C blocks")
    check(oracle.multiply(w.alpha, w.A, w.B, w.beta, None, w.eps), got)


def test_mixed_dense_full_size():
    w = W.mixed_dense()
    got = gpu_multiply(w.A, w.B, w.C_old, w.alpha, w.beta, w.eps)
    assert got[4]["products"] == 64 ** 3 and got[4]["nnzb"] == 64 * 64
    check(oracle.multiply(w.alpha, w.A, w.B, w.beta, w.C_old, w.eps), got)


def test_mixed_dense_small_full():
    w = W.mixed_dense(nb=9)
    check(oracle.multiply(w.alpha, w.A, w.B, w.beta, w.C_old, w.eps),
          gpu_multiply(w.A, w.B, w.C_old, w.alpha, w.beta, w.eps))


@pytest.mark.parametrize("s", [4, 6, 16, 17, 22, 23, 24, 32, 33, 45, 78])
def test_block_stream(s):
    w = W.block_stream(8000 + s, s, s, s, 37)
    check(oracle.multiply(w.alpha, w.A, w.B, w.beta, w.C_old, w.eps),
          gpu_multiply(w.A, w.B, w.C_old, w.alpha, w.beta, w.eps))


@pytest.mark.parametrize("mnk", [(9, 22, 32), (32, 9, 22), (22, 32, 9), (1, 32, 32), (32, 1, 17)])
def test_block_stream_rectangular(mnk):
    m, n, k = mnk
    w = W.block_stream(8100, m, n, k, 29)
    check(oracle.multiply(w.alpha, w.A, w.B, w.beta, w.C_old, w.eps),
          gpu_multiply(w.A, w.B, w.C_old, w.alpha, w.beta, w.eps))
