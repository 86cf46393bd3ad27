"""The sign chain at its configured size, teacher-forced against the oracle.

2048 molecules as 23x23 blocks (N = 47,104), 12 Newton-Schulz steps with the
on-the-fly filter and a filter of every result at 1e-7, then the residual
multiply.  The chain runs eagerly through the C-ABI; after the two multiplies
of chosen steps (sparse, filling in, dense) and after the residual multiply,
the GPU's own inputs of that multiply are read back and the oracle multiplies
the same sampled block rows of them.  The GPU's output rows must match:
pattern exact, values within the FP64 tolerance (1e-12 relative Frobenius
over the sampled rows).  The dense steps have rows of 2048 blocks (the huge
symbolic forms) and 8.6 G candidate products, built and consumed in stack
panels; their product stacks are not kept, so the stacks are not compared
here (the panel tests compare panelled results with whole-stack ones bit for
bit).
"""
import time

import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import bsmm
from paper_1708_03604_amd import workloads as W
from test_gpu_parity import REL_TOL, rel_err, take_rows

pytestmark = pytest.mark.gpu

NMOL = 2048
CHECK_STEPS = (0, 3, 7, 11, 12)  # 12: the residual multiply
ROWS = sorted({0, NMOL - 1} | set(np.random.default_rng(2048).choice(NMOL, 3, replace=False).tolist()))


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def host(M):
    rp, ci, v = M.to_host()
    return W.with_pattern(M.row_sizes, M.col_sizes, rp, ci, v)


def check_rows(alpha, A, B, beta, Cin, C, eps):
    """Oracle on rows ROWS of the host copies of one multiply's operands
    against the same rows of its GPU result; returns (max blocks per sampled
    row, relative Frobenius error over the sampled rows)."""
    Asub = take_rows(A, ROWS)[0]
    Csub = take_rows(Cin, ROWS)[0] if (beta != 0.0 and Cin is not None) else None
    ref = oracle.multiply(alpha, Asub, B, beta, Csub, eps)
    got = take_rows(C, ROWS)[0]
    assert np.array_equal(np.asarray(got.row_ptr), np.asarray(ref.row_ptr)), "pattern: row lengths"
    assert np.array_equal(np.asarray(got.col_idx), np.asarray(ref.col_idx)), "pattern: block columns"
    err = rel_err(np.asarray(got.values), np.asarray(ref.values))
    assert err <= REL_TOL, f"relative Frobenius error {err:.3e}"
    return int(np.diff(np.asarray(ref.row_ptr)).max()), err


@pytest.mark.timeout(900)
def test_sign_chain_2048_teacher_forced():
    from paper_1708_03604_amd.chain import SignChain
    X0, _ = W.symmetric_scaled(nmol=NMOL)
    ch = SignChain(X0, steps=12, eps=1e-7)
    seen = []
    t0 = time.time()

    def after(step, args):
        if step not in CHECK_STEPS:
            return
        alpha, A, B, beta, Cin, C, eps = args
        Ah = host(A)
        Bh = Ah if B is A else host(B)
        Ch = host(C)
        Cinh = host(Cin) if Cin is not None else None
        width, err = check_rows(alpha, Ah, Bh, beta, Cinh, Ch, eps)
        seen.append((step, width, err))
        print(f"step {step}: sampled rows up to {width} blocks, rel. error {err:.2e}, "
              f"{time.time() - t0:.0f} s", flush=True)

    ch.count_flops(after_multiply=after)
    ch.close()
    assert [s for s, _, _ in seen] == [0, 0, 3, 3, 7, 7, 11, 11, 12]
    # the dense end of the chain went through rows beyond the ordinary forms
    assert max(w for _, w, _ in seen) > 1024
