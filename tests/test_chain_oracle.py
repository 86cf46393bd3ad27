"""Pins of the Newton-Schulz chain as run with the oracle (CPU).

The chain alternates T = 3I - X X and X <- 1/2 X T.  For a block-diagonal
X0 = lambda*I every multiply has one nonzero product per diagonal entry, so
each diagonal entry follows the scalar recursion x <- 1/2 x (3 - x^2)
rounded exactly as the oracle rounds it, the off-diagonal entries of the
diagonal blocks stay exactly zero, and ||X X - I||_F = sqrt(N) |x^2 - 1|.
For the same X0 with a sign change on half the blocks the iteration
converges to the signs (+1 / -1) and the residual to 0.
"""
import math

import numpy as np
import pytest

from helpers import dense, oracle_sign_chain
from paper_1708_03604_amd.workloads import identity_like, random_matrix, with_pattern


def scalar_ns(x, steps):
    for _ in range(steps):
        t = 3.0 - x * x
        x = 0.5 * (x * t)
    return x


@pytest.mark.parametrize("lam,steps", [(0.3, 12), (0.9, 5), (1e-3, 3)])
def test_block_diagonal_follows_scalar_recursion(lam, steps):
    sizes = [23, 5, 13, 23]
    X0 = identity_like(random_matrix(0, sizes, sizes, 0.0), lam)
    X, res = oracle_sign_chain(X0, steps, 0.0)
    x = scalar_ns(lam, steps)
    D = dense(X)
    assert np.array_equal(np.diag(D), np.full(D.shape[0], x))
    assert np.count_nonzero(D - np.diag(np.diag(D))) == 0
    n = D.shape[0]
    assert math.isclose(res, math.sqrt(n) * abs(x * x - 1.0), rel_tol=1e-14)


def test_converges_to_signs():
    sizes = [23] * 4 + [5] * 4
    vals = []
    for b, s in enumerate(sizes):
        vals.append(((-1.0) ** b) * 0.4 * np.eye(s).ravel())
    n = len(sizes)
    X0 = with_pattern(sizes, sizes, np.arange(n + 1), np.arange(n), np.concatenate(vals))
    X, res = oracle_sign_chain(X0, 12, 0.0)
    D = np.diag(dense(X))
    expect = np.concatenate([np.full(s, (-1.0) ** b) for b, s in enumerate(sizes)])
    assert np.allclose(D, expect, atol=1e-15, rtol=0)
    assert res < 1e-14


def test_filter_drops_vanishing_blocks():
    # two diagonal blocks, one far below eps: it is dropped from T and X
    sizes = [5, 5]
    vals = np.concatenate([0.5 * np.eye(5).ravel(), 1e-12 * np.eye(5).ravel()])
    X0 = with_pattern(sizes, sizes, [0, 1, 2], [0, 1], vals)
    X, _ = oracle_sign_chain(X0, 1, 1e-7)
    # product norms of the small block are ~1e-24 * 5: dropped on the fly;
    # T keeps 3I there (from the C_in pattern), X's small block is dropped
    assert list(X.col_idx) == [0]
