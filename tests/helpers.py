"""Independent numpy utilities for the tests: dense expansion, block transpose
and permutation, brute-force product enumeration.  None of this is used by
the oracle or by the GPU library."""
import numpy as np

from paper_1708_03604_amd.workloads import BlockCSR


def starts(sizes):
    s = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(np.asarray(sizes, dtype=np.int64), out=s[1:])
    return s


def dense(M):
    """Zero-filled dense expansion of a block-CSR matrix."""
    rs, cs = starts(M.row_sizes), starts(M.col_sizes)
    D = np.zeros((rs[-1], cs[-1]))
    off = 0
    for i in range(len(M.row_sizes)):
        for b in range(M.row_ptr[i], M.row_ptr[i + 1]):
            j = M.col_idx[b]
            m, n = M.row_sizes[i], M.col_sizes[j]
            D[rs[i]:rs[i] + m, cs[j]:cs[j] + n] = np.asarray(M.values[off:off + m * n]).reshape(m, n)
            off += m * n
    assert off == len(M.values)
    return D


def mask(M):
    """Dense boolean block mask."""
    out = np.zeros((len(M.row_sizes), len(M.col_sizes)), dtype=bool)
    for i in range(len(M.row_sizes)):
        out[i, M.col_idx[M.row_ptr[i]:M.row_ptr[i + 1]]] = True
    return out


def from_dense(D, row_sizes, col_sizes, blockmask):
    """Block-CSR with the given pattern and values cut out of dense D."""
    rs, cs = starts(row_sizes), starts(col_sizes)
    rp = [0]
    ci, vals = [], []
    for i in range(len(row_sizes)):
        for j in np.nonzero(blockmask[i])[0]:
            ci.append(j)
            vals.append(D[rs[i]:rs[i + 1], cs[j]:cs[j + 1]].ravel())
        rp.append(len(ci))
    v = np.concatenate(vals) if vals else np.zeros(0)
    return BlockCSR(row_sizes, col_sizes, np.array(rp), np.array(ci, dtype=np.int32), v)


def transpose(M):
    D = dense(M)
    return from_dense(D.T, M.col_sizes, M.row_sizes, mask(M).T)


def permute(M, p):
    """P M P^T for a square block structure, block permutation p (new i = old p[i])."""
    p = np.asarray(p)
    D = dense(M)
    rs = starts(M.row_sizes)
    idx = np.concatenate([np.arange(rs[k], rs[k + 1]) for k in p])
    sizes = M.row_sizes[p]
    return from_dense(D[np.ix_(idx, idx)], sizes, sizes, mask(M)[np.ix_(p, p)])


def block(M, b):
    rows = np.repeat(np.arange(len(M.row_sizes)), np.diff(M.row_ptr))
    m, n = M.row_sizes[rows[b]], M.col_sizes[M.col_idx[b]]
    off = 0
    for x in range(b):
        off += M.row_sizes[rows[x]] * M.col_sizes[M.col_idx[x]]
    return np.asarray(M.values[off:off + m * n]).reshape(m, n)


def frob_norms_numpy(M):
    """Block norms via numpy (library routine, any summation order)."""
    return np.array([np.linalg.norm(block(M, b)) for b in range(len(M.col_idx))])


def brute_products(A, B, nA=None, nB=None, eps=0.0):
    """Every (i, k, j, a_blk, b_blk) with both blocks present and the filter
    passed, by explicit loops over the block grid."""
    out = []
    for i in range(len(A.row_sizes)):
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            k = A.col_idx[p]
            for q in range(B.row_ptr[k], B.row_ptr[k + 1]):
                if eps > 0 and not (nA[p] * nB[q] > eps):
                    continue
                out.append((i, k, B.col_idx[q], p, q))
    return out


def oracle_sign_chain(X0, steps, eps):
    """The Newton-Schulz sequence of the chain driver, run with the oracle:
    T = 3I - X X (on-the-fly filter eps, then filter eps), X <- 1/2 X T
    (same), then R = X X - I and ||R||_F.  Returns (X, ||R||_F)."""
    import oracle
    from paper_1708_03604_amd.workloads import identity_like
    I3, I1 = identity_like(X0, 3.0), identity_like(X0, 1.0)
    X = X0
    for _ in range(steps):
        T = oracle.filter(oracle.multiply(-1.0, X, X, 1.0, I3, eps), eps)
        X = oracle.filter(oracle.multiply(0.5, X, T, 0.0, None, eps), eps)
    R = oracle.multiply(1.0, X, X, -1.0, I1, 0.0)
    return X, oracle.frobenius(R)
