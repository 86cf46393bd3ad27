"""GPU path against the CPU oracle, through the C-ABI.

Pattern and product stack: bit-exact.  FP64 values: relative Frobenius error
<= 1e-12 (the stated tolerance); small-integer inputs: bit-exact (every sum is
exact in FP64).  Norms and filter: bit-exact (both sides use the same fixed
summation order and correctly rounded square root).
"""
import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import bsmm
from paper_1708_03604_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def gpu_multiply(A, B, Cold, alpha, beta, eps, in_place=False):
    dA = bsmm.Matrix.from_csr(A)
    dB = dA if B is A else bsmm.Matrix.from_csr(B)
    if in_place:
        dC = bsmm.Matrix.from_csr(Cold)
        dCin = dC
    else:
        dCin = bsmm.Matrix.from_csr(Cold) if Cold is not None else None
        dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(alpha, dA, dB, beta, dCin, dC, eps)
    rp, ci, v = dC.to_host()
    st = dC.stack()
    stats = bsmm.bsmm_stats(dC.handle)
    for m in {id(x): x for x in (dA, dB, dCin, dC) if x is not None}.values():
        m.close()
    return rp, ci, v, st, stats


def rel_err(got, ref):
    d = np.linalg.norm(got - ref)
    n = np.linalg.norm(ref)
    return d / n if n > 0 else d


def check(ref, got, exact=False):
    rp, ci, v, st, stats = got
    assert np.array_equal(rp, ref.row_ptr), "row_ptr"
    assert np.array_equal(ci, ref.col_idx), "col_idx"
    assert np.array_equal(st, ref.stack.reshape(-1, 3)), "product stack"
    assert len(v) == len(ref.values)
    if exact:
        assert np.array_equal(v, ref.values)
    else:
        assert rel_err(v, ref.values) <= REL_TOL
    assert stats["products"] == len(ref.stack)
    assert stats["nnzb"] == len(ref.col_idx)


SIZE_SETS = {
    "b23": ([23] * 24, [23] * 24, [23] * 24),
    "b5_13": ([5, 13, 13, 5, 5, 13] * 4, [13, 5, 5, 13] * 5, [5, 13, 5] * 7),
    "mixed_small": ([1, 2, 3, 7] * 5, [4, 1, 9] * 6, [2, 2, 1, 11] * 4),
    "b6": ([6] * 30, [6] * 30, [6] * 30),
    "b32": ([32] * 10, [32] * 10, [32] * 10),
    # every class boundary of the small-block path: edges 1, 8, 9, 15, 16
    "edge16": ([16, 9, 8, 1, 15] * 5, [16, 8, 3, 16, 9] * 6, [9, 16, 8, 2] * 6),
    # every edge >= 16, not uniform: the generic path's matrix-core form, with
    # partial 32x32 sub-tiles, K chunks past 32 and inner sizes not a multiple of 8
    "wide": ([16, 40, 33, 64, 17] * 2, [24, 48, 16, 31, 65] * 2, [20, 65, 32, 16] * 3),
}


def _eps_median(A, B):
    nA, nB = oracle.norms(A), oracle.norms(B)
    prods = []
    for i in range(A.nbrows):
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            k = A.col_idx[p]
            prods.extend(nA[p] * nB[B.row_ptr[k]:B.row_ptr[k + 1]])
    return float(np.median(prods)) if prods else 1.0


@pytest.mark.parametrize("name", sorted(SIZE_SETS))
@pytest.mark.parametrize("alpha,beta,filt", [(1.0, 0.0, False), (-0.75, 1.25, False), (1.0, 1.0, True),
                                             (2.0, 0.0, True)])
def test_random_parity(name, alpha, beta, filt):
    rs, ks, cs = SIZE_SETS[name]
    A = W.random_matrix(11, rs, ks, 0.3)
    B = W.random_matrix(12, ks, cs, 0.3)
    Co = W.random_matrix(13, rs, cs, 0.2)
    eps = _eps_median(A, B) if filt else 0.0
    ref = oracle.multiply(alpha, A, B, beta, Co if beta else None, eps)
    check(ref, gpu_multiply(A, B, Co if beta else None, alpha, beta, eps))


@pytest.mark.parametrize("name", sorted(SIZE_SETS))
def test_integer_bit_exact(name):
    rs, ks, cs = SIZE_SETS[name]
    A = W.random_matrix(21, rs, ks, 0.4, kind="int")
    B = W.random_matrix(22, ks, cs, 0.4, kind="int")
    Co = W.random_matrix(23, rs, cs, 0.3, kind="int")
    ref = oracle.multiply(3.0, A, B, -2.0, Co, 0.0)
    check(ref, gpu_multiply(A, B, Co, 3.0, -2.0, 0.0), exact=True)


def test_square_same_operand_and_in_place():
    sizes = [23] * 20
    X = W.random_matrix(31, sizes, sizes, 0.25)
    Co = W.random_matrix(32, sizes, sizes, 0.25)
    ref = oracle.multiply(-1.0, X, X, 1.0, Co, 5.0)
    check(ref, gpu_multiply(X, X, Co, -1.0, 1.0, 5.0))
    check(ref, gpu_multiply(X, X, Co, -1.0, 1.0, 5.0, in_place=True))


@pytest.mark.parametrize("sizes", [[1, 2, 5, 13, 23, 30, 64, 65, 100],   # one block per wave
                                   [1, 2, 3, 5, 6, 8, 13, 15, 16] * 3])  # blocks of <= 256 values: four per wave
def test_norms_bit_exact(sizes):
    import torch
    M = W.random_matrix(41, sizes, sizes[::-1], 0.7)
    M.values[:64] *= 1e-160       # tiny and huge magnitudes
    M.values[-64:] *= 1e150
    dM = bsmm.Matrix.from_csr(M)
    out = torch.empty(M.nnzb, dtype=torch.float64, device="cuda")
    bsmm.bsmm_norms(dM.handle, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle.norms(M)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    dM.close()


def test_norm_golden_cases_on_gpu():
    import json
    import os
    import torch
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "norm_cases.json")))
    for case in g["cases"]:
        m, n = case["shape"]
        if "fill_hex" in case:
            vals = np.full(m * n, float.fromhex(case["fill_hex"]))
        else:
            vals = np.array([float.fromhex(h) for h in case["values_hex"]])
        M = W.BlockCSR([m], [n], [0, 1], [0], vals)
        dM = bsmm.Matrix.from_csr(M)
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        bsmm.bsmm_norms(dM.handle, out)
        torch.cuda.synchronize()
        assert out.item() == float.fromhex(case["norm_hex"]), case["name"]
        dM.close()


@pytest.mark.parametrize("quantile", [0.0, 0.3, 0.7, 1.0])
def test_filter_bit_exact(quantile):
    sizes = [5, 13, 23, 5, 13] * 6
    M = W.random_matrix(51, sizes, sizes, 0.4)
    n = np.sort(oracle.norms(M))
    eps = 0.0 if quantile == 0.0 else float(n[min(int(quantile * len(n)), len(n) - 1)])
    ref = oracle.filter(M, eps)
    dM = bsmm.Matrix.from_csr(M)
    bsmm.bsmm_filter(dM.handle, eps)
    rp, ci, v = dM.to_host()
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    assert np.array_equal(v, ref.values)
    dM.close()


def test_deterministic_bits():
    sizes = [23] * 32
    A = W.random_matrix(61, sizes, sizes, 0.3)
    B = W.random_matrix(62, sizes, sizes, 0.3)
    r1 = gpu_multiply(A, B, None, 1.0, 0.0, 0.0)
    r2 = gpu_multiply(A, B, None, 1.0, 0.0, 0.0)
    assert r1[2].tobytes() == r2[2].tobytes()


def test_beta_zero_ignores_nan_cold():
    sizes = [23] * 8
    A = W.random_matrix(71, sizes, sizes, 0.5)
    B = W.random_matrix(72, sizes, sizes, 0.5)
    Co = W.random_matrix(73, sizes, sizes, 0.5)
    Co.values[:] = np.nan
    dA, dB, dCo = (bsmm.Matrix.from_csr(x) for x in (A, B, Co))
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(1.0, dA, dB, 0.0, dCo, dC, 0.0)
    _, _, v = dC.to_host()
    assert np.all(np.isfinite(v))
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    assert rel_err(v, ref.values) <= REL_TOL


def test_empty_and_degenerate():
    # no A blocks at all
    A = W.with_pattern([23, 23], [23], [0, 0, 0], [])
    B = W.random_matrix(81, [23], [23, 23], 1.0)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    check(ref, gpu_multiply(A, B, None, 1.0, 0.0, 0.0))
    # empty product but beta != 0: result is beta * C_in
    Co = W.random_matrix(82, [23, 23], [23, 23], 0.5)
    ref = oracle.multiply(1.0, A, B, 0.5, Co, 0.0)
    check(ref, gpu_multiply(A, B, Co, 1.0, 0.5, 0.0))
    # filter drops everything
    A = W.random_matrix(83, [23] * 3, [23] * 3, 1.0)
    ref = oracle.multiply(1.0, A, A, 0.0, None, 1e30)
    check(ref, gpu_multiply(A, A, None, 1.0, 0.0, 1e30))
    # 1x1 blocks
    A = W.random_matrix(84, [1] * 50, [1] * 40, 0.2)
    B = W.random_matrix(85, [1] * 40, [1] * 30, 0.2)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    check(ref, gpu_multiply(A, B, None, 1.0, 0.0, 0.0))


@pytest.mark.parametrize("edges", [[5, 13], [9, 22, 32], [6]])
def test_degenerate_on_every_path(edges):
    # the small-block and tiled paths on the same degenerate inputs
    rs = np.resize(np.array(edges, dtype=np.int32), 4)
    A0 = W.with_pattern(rs, rs[:3], [0, 0, 0, 0, 0], [])
    B = W.random_matrix(86, rs[:3], rs, 1.0)
    Co = W.random_matrix(87, rs, rs, 0.5)
    # no A blocks, beta = 0: empty result
    check(oracle.multiply(1.0, A0, B, 0.0, None, 0.0), gpu_multiply(A0, B, None, 1.0, 0.0, 0.0))
    # no products but beta != 0: beta * C_in
    check(oracle.multiply(1.0, A0, B, -2.0, Co, 0.0), gpu_multiply(A0, B, Co, 1.0, -2.0, 0.0))
    # the filter drops every product; C_in's pattern stays
    A = W.random_matrix(88, rs, rs[:3], 1.0)
    check(oracle.multiply(1.0, A, B, 0.5, Co, 1e30), gpu_multiply(A, B, Co, 1.0, 0.5, 1e30))
    # a single block
    A1 = W.random_matrix(89, rs[:1], rs[:1], 1.0)
    check(oracle.multiply(1.0, A1, A1, 0.0, None, 0.0), gpu_multiply(A1, A1, None, 1.0, 0.0, 0.0))


def test_error_paths():
    sizes = [23] * 4
    A = bsmm.Matrix.from_csr(W.random_matrix(91, sizes, sizes, 0.5))
    B = bsmm.Matrix.from_csr(W.random_matrix(92, [5] * 4, sizes, 0.5))
    C = bsmm.Matrix.empty(sizes, sizes)
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.multiply(1.0, A, B, 0.0, None, C, 0.0)
    assert e.value.status == "BSMM_E_SHAPE"
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.multiply(1.0, A, A, 0.0, None, A, 0.0)
    assert e.value.status == "BSMM_E_ALIAS"
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.multiply(1.0, A, A, 0.0, None, C, float("nan"))
    assert e.value.status == "BSMM_E_ARG"
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.multiply(1.0, A, A, 0.0, None, C, 0.0, prec=99)
    assert e.value.status == "BSMM_E_ARG"
    # C unchanged by failed calls
    assert C.info()[2] == 0
    for m in (A, B, C):
        m.close()


@pytest.mark.parametrize("case", ["a_row_too_long", "c_row_too_wide"])
def test_row_limits_reported(case):
    # more than 2048 stored A blocks in a row, or more than 2048 result blocks
    # in a row: BSMM_E_UNSUPPORTED, and the other rows do not matter
    if case == "a_row_too_long":
        ma = np.zeros((3, 2100), dtype=bool)
        ma[1, :] = True
        mb = np.zeros((2100, 2), dtype=bool)
        mb[:, 0] = True
    else:
        ma = np.ones((3, 2), dtype=bool)
        mb = np.ones((2, 2100), dtype=bool)
    A = W.with_pattern(np.ones(ma.shape[0], np.int32), np.ones(ma.shape[1], np.int32), *W.pattern_from_mask(ma))
    B = W.with_pattern(np.ones(mb.shape[0], np.int32), np.ones(mb.shape[1], np.int32), *W.pattern_from_mask(mb))
    dA, dB = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B)
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.multiply(1.0, dA, dB, 0.0, None, dC, 0.0)
    assert e.value.status == "BSMM_E_UNSUPPORTED"
    assert dC.info()[2] == 0
    for m in (dA, dB, dC):
        m.close()


# ------------------------------------------------------------- full sizes

def take_rows(M, rows):
    off = M.block_offsets()
    rp = [0]
    ci, vals, bmap = [], [], []
    for i in rows:
        b0, b1 = M.row_ptr[i], M.row_ptr[i + 1]
        ci.append(M.col_idx[b0:b1])
        vals.append(M.values[off[b0]:off[b1]])
        bmap.extend(range(b0, b1))
        rp.append(rp[-1] + b1 - b0)
    return (W.BlockCSR(M.row_sizes[rows], M.col_sizes, rp, np.concatenate(ci), np.concatenate(vals)),
            np.array(bmap, dtype=np.int64))


def sampled_rows_check(w, rows, got):
    """Compare GPU rows `rows` of a full-size multiply with the oracle run on
    the same rows of A (and C_in): pattern, stack and values."""
    rp, ci, v, st, _ = got
    Asub, amap = take_rows(w.A, rows)
    Csub = take_rows(w.C_old, rows)[0] if w.C_old is not None else None
    ref = oracle.multiply(w.alpha, Asub, w.B, w.beta, Csub, w.eps)
    # value offsets of the GPU result
    nb = np.diff(rp)
    rowsz = w.A.row_sizes
    colsz = w.B.col_sizes
    brow = np.repeat(np.arange(len(rowsz)), nb)
    boff = np.zeros(len(ci) + 1, dtype=np.int64)
    np.cumsum(rowsz[brow].astype(np.int64) * colsz[ci], out=boff[1:])
    ref_off = ref.row_ptr
    gvals, rvals = [], []
    rstarts = np.zeros(len(ref.col_idx) + 1, dtype=np.int64)
    np.cumsum(ref.row_sizes[np.repeat(np.arange(len(rows)), np.diff(ref.row_ptr))].astype(np.int64)
              * colsz[ref.col_idx], out=rstarts[1:])
    for x, i in enumerate(rows):
        g0, g1 = rp[i], rp[i + 1]
        r0, r1 = ref_off[x], ref_off[x + 1]
        assert np.array_equal(ci[g0:g1], ref.col_idx[r0:r1]), f"pattern of row {i}"
        gvals.append(v[boff[g0]:boff[g1]])
        rvals.append(ref.values[rstarts[r0]:rstarts[r1]])
        # stack entries of this row, mapped to full indices
        gs = st[(st[:, 0] >= g0) & (st[:, 0] < g1)]
        rs_ = ref.stack[(ref.stack[:, 0] >= r0) & (ref.stack[:, 0] < r1)]
        mapped = np.stack([rs_[:, 0] - r0 + g0, amap[rs_[:, 1]], rs_[:, 2]], axis=1)
        assert np.array_equal(gs, mapped), f"stack of row {i}"
    gv, rv = np.concatenate(gvals), np.concatenate(rvals)
    assert rel_err(gv, rv) <= REL_TOL


def test_grid23_full():
    w = W.grid23()
    ref = oracle.multiply(w.alpha, w.A, w.B, w.beta, None, w.eps)
    check(ref, gpu_multiply(w.A, w.B, None, w.alpha, w.beta, w.eps))


def test_molecules_full_size():
    # the benchmark workload at full size, every row: pattern and stack bit for
    # bit, values within the tolerance (covers the per-XCD split points and
    # the per-wave chunk boundaries of the 23x23 kernel at its real launch)
    w = W.molecules()
    got = gpu_multiply(w.A, w.B, w.C_old, w.alpha, w.beta, w.eps)
    ref = oracle.multiply(w.alpha, w.A, w.B, w.beta, w.C_old, w.eps)
    check(ref, got)


def test_molecules_filter_variant_sampled_rows():
    w = W.molecules(nmol=1024)
    w.eps = _eps_median(w.A, w.B)
    got = gpu_multiply(w.A, w.B, w.C_old, w.alpha, w.beta, w.eps)
    assert 0 < got[4]["products"] < got[4]["candidates"]
    rows = sorted(set(np.random.default_rng(6).choice(w.A.nbrows, 16, replace=False).tolist()) | {0, 1023})
    sampled_rows_check(w, rows, got)


def test_water_atoms_full_size():
    # the mixed 5/13 workload at full size, every row
    w = W.water_atoms()
    got = gpu_multiply(w.A, w.B, None, w.alpha, w.beta, w.eps)
    ref = oracle.multiply(w.alpha, w.A, w.B, w.beta, None, w.eps)
    check(ref, got)


def _rows_dense_mask(seed, nr, nc, dense_rows, p):
    rng = np.random.default_rng(seed)
    mask = rng.random((nr, nc)) < p
    mask[dense_rows, :] = True
    return mask


@pytest.mark.parametrize("case", ["long_a_rows", "wide_c_rows", "medium_rows"])
def test_fill_both_forms(case):
    # The fill runs in three forms by row size: tiny (at most 128 A blocks and
    # 256 result blocks), small (256 and 512) and large (the rest, up to the
    # limits); rows of several forms meet in one multiply.
    if case == "medium_rows":
        nr, nk, nc = 24, 300, 450
        ma = _rows_dense_mask(507, nr, nk, [], 0.05)
        ma[[2, 9], :200] = True
        mb = _rows_dense_mask(508, nk, nc, [], 0.02)
    elif case == "long_a_rows":
        nr, nk, nc = 24, 600, 40
        ma = _rows_dense_mask(501, nr, nk, [0, 7, 23], 0.05)
        mb = _rows_dense_mask(502, nk, nc, [], 0.3)
    else:
        nr, nk, nc = 24, 30, 900
        ma = _rows_dense_mask(503, nr, nk, [], 0.2)
        mb = _rows_dense_mask(504, nk, nc, [3, 11], 0.02)
    rs = np.resize(np.array([1, 2, 3], dtype=np.int32), nr)
    ks = np.resize(np.array([2, 1], dtype=np.int32), nk)
    cs = np.resize(np.array([1, 3, 2], dtype=np.int32), nc)
    rpa, cia = W.pattern_from_mask(ma)
    rpb, cib = W.pattern_from_mask(mb)
    A = W.with_pattern(rs, ks, rpa, cia)
    A.values = W.values_int(505, A.nvals)
    B = W.with_pattern(ks, cs, rpb, cib)
    B.values = W.values_int(506, B.nvals)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    nA = np.diff(A.row_ptr)
    nC = np.diff(ref.row_ptr)
    tiny = (nA <= 128) & (nC <= 256)
    small = (nA <= 256) & (nC <= 512) & ~tiny
    large = ~tiny & ~small
    assert tiny.any() and (small.any() if case == "medium_rows" else large.any())
    check(ref, gpu_multiply(A, B, None, 1.0, 0.0, 0.0), exact=True)


@pytest.mark.parametrize("beta,filt", [(0.0, False), (1.0, True)])
def test_thin_and_wide_rows(beta, filt):
    """Rows taken by the one-thread path (empty rows, one A block with short B
    rows, few C_in blocks) mixed with rows the workgroup forms take, in one
    multiply: pattern and stack exact, values within tolerance; the same in
    reserved (device-sized) mode."""
    rs, ks, cs = [5, 13, 23, 6] * 6, [13, 5, 7] * 8, [6, 23, 5] * 8
    rng = np.random.default_rng(4242)
    nr, nk, nc = len(rs), len(ks), len(cs)
    mask_a = np.zeros((nr, nk), dtype=bool)
    for i in range(nr):
        if i % 3 == 0:
            mask_a[i] = rng.random(nk) < 0.8       # wide row
        elif i % 3 == 1:
            mask_a[i, rng.integers(nk)] = True     # one A block
    mask_b = rng.random((nk, nc)) < 0.15
    mask_c = rng.random((nr, nc)) < 0.1
    A = W.with_pattern(rs, ks, *W.pattern_from_mask(mask_a))
    A.values = W.values_uniform(21, A.block_elems())
    B = W.with_pattern(ks, cs, *W.pattern_from_mask(mask_b))
    B.values = W.values_uniform(22, B.block_elems())
    Co = W.with_pattern(rs, cs, *W.pattern_from_mask(mask_c))
    Co.values = W.values_uniform(23, Co.block_elems())
    eps = _eps_median(A, B) if filt else 0.0
    ref = oracle.multiply(0.7, A, B, beta, Co if beta else None, eps)
    check(ref, gpu_multiply(A, B, Co if beta else None, 0.7, beta, eps))
    dA, dB, dCo = (bsmm.Matrix.from_csr(x) for x in (A, B, Co))
    dC = bsmm.Matrix.empty(rs, cs)
    bsmm.bsmm_reserve(dC.handle, nr * nc, int(np.sum(rs)) * int(np.sum(cs)), nr * nk * nc)
    bsmm.multiply(0.7, dA, dB, beta, dCo if beta else None, dC, eps)
    rp, ci, v = dC.to_host()
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    assert np.array_equal(dC.stack(), ref.stack.reshape(-1, 3))
    assert rel_err(v, ref.values) <= REL_TOL
    for m in (dA, dB, dCo, dC):
        m.close()
