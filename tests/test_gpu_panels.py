"""Product stacks built and consumed in panels of C block rows (the 23x23
paths, bsmm_set_stack_limit) and block rows beyond the ordinary symbolic
forms (the huge forms: up to 2048 A blocks and 2048 result blocks per row),
through the C-ABI.

A panelled multiply runs every C block's products in the same order as the
whole-stack multiply, so its values must equal the whole-stack values bit for
bit, in every precision; its pattern must equal the oracle's.  Rows served by
the huge forms must match the oracle as any other row: pattern and product
stack exact, values within the FP64 tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import bsmm
from paper_1708_03604_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-12
PRECS = {"fp64": bsmm.BSMM_FP64, "split": bsmm.BSMM_SPLIT_BF16X3, "slice": bsmm.BSMM_SLICE_INT8X7}


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def rel_err(got, ref):
    d = np.linalg.norm(got - ref)
    n = np.linalg.norm(ref)
    return d / n if n > 0 else d


def row_products(ref):
    """Kept block products per C block row of an oracle result."""
    rows = np.repeat(np.arange(len(ref.row_ptr) - 1), np.diff(ref.row_ptr))
    c = np.asarray(ref.stack).reshape(-1, 3)[:, 0]
    return np.bincount(rows[c], minlength=len(ref.row_ptr) - 1)


def expected_panels(ref, limit):
    """Panels that hold a block row when panel starts lie max(limit - R,
    limit // 2) products apart (R: the most products of one row): one per
    distinct start window of the rows' first products."""
    per = row_products(ref)
    w = max(limit - int(per.max()), limit // 2)
    starts = np.concatenate(([0], np.cumsum(per)[:-1]))
    return len(np.unique(starts // w))


def run(A, B, Co, alpha, beta, eps, prec=bsmm.BSMM_FP64, limit=None, in_place=False, reserve=None):
    dA = bsmm.Matrix.from_csr(A)
    dB = bsmm.Matrix.from_csr(B)
    if in_place:
        dC = bsmm.Matrix.from_csr(Co)
        dCin = dC
    else:
        dCin = bsmm.Matrix.from_csr(Co) if Co is not None else None
        dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    if limit is not None:
        bsmm.bsmm_set_stack_limit(dC.handle, limit)
    if reserve is not None:
        bsmm.bsmm_reserve(dC.handle, *reserve)
    bsmm.multiply(alpha, dA, dB, beta, dCin, dC, eps, prec=prec)
    out = dC.to_host() + (bsmm.bsmm_stats(dC.handle),)
    for m in {id(x): x for x in (dA, dB, dCin, dC) if x is not None}.values():
        m.close()
    return out


def operands(seed, nb=40, density=0.3):
    sizes = [23] * nb
    A = W.random_matrix(seed, sizes, sizes, density)
    B = W.random_matrix(seed + 1, sizes, sizes, density)
    Co = W.random_matrix(seed + 2, sizes, sizes, 0.2)
    return A, B, Co


@pytest.mark.parametrize("prec", sorted(PRECS))
@pytest.mark.parametrize("alpha,beta,filt", [(1.0, 0.0, 0.0), (-0.5, 1.5, 0.0), (1.0, 1.0, 1.0)])
def test_panels_bit_identical_to_whole_stack(prec, alpha, beta, filt):
    A, B, Co = operands(501)
    Co = Co if beta else None
    ref = oracle.multiply(alpha, A, B, beta, Co, filt)
    most = int(row_products(ref).max())
    whole = run(A, B, Co, alpha, beta, filt, prec=PRECS[prec])
    for limit in (2 * most, 2 * most + 37, len(ref.stack) - 1):
        got = run(A, B, Co, alpha, beta, filt, prec=PRECS[prec], limit=limit)
        assert got[3]["panels"] == expected_panels(ref, limit) > 1
        assert np.array_equal(got[0], ref.row_ptr) and np.array_equal(got[1], ref.col_idx)
        assert np.array_equal(got[2], whole[2]), f"limit {limit}"
        assert got[3]["products"] == len(ref.stack)
    assert whole[3]["panels"] == 1
    if prec == "fp64":
        assert rel_err(whole[2], ref.values) <= REL_TOL


def test_panels_in_place():
    A, B, Co = operands(511)
    ref = oracle.multiply(0.75, A, B, -1.25, Co, 0.0)
    most = int(row_products(ref).max())
    whole = run(A, B, Co, 0.75, -1.25, 0.0, in_place=True)
    got = run(A, B, Co, 0.75, -1.25, 0.0, in_place=True, limit=2 * most)
    assert got[3]["panels"] > 1
    assert np.array_equal(got[1], ref.col_idx)
    assert np.array_equal(got[2], whole[2])
    assert rel_err(got[2], ref.values) <= REL_TOL


def test_panel_limit_below_a_row_is_rejected():
    # a block row with more products than half the limit: BSMM_E_CAPACITY and
    # C unchanged
    A, B, _ = operands(521)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    most = int(row_products(ref).max())
    dA, dB = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B)
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(1.0, dA, dA, 0.0, None, dC, 0.0)
    before = dC.to_host()
    bsmm.bsmm_set_stack_limit(dC.handle, most - 1)  # the longest row alone exceeds it
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.multiply(1.0, dA, dB, 0.0, None, dC, 0.0)
    assert e.value.status == "BSMM_E_CAPACITY"
    for x, y in zip(before, dC.to_host()):
        assert np.array_equal(x, y)
    for bad in (0, 1, 2 ** 31):
        with pytest.raises(bsmm.BsmmError) as e:
            bsmm.bsmm_set_stack_limit(dC.handle, bad)
        assert e.value.status == "BSMM_E_ARG"
    for m in (dA, dB, dC):
        m.close()


def test_panelled_stack_is_not_exported():
    A, B, _ = operands(531, nb=20)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    dA, dB = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B)
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.bsmm_set_stack_limit(dC.handle, 2 * int(row_products(ref).max()))
    bsmm.multiply(1.0, dA, dB, 0.0, None, dC, 0.0)
    with pytest.raises(bsmm.BsmmError) as e:
        dC.stack()
    assert e.value.status == "BSMM_E_UNSUPPORTED"
    bsmm.bsmm_filter(dC.handle, 0.0)  # new block indices: no stack at all
    assert len(dC.stack()) == 0
    for m in (dA, dB, dC):
        m.close()


@pytest.mark.parametrize("prec", ["fp64", "split"])
def test_reserved_panels_equal_whole_stack(prec):
    # reserved output with a product capacity three times the products: many
    # panels, the later ones empty; then the limit may not change
    A, B, Co = operands(541)
    ref = oracle.multiply(1.0, A, B, 1.0, Co, 0.0)
    most = int(row_products(ref).max())
    nb = len(A.row_sizes)
    caps = (nb * nb, (nb * 23) ** 2, 3 * len(ref.stack))
    whole = run(A, B, Co, 1.0, 1.0, 0.0, prec=PRECS[prec])
    got = run(A, B, Co, 1.0, 1.0, 0.0, prec=PRECS[prec], limit=2 * most, reserve=caps)
    # the stats count the panels that held a row, not the ones launched
    assert got[3]["panels"] == expected_panels(ref, 2 * most) > 1
    assert np.array_equal(got[1], ref.col_idx)
    assert np.array_equal(got[2], whole[2])
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.bsmm_reserve(dC.handle, *caps)
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.bsmm_set_stack_limit(dC.handle, 1000)
    assert e.value.status == "BSMM_E_ARG"
    dC.close()


def test_chain_with_panels_replays_bit_identical():
    # the sign chain with every multiply in panels, eager and as graph
    # replays, against the chain with whole stacks
    import torch
    from paper_1708_03604_amd.chain import SignChain
    X0, _ = W.symmetric_scaled(seed=5200, nmol=16)
    ref_ch = SignChain(X0, steps=6, eps=1e-7)
    ref_ch.enqueue()
    ref_ch.stream.synchronize()
    ref = ref_ch.final.to_host()
    ref_res = float(ref_ch.residual.cpu()[0])
    ref_ch.close()
    ch = SignChain(X0, steps=6, eps=1e-7, stack_limit=2 * 16 * 16 + 8)
    ch.enqueue()
    ch.stream.synchronize()
    assert bsmm.bsmm_stats(ch.T.handle)["panels"] > 1
    for x, y in zip(ref, ch.final.to_host()):
        assert np.array_equal(x, y)
    ch.capture()
    for rep in range(3):
        ch.residual.zero_()
        torch.cuda.synchronize()
        ch.replay()
        ch.stream.synchronize()
        for x, y in zip(ref, ch.final.to_host()):
            assert np.array_equal(x, y), f"replay {rep}"
        assert float(ch.residual.cpu()[0]) == ref_res
    ch.close()


# ------------------------------------------------------------ huge rows

def _long_rows(seed, bs, na, nc, kdens, ragged=True):
    """Two block rows of A with every one of na blocks, a third ragged one,
    and B (na x nc) sparse enough that the result rows reach about nc
    blocks: rows beyond the ordinary forms (1024) but within 2048."""
    rng = np.random.default_rng(seed)
    ma = np.zeros((3, na), dtype=bool)
    ma[:2, :] = True
    ma[2, :] = rng.random(na) < (0.6 if ragged else 1.0)
    mb = rng.random((na, nc)) < kdens
    mb[np.arange(na), np.arange(na) % nc] = True
    A = W.with_pattern(np.full(3, bs, np.int32), np.full(na, bs, np.int32), *W.pattern_from_mask(ma))
    B = W.with_pattern(np.full(na, bs, np.int32), np.full(nc, bs, np.int32), *W.pattern_from_mask(mb))
    A.values = W.values_uniform(seed + 1, A.block_elems())
    B.values = W.values_uniform(seed + 2, B.block_elems())
    return A, B


@pytest.mark.parametrize("bs,na,nc", [(23, 1100, 1050), (5, 1500, 1300), (1, 2048, 2048)])
def test_huge_rows_match_oracle(bs, na, nc):
    A, B = _long_rows(551 + bs, bs, na, nc, 0.01)
    Co = W.random_matrix(560 + bs, A.row_sizes, B.col_sizes, 0.3)
    for beta, eps in ((0.0, 0.0), (0.5, 1e-3)):
        ref = oracle.multiply(1.0, A, B, beta, Co if beta else None, eps)
        assert np.diff(ref.row_ptr).max() > 1024
        dA, dB = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B)
        dCin = bsmm.Matrix.from_csr(Co) if beta else None
        dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
        bsmm.multiply(1.0, dA, dB, beta, dCin, dC, eps)
        rp, ci, v = dC.to_host()
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
        assert np.array_equal(dC.stack(), np.asarray(ref.stack).reshape(-1, 3))
        assert rel_err(v, ref.values) <= REL_TOL
        for m in (dA, dB, dCin, dC):
            if m is not None:
                m.close()


def test_huge_rows_with_panels():
    # rows from the huge fill form inside a panelled 23x23 multiply
    A, B = _long_rows(571, 23, 1100, 1050, 0.004)
    ref = oracle.multiply(1.0, A, B, 0.0, None, 0.0)
    most = int(row_products(ref).max())
    whole = run(A, B, None, 1.0, 0.0, 0.0)
    got = run(A, B, None, 1.0, 0.0, 0.0, limit=2 * most)
    assert got[3]["panels"] > 1
    assert np.array_equal(got[1], ref.col_idx)
    assert np.array_equal(got[2], whole[2])
    assert rel_err(got[2], ref.values) <= REL_TOL
