"""Tile shapes and forms of the generic path and its autotuner, through the C-ABI.

The generic path (block sizes neither all <= 16 nor all 23x23) has eight
variants: 32x32 sub-tiles or, for C blocks with both edges <= 16, one 16x16
sub-tile, on the FP64 vector units or, for 32x32 sub-tiles of C blocks with
both edges >= 16 when every inner edge is >= 16, on the FP64 matrix cores;
each with or without C_in loaded ahead of a sub-tile's last chunk.  Every variant must give the
oracle's pattern and product stack exactly and its values within the FP64
tolerance; integer inputs exactly.  The vector form sums every output over the
same inner indices in the same order with either tile size and either C_in
load, so variants 0, 1, 4 and 5 must give identical bits, and so must 2 and 6,
3 and 7.  The tuner must leave C as a plain multiply with
its chosen variant does and enter that variant into the table.
"""
import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import bsmm
from paper_1708_03604_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-12

SETS = {
    # the H2O-64-shaped mix: 9x9 C blocks pad to 16x16 instead of 32x32
    "mixed_9_22_32": ([9, 22, 32] * 6, [9, 22, 32] * 6, [9, 22, 32] * 6),
    # narrow and wide edges, partial sub-tiles of both sizes, K chunks past 32
    "narrow_wide": ([9, 40, 17, 3] * 4, [40, 9, 20, 70] * 4, [33, 9, 48, 2] * 4),
    # every inner edge >= 16: all four variants are allowed
    "wide": ([16, 40, 33, 64, 17] * 2, [24, 48, 16, 31, 65] * 2, [20, 65, 32, 16, 9] * 3),
    "edge40": ([40] * 8, [40] * 8, [40] * 8),
}


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


@pytest.fixture()
def table():
    """Restore the process-wide table of the generic path after the test."""
    saved = bsmm.bsmm_mid_entries()
    yield
    for k in bsmm.bsmm_mid_entries():
        bsmm.bsmm_mid_set(k, None)
    for k, v in saved.items():
        bsmm.bsmm_mid_set(k, v)


def rel_err(got, ref):
    n = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / n if n > 0 else np.linalg.norm(got)


def operands(name, seed, kind="uniform"):
    rs, ks, cs = SETS[name]
    A = W.random_matrix(seed, rs, ks, 0.4, kind=kind)
    B = W.random_matrix(seed + 1, ks, cs, 0.4, kind=kind)
    Co = W.random_matrix(seed + 2, rs, cs, 0.3, kind=kind)
    return A, B, Co


def wide_inner(ks):
    return min(ks) >= 16


def run(A, B, Co, variant, alpha, beta, eps):
    dA, dB, dCin = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B), bsmm.Matrix.from_csr(Co)
    masks = bsmm.bsmm_mid_key(dA.handle, dB.handle)
    bsmm.bsmm_mid_set(masks, variant)
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(alpha, dA, dB, beta, dCin, dC, eps)
    out = dC.to_host() + (dC.stack(), bsmm.bsmm_stats(dC.handle))
    for m in (dA, dB, dCin, dC):
        m.close()
    return out


def check(ref, out, variant, exact):
    rp, ci, v, st, stats = out
    assert stats["path"] == bsmm.BSMM_PATH_GENERIC
    assert stats["variants"][0] == variant
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    assert np.array_equal(st, ref.stack.reshape(-1, 3)), "product stack"
    if exact:
        assert np.array_equal(v, ref.values)
    else:
        assert rel_err(v, ref.values) <= REL_TOL


@pytest.mark.parametrize("name", sorted(SETS))
def test_every_variant_matches_the_oracle(table, name):
    A, B, Co = operands(name, 931)
    eps = 0.05
    ref = oracle.multiply(0.75, A, B, -0.5, Co, eps)
    allowed = range(bsmm.BSMM_MID_VARIANTS) if wide_inner(SETS[name][1]) else (0, 1, 4, 5)
    vals = {}
    for v in allowed:
        out = run(A, B, Co, v, 0.75, -0.5, eps)
        check(ref, out, v, exact=False)
        vals[v] = out[2]
    # the vector form gives the same bits with 16x16 and 32x32 sub-tiles and
    # with or without the C_in prefetch; so does each matrix-core variant
    for v in (1, 4, 5):
        assert np.array_equal(vals[0], vals[v])
    for v in (2, 3):
        if v in vals:
            assert np.array_equal(vals[v], vals[v + 4])


@pytest.mark.parametrize("name", sorted(SETS))
def test_every_variant_exact_on_integers(table, name):
    A, B, Co = operands(name, 951, kind="int")
    ref = oracle.multiply(1.0, A, B, 2.0, Co, 0.0)
    allowed = range(bsmm.BSMM_MID_VARIANTS) if wide_inner(SETS[name][1]) else (0, 1, 4, 5)
    for v in allowed:
        check(ref, run(A, B, Co, v, 1.0, 2.0, 0.0), v, exact=True)


def test_matrix_core_bit_dropped_for_narrow_inner_edges(table):
    A, B, Co = operands("mixed_9_22_32", 961)
    ref = oracle.multiply(1.0, A, B, 1.0, Co, 0.0)
    for v, used in ((2, 0), (3, 1), (6, 4), (7, 5)):
        check(ref, run(A, B, Co, v, 1.0, 1.0, 0.0), used, exact=False)


def test_tuner_result_and_table(table):
    A, B, Co = operands("wide", 971)
    ref = oracle.multiply(0.5, A, B, 1.5, Co, 0.0)
    dA, dB, dCin = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B), bsmm.Matrix.from_csr(Co)
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    v, ms = bsmm.bsmm_tune_mid(0.5, dA.handle, dB.handle, 1.5, dCin.handle, dC.handle, 0.0, 2)
    assert 0 <= v < bsmm.BSMM_MID_VARIANTS and (ms > 0).all()
    assert bsmm.bsmm_mid_get(bsmm.bsmm_mid_key(dA.handle, dB.handle)) == v
    rp, ci, vals = dC.to_host()
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    assert rel_err(vals, ref.values) <= REL_TOL
    assert bsmm.bsmm_stats(dC.handle)["variants"][0] == v
    # a later multiply takes the tuned variant and gives the tuner's bits
    dD = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(0.5, dA, dB, 1.5, dCin, dD, 0.0)
    assert bsmm.bsmm_stats(dD.handle)["variants"][0] == v
    assert np.array_equal(dD.to_host()[2], vals)
    # narrow inner edges: the matrix-core variants are not timed
    N, K, Q = operands("mixed_9_22_32", 972)
    dN, dK, dQ = bsmm.Matrix.from_csr(N), bsmm.Matrix.from_csr(K), bsmm.Matrix.from_csr(Q)
    dE = bsmm.Matrix.empty(N.row_sizes, K.col_sizes)
    v2, ms2 = bsmm.bsmm_tune_mid(1.0, dN.handle, dK.handle, 1.0, dQ.handle, dE.handle, 0.0, 1)
    assert v2 in (0, 1, 4, 5) and all(ms2[u] > 0 for u in (0, 1, 4, 5)) and not ms2[[2, 3, 6, 7]].any()
    for m in (dA, dB, dCin, dC, dD, dN, dK, dQ, dE):
        m.close()


def test_tuner_other_paths_and_errors(table):
    S = W.random_matrix(981, [5, 13] * 3, [5, 13] * 3, 0.5)
    dS, dT = bsmm.Matrix.from_csr(S), bsmm.Matrix.from_csr(S)
    before = bsmm.bsmm_mid_entries()
    v, ms = bsmm.bsmm_tune_mid(1.0, dS.handle, dS.handle, 0.0, None, dT.handle, 0.0, 2)
    assert v == -1 and not ms.any() and bsmm.bsmm_mid_entries() == before
    assert bsmm.bsmm_stats(dT.handle)["path"] == bsmm.BSMM_PATH_SMALL
    for reps in (0, 1001):
        with pytest.raises(bsmm.BsmmError) as e:
            bsmm.bsmm_tune_mid(1.0, dS.handle, dS.handle, 0.0, None, dT.handle, 0.0, reps)
        assert e.value.status == "BSMM_E_ARG"
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.bsmm_tune_mid(1.0, dS.handle, dS.handle, 1.0, dT.handle, dT.handle, 0.0, 1)
    assert e.value.status == "BSMM_E_ARG"
    dS.close()
    dT.close()


def test_tuned_variant_in_reserved_and_captured_multiplies(table):
    """A reserved (device-sized) multiply takes the table's variant like an
    eager one, and every replay of its captured graph gives the eager bits."""
    import torch
    A, B, Co = operands("mixed_9_22_32", 991)
    ref = oracle.multiply(1.25, A, B, 0.5, Co, 0.0)
    stream = torch.cuda.Stream()
    dA, dB, dCin = (bsmm.Matrix.from_csr(x, stream) for x in (A, B, Co))
    bsmm.bsmm_mid_set(bsmm.bsmm_mid_key(dA.handle, dB.handle), 1)
    dE = bsmm.Matrix.empty(A.row_sizes, B.col_sizes, stream)
    bsmm.multiply(1.25, dA, dB, 0.5, dCin, dE, 0.0, stream=stream)
    eager = dE.to_host(stream)
    assert bsmm.bsmm_stats(dE.handle)["variants"][0] == 1
    assert rel_err(eager[2], ref.values) <= REL_TOL
    nr, nc = len(A.row_sizes), len(B.col_sizes)
    dR = bsmm.Matrix.empty(A.row_sizes, B.col_sizes, stream)
    bsmm.bsmm_reserve(dR.handle, nr * nc, int(np.sum(A.row_sizes)) * int(np.sum(B.col_sizes)),
                      nr * len(A.col_sizes) * nc, stream)
    bsmm.multiply(1.25, dA, dB, 0.5, dCin, dR, 0.0, stream=stream)
    got = dR.to_host(stream)
    assert bsmm.bsmm_stats(dR.handle)["variants"][0] == 1
    for r, g in zip(eager, got):
        assert np.array_equal(r, g)
    stream.synchronize()
    bsmm.bsmm_capture_begin(stream)
    try:
        bsmm.multiply(1.25, dA, dB, 0.5, dCin, dR, 0.0, stream=stream)
    finally:
        graph = bsmm.bsmm_capture_end(stream)
    try:
        for _ in range(3):
            bsmm.bsmm_graph_launch(graph, stream)
            got = dR.to_host(stream)
            for r, g in zip(eager, got):
                assert np.array_equal(r, g)
            # eager work between the replays
            bsmm.multiply(1.0, dA, dB, 0.0, None, dE, 0.0, stream=stream)
            stream.synchronize()
    finally:
        bsmm.bsmm_graph_destroy(graph)
    for m in (dA, dB, dCin, dE, dR):
        m.close()
