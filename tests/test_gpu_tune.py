"""Autotuner of the small-block path, through the C-ABI.

Variants that share the form of each class (on the vector units several
products per step, or one product over four K slices; or the FP64
matrix-core form) compute each C element with the same operations in the
same order, so they must give identical bits; different forms add the same
terms in different orders.  Every variant must match the oracle to the FP64
tolerance, and a multiply whose classes run different variants must give, in
each class, the bits of that class's variant.  The tuner must leave C as a
plain multiply with its chosen variants does and enter its choice (one variant
per class) into the table that later multiplies use.
"""
import numpy as np
import pytest

import oracle
from paper_1708_03604_amd import bsmm, tune
from paper_1708_03604_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-12

# every class of the small-block path: (8|16) x (8|16) with k in 1..16
SIZES = ([5, 13, 13, 5, 16, 1, 9] * 4, [13, 5, 5, 13, 8, 16] * 4, [5, 13, 5, 2, 15] * 5)


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
    """Restore the process-wide tuning table after the test."""
    saved = bsmm.bsmm_tune_entries()
    yield
    for k in bsmm.bsmm_tune_entries():
        bsmm.bsmm_tune_set(k, None)
    for k, v in saved.items():
        bsmm.bsmm_tune_set(k, v)


def operands(seed, beta):
    rs, ks, cs = SIZES
    A = W.random_matrix(seed, rs, ks, 0.35)
    B = W.random_matrix(seed + 1, ks, cs, 0.35)
    Co = W.random_matrix(seed + 2, rs, cs, 0.3) if beta else None
    return A, B, Co


def rel_err(got, ref):
    n = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / n if n > 0 else np.linalg.norm(got)


def form_of(v):
    """Form of each class under variant v: 'm' matrix cores, else whether the
    vector-unit form takes several products per step."""
    return tuple("m" if d > 16 else (d in (1, 8)) for d in bsmm.bsmm_small_variant(v))


def class_of_values(M):
    """Shape class (0 8x8, 1 8x16, 2 16x8, 3 16x16) of every value of M."""
    rows = np.repeat(np.arange(M.nbrows), np.diff(M.row_ptr))
    m = M.row_sizes[rows]
    n = M.col_sizes[M.col_idx]
    cls = (m > 8).astype(int) * 2 + (n > 8).astype(int)
    return np.repeat(cls, m * n)


def run_variants(dA, dB, dCin, A, B, key, variants):
    bsmm.bsmm_tune_set(key, variants)
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(0.75, dA, dB, -0.5, dCin, dC, 0.0)
    s = bsmm.bsmm_stats(dC.handle)
    out = dC.to_host()
    dC.close()
    return s, out


def test_variants_of_one_form_give_the_same_bits(table):
    A, B, Co = operands(401, 1.0)
    ref = oracle.multiply(0.75, A, B, -0.5, Co, 0.0)
    dA, dB, dCin = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B), bsmm.Matrix.from_csr(Co)
    key = bsmm.bsmm_tune_key(dA.handle, dB.handle)
    first = {}
    runs = {}
    for v in range(bsmm.BSMM_SMALL_VARIANTS):
        s, (rp, ci, vals) = run_variants(dA, dB, dCin, A, B, key, [v] * 4)
        # the variant for block edges of at most 8 falls back to variant 1 here
        used = 1 if bsmm.bsmm_small_variant(v)[0] == 8 else v
        assert s["path"] == bsmm.BSMM_PATH_SMALL and s["variants"] == [used] * 4
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
        assert rel_err(vals, ref.values) <= REL_TOL
        runs[v] = vals
        form = form_of(used)
        if form not in first:
            first[form] = (v, vals)
        else:
            assert np.array_equal(vals, first[form][1]), f"variant {v} differs from variant {first[form][0]}"
    assert len(first) >= 4  # several combinations of forms were run, the matrix-core form among them
    assert any("m" in f for f in first)
    # classes on different variants: each class has the bits of its variant
    C = W.with_pattern(A.row_sizes, B.col_sizes, ref.row_ptr, ref.col_idx, ref.values)
    cls = class_of_values(C)
    assert set(cls.tolist()) == {0, 1, 2, 3}
    for plan in ([6, 1, 7, 0], [0, 6, 3, 7], [7, 7, 1, 6]):
        s, (rp, ci, vals) = run_variants(dA, dB, dCin, A, B, key, plan)
        assert s["variants"] == plan
        assert np.array_equal(ci, ref.col_idx)
        for c in range(4):
            sel = cls == c
            assert np.array_equal(vals[sel], runs[plan[c]][sel]), f"class {c} of plan {plan}"
    for m in (dA, dB, dCin):
        m.close()


def test_variant_for_edges_up_to_8(table):
    # two steps of four 8x8 products in flight: only for block edges <= 8
    rs, ks, cs = [3, 8, 1, 5, 6] * 5, [8, 2, 7, 4] * 6, [6, 8, 3] * 7
    A = W.random_matrix(431, rs, ks, 0.4)
    B = W.random_matrix(432, ks, cs, 0.4)
    Co = W.random_matrix(433, rs, cs, 0.3)
    ref = oracle.multiply(1.25, A, B, 0.5, Co, 0.0)
    dA, dB, dCin = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B), bsmm.Matrix.from_csr(Co)
    key = bsmm.bsmm_tune_key(dA.handle, dB.handle)
    lite = [v for v in range(bsmm.BSMM_SMALL_VARIANTS) if bsmm.bsmm_small_variant(v)[0] == 8]
    assert lite
    vals = {}
    for v in lite + [0]:
        bsmm.bsmm_tune_set(key, [v] * 4)
        dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
        bsmm.multiply(1.25, dA, dB, 0.5, dCin, dC, 0.0)
        assert bsmm.bsmm_stats(dC.handle)["variants"] == [v] * 4
        rp, ci, vals[v] = dC.to_host()
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
        assert rel_err(vals[v], ref.values) <= REL_TOL
        dC.close()
    # every C block is in the 8x8 class, which both variants run four products
    # per step: same operations, same bits
    assert all(np.array_equal(vals[v], vals[0]) for v in lite)
    for m in (dA, dB, dCin):
        m.close()


def test_tuner_result_and_table(table):
    A, B, Co = operands(411, 1.0)
    ref = oracle.multiply(1.0, A, B, 1.0, Co, 0.0)
    dA, dB, dCin = bsmm.Matrix.from_csr(A), bsmm.Matrix.from_csr(B), bsmm.Matrix.from_csr(Co)
    dC = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    key = bsmm.bsmm_tune_key(dA.handle, dB.handle)
    bsmm.bsmm_tune_set(key, None)
    entry = tune.tune(1.0, dA, dB, 1.0, dCin, dC, 0.0, reps=2)
    v = entry["variants"]
    assert len(v) == 4 and all(0 <= x < bsmm.BSMM_SMALL_VARIANTS for x in v)
    assert entry["depths"] == [bsmm.bsmm_small_variant(x)[c] for c, x in enumerate(v)]
    assert tune.edges_key(entry["rows"], entry["inner"], entry["cols"]) == key
    ms = np.array(entry["ms"])
    assert ms.shape == (bsmm.BSMM_SMALL_VARIANTS, 4)
    for u in range(bsmm.BSMM_SMALL_VARIANTS):
        # the variant for block edges of at most 8 is not timed for these sizes
        assert np.all(ms[u] == 0) if bsmm.bsmm_small_variant(u)[0] == 8 else np.all(ms[u] > 0)
    # each class took its fastest variant
    for c in range(4):
        timed = [u for u in range(bsmm.BSMM_SMALL_VARIANTS) if ms[u, c] > 0]
        assert ms[v[c], c] == min(ms[u, c] for u in timed)
    assert bsmm.bsmm_tune_get(key) == v
    assert bsmm.bsmm_stats(dC.handle)["variants"] == v
    rp, ci, vals = dC.to_host()
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    assert rel_err(vals, ref.values) <= REL_TOL
    # a later multiply with the same edge sets uses the tuned variant, same bits
    dC2 = bsmm.Matrix.empty(A.row_sizes, B.col_sizes)
    bsmm.multiply(1.0, dA, dB, 1.0, dCin, dC2, 0.0)
    assert bsmm.bsmm_stats(dC2.handle)["variants"] == v
    assert np.array_equal(dC2.to_host()[2], vals)
    for m in (dA, dB, dCin, dC, dC2):
        m.close()


def test_tuner_other_paths_and_errors(table):
    sizes = [23] * 6
    A = bsmm.Matrix.from_csr(W.random_matrix(421, sizes, sizes, 0.5))
    C = bsmm.Matrix.empty(sizes, sizes)
    before = bsmm.bsmm_tune_entries()
    v, ms = bsmm.bsmm_tune_small(1.0, A.handle, A.handle, 0.0, None, C.handle, 0.0, 2)
    assert v == [-1] * 4 and not ms.any() and bsmm.bsmm_tune_entries() == before
    assert bsmm.bsmm_stats(C.handle)["path"] == bsmm.BSMM_PATH_TILE23
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.bsmm_tune_key(A.handle, A.handle)
    assert e.value.status == "BSMM_E_UNSUPPORTED"
    S = W.random_matrix(422, [5, 13] * 3, [5, 13] * 3, 0.5)
    dS = bsmm.Matrix.from_csr(S)
    dT = bsmm.Matrix.from_csr(S)
    for reps in (0, 1001):
        with pytest.raises(bsmm.BsmmError) as e:
            bsmm.bsmm_tune_small(1.0, dS.handle, dS.handle, 0.0, None, dT.handle, 0.0, reps)
        assert e.value.status == "BSMM_E_ARG"
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.bsmm_tune_small(1.0, dS.handle, dS.handle, 1.0, dT.handle, dT.handle, 0.0, 1)
    assert e.value.status == "BSMM_E_ARG"
    for m in (A, C, dS, dT):
        m.close()
