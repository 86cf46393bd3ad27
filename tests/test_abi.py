"""The C-ABI library: it loads, exports every function include/bsmm.h declares,
and rejects invalid input on the host before touching a device.  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1708_03604_amd import bsmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "bsmm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bsmm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("bsmm_create", "bsmm_destroy", "bsmm_multiply", "bsmm_filter", "bsmm_norms"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(bsmm.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    # the binding covers the same set with the same names
    assert sorted(bsmm.SIGNATURES) == _declared()


def test_host_side_validation_without_device():
    L = bsmm.lib()
    assert L.bsmm_destroy(None) == 0
    assert L.bsmm_info(None, None, None, None, None) == 1
    assert "NULL" in bsmm.bsmm_last_error()
    rs = np.array([2, 3], dtype=np.int32)
    cs = np.array([4], dtype=np.int32)
    cases = [
        (np.array([0, 2, 1], dtype=np.int32), np.array([0], dtype=np.int32), 1, "BSMM_E_PATTERN"),
        (np.array([1, 1, 1], dtype=np.int32), np.array([0], dtype=np.int32), 1, "BSMM_E_PATTERN"),
        (np.array([0, 1, 2], dtype=np.int32), np.array([0, 1], dtype=np.int32), 2, "BSMM_E_PATTERN"),
        (np.array([0, 2, 2], dtype=np.int32), np.array([0, 0], dtype=np.int32), 2, "BSMM_E_PATTERN"),
    ]
    for rp, ci, nnzb, status in cases:
        with pytest.raises(bsmm.BsmmError) as e:
            bsmm.bsmm_create(2, 1, rs, cs, nnzb, rp, ci, None, bsmm.BSMM_PTR_HOST)
        assert e.value.status == status
    with pytest.raises(bsmm.BsmmError) as e:
        bsmm.bsmm_create(2, 1, np.array([2, 0], dtype=np.int32), cs, 0, np.zeros(3, dtype=np.int32), None, None,
                         bsmm.BSMM_PTR_HOST)
    assert e.value.status == "BSMM_E_ARG"


def test_tuning_table_without_device():
    from paper_1708_03604_amd import tune
    bsmm.lib()
    depths = [bsmm.bsmm_small_variant(v) for v in range(bsmm.BSMM_SMALL_VARIANTS)]
    assert len(set(map(tuple, depths))) == bsmm.BSMM_SMALL_VARIANTS
    assert depths[1] == [1, 2, 2, 2]  # the untuned choice
    for d in depths:
        # vector-unit forms, or the matrix-core form (16 + products in flight) in every class
        assert (d[0] in (1, 4, 8) and d[1] in (1, 2, 4) and d[2] in (1, 2, 4) and d[3] == 2) or \
            (d[0] > 16 and d == [d[0]] * 4)
    with pytest.raises(bsmm.BsmmError):
        bsmm.bsmm_small_variant(bsmm.BSMM_SMALL_VARIANTS)
    key = tune.edges_key([5, 13], [13], [1, 16])
    assert key == (1 << 4) | (1 << 12) | (1 << (16 + 12)) | (1 << 32) | (1 << 47)
    assert tune.key_edges(key) == ([5, 13], [13], [1, 16])
    with pytest.raises(ValueError):
        tune.edges_key([17], [1], [1])
    saved = bsmm.bsmm_tune_entries()
    try:
        bsmm.bsmm_tune_set(key, [3, 6, 0, 7])
        assert bsmm.bsmm_tune_get(key) == [3, 6, 0, 7]
        assert bsmm.bsmm_tune_entries()[key] == [3, 6, 0, 7]
        bsmm.bsmm_tune_set(key, None)
        assert bsmm.bsmm_tune_get(key) == [-1] * 4 and key not in bsmm.bsmm_tune_entries()
        for bad in ([0, 0, 0, bsmm.BSMM_SMALL_VARIANTS], [-1, 0, 0, 0]):
            with pytest.raises(bsmm.BsmmError) as e:
                bsmm.bsmm_tune_set(key, bad)
            assert e.value.status == "BSMM_E_ARG"
        assert key not in bsmm.bsmm_tune_entries()
    finally:
        assert bsmm.bsmm_tune_entries() == saved


def test_saved_tuning_table():
    from paper_1708_03604_amd import tune
    if not os.path.exists(tune.TABLE):
        pytest.skip("no saved table")
    bsmm.lib()  # loads the saved table
    import json
    table = json.load(open(tune.TABLE))
    assert table["arch"] == "gfx950"
    for e in table["entries"]:
        assert all(0 <= v < bsmm.BSMM_SMALL_VARIANTS for v in e["variants"]) and len(e["variants"]) == 4
        assert e["depths"] == [bsmm.bsmm_small_variant(v)[c] for c, v in enumerate(e["variants"])]
        assert bsmm.bsmm_tune_get(tune.edges_key(e["rows"], e["inner"], e["cols"])) == e["variants"]


def test_tuning_table_json_roundtrip(tmp_path):
    from paper_1708_03604_amd import tune
    bsmm.lib()
    saved = bsmm.bsmm_tune_entries()
    entries = [{"rows": [5, 13], "inner": [5, 13], "cols": [5, 13], "variants": [3, 6, 6, 7], "depths": [1, 18, 18, 19]},
               {"rows": [2], "inner": [7, 8], "cols": [1, 16], "variants": [0, 0, 0, 0], "depths": [1, 1, 1, 2]}]
    path = str(tmp_path / "table.json")
    try:
        tune.save(entries, path, note="test")
        loaded = tune.load(path)
        assert loaded == entries
        for e in entries:
            assert bsmm.bsmm_tune_get(tune.edges_key(e["rows"], e["inner"], e["cols"])) == e["variants"]
    finally:
        for k in bsmm.bsmm_tune_entries():
            bsmm.bsmm_tune_set(k, None)
        for k, v in saved.items():
            bsmm.bsmm_tune_set(k, v)


def test_generic_path_table_without_device(tmp_path):
    """The generic path's table (edge masks -> variant) and its JSON form."""
    from paper_1708_03604_amd import tune
    bsmm.lib()
    saved = bsmm.bsmm_mid_entries()
    key = (1 << 8 | 1 << 21 | 1 << 31, 1 << 8, 1 << 31)  # rows {9, 22, >=32}, inner {9}, cols {>=32}
    try:
        assert tune.mask_edges(key[0]) == [9, 22, 32]
        bsmm.bsmm_mid_set(key, 1)
        assert bsmm.bsmm_mid_get(key) == 1 and bsmm.bsmm_mid_entries()[key] == 1
        for bad in (-2, bsmm.BSMM_MID_VARIANTS):
            with pytest.raises(bsmm.BsmmError) as e:
                bsmm.bsmm_mid_set(key, bad)
            assert e.value.status == "BSMM_E_ARG"
        bsmm.bsmm_mid_set(key, None)
        assert bsmm.bsmm_mid_get(key) == -1 and key not in bsmm.bsmm_mid_entries()
        mid = [{"masks": list(key), "rows": [9, 22, 32], "inner": [9], "cols": [32], "variant": 3, "ms": [1, 2, 0, 0]}]
        path = str(tmp_path / "table.json")
        tune.save([], path, note="test", mid_entries=mid)
        assert tune.load(path) == []
        assert bsmm.bsmm_mid_get(key) == 3
    finally:
        for k in bsmm.bsmm_mid_entries():
            bsmm.bsmm_mid_set(k, None)
        for k, v in saved.items():
            bsmm.bsmm_mid_set(k, v)
        assert bsmm.bsmm_mid_entries() == saved
