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
