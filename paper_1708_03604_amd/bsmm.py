"""Thin ctypes binding of libbsmm (see include/bsmm.h).

Argument marshalling only: every step of the multiply runs in the HIP library.
The functions carry the C names; each raises BsmmError on a non-OK status.
Host arrays are numpy arrays; device arrays are torch tensors on a ROCm
device, which is also where streams come from.

If libbsmm.so has not been built, loading fails loudly: there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsmm.so")

BSMM_OK = 0
STATUS_NAMES = {0: "BSMM_OK", 1: "BSMM_E_ARG", 2: "BSMM_E_SHAPE", 3: "BSMM_E_PATTERN", 4: "BSMM_E_ALIAS",
                5: "BSMM_E_NOMEM", 6: "BSMM_E_CAPACITY", 7: "BSMM_E_HIP", 8: "BSMM_E_UNSUPPORTED"}
BSMM_FP64 = 0
BSMM_SPLIT_F32X2 = 1
BSMM_SPLIT_BF16X3 = 2
BSMM_SLICE_INT8X7 = 3
BSMM_PTR_HOST = 0
BSMM_PTR_DEVICE = 1
BSMM_PATH_GENERIC = 0
BSMM_PATH_TILE23 = 1
BSMM_PATH_SMALL = 2
BSMM_PATH_SPLIT23 = 3
BSMM_PATH_SLICE23 = 4
BSMM_SMALL_VARIANTS = 8
BSMM_MID_VARIANTS = 8


class BsmmError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS_NAMES.get(code, str(code))


class MultStats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("products", ctypes.c_int64), ("nnzb", ctypes.c_int64),
                ("nvals", ctypes.c_int64), ("useful_flops", ctypes.c_double), ("path", ctypes.c_int32),
                ("variants", ctypes.c_int32 * 4), ("panels", ctypes.c_int32)]


# every function declared in include/bsmm.h, with its ctypes signature
_vp, _i32, _i64, _dbl, _int = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int
_u64 = ctypes.c_uint64
SIGNATURES = {
    "bsmm_create": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _int, _vp], _int),
    "bsmm_destroy": ([_vp], _int),
    "bsmm_multiply": ([_dbl, _vp, _vp, _dbl, _vp, _vp, _dbl, _int, _vp], _int),
    "bsmm_filter": ([_vp, _dbl, _vp], _int),
    "bsmm_filter_noalloc": ([_vp, _dbl, _vp], _int),
    "bsmm_norms": ([_vp, _vp, _vp], _int),
    "bsmm_info": ([_vp, _vp, _vp, _vp, _vp], _int),
    "bsmm_export": ([_vp, _vp, _vp, _vp, _int, _vp], _int),
    "bsmm_export_stack": ([_vp, _vp, _vp, _vp, _vp, _int, _vp], _int),
    "bsmm_stats": ([_vp, _vp], _int),
    "bsmm_timing": ([_vp, _int], _int),
    "bsmm_phase_times": ([_vp, _vp, _vp], _int),
    "bsmm_last_error": ([], ctypes.c_char_p),
    "bsmm_reserve": ([_vp, _i64, _i64, _i64, _vp], _int),
    "bsmm_set_stack_limit": ([_vp, _i64], _int),
    "bsmm_frobenius": ([_vp, _vp, _vp], _int),
    "bsmm_capture_begin": ([_vp], _int),
    "bsmm_capture_end": ([_vp, _vp], _int),
    "bsmm_graph_launch": ([_vp, _vp], _int),
    "bsmm_graph_destroy": ([_vp], _int),
    "bsmm_tune_small": ([_dbl, _vp, _vp, _dbl, _vp, _vp, _dbl, _i32, _vp, _vp, _vp], _int),
    "bsmm_small_variant": ([_i32, _vp], _int),
    "bsmm_tune_key": ([_vp, _vp, _vp], _int),
    "bsmm_tune_set": ([_u64, _vp], _int),
    "bsmm_tune_get": ([_u64, _vp], _int),
    "bsmm_tune_entries": ([_vp, _vp, _i32, _vp], _int),
    "bsmm_tune_mid": ([_dbl, _vp, _vp, _dbl, _vp, _vp, _dbl, _i32, _vp, _vp, _vp], _int),
    "bsmm_mid_key": ([_vp, _vp, _vp], _int),
    "bsmm_mid_set": ([_vp, _i32], _int),
    "bsmm_mid_get": ([_vp, _vp], _int),
    "bsmm_mid_entries": ([_vp, _vp, _i32, _vp], _int),
}

_lib = None


def lib():
    """Load libbsmm.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1708_03604_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        from . import tune
        if os.path.exists(tune.TABLE):
            tune.load(tune.TABLE)
    return _lib


def _check(fn, rc):
    if rc != BSMM_OK:
        raise BsmmError(rc, fn, lib().bsmm_last_error().decode())


def _stream(stream):
    if stream is not None:
        return getattr(stream, "cuda_stream", stream)
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except ImportError:
        pass
    return None


def _addr(x):
    """(address, kind) of a numpy array (host) or a torch tensor (its device)."""
    if x is None:
        return None, BSMM_PTR_HOST
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be contiguous")
        return (x.ctypes.data if x.size else None), BSMM_PTR_HOST
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return (x.data_ptr() if x.numel() else None), (BSMM_PTR_DEVICE if x.is_cuda else BSMM_PTR_HOST)
    raise TypeError(type(x))


# ------------------------------------------------------------ C functions

def bsmm_create(nbrows, nbcols, row_sizes, col_sizes, nnzb, row_ptr, col_idx, values, ptr_kind=None,
                stream=None):
    rs = np.ascontiguousarray(row_sizes, dtype=np.int32)
    cs = np.ascontiguousarray(col_sizes, dtype=np.int32)
    prp, k1 = _addr(row_ptr)
    pci, k2 = _addr(col_idx)
    pv, k3 = _addr(values)
    if ptr_kind is None:
        ptr_kind = k1
    h = ctypes.c_void_p()
    rc = lib().bsmm_create(ctypes.byref(h), int(nbrows), int(nbcols), rs.ctypes.data if rs.size else None,
                           cs.ctypes.data if cs.size else None, int(nnzb), prp, pci, pv, int(ptr_kind),
                           _stream(stream))
    _check("bsmm_create", rc)
    return h


def bsmm_destroy(h):
    _check("bsmm_destroy", lib().bsmm_destroy(h))


def bsmm_multiply(alpha, A, B, beta, C_in, C_out, filter_eps, prec=BSMM_FP64, stream=None):
    rc = lib().bsmm_multiply(float(alpha), A, B, float(beta), C_in, C_out, float(filter_eps), int(prec),
                             _stream(stream))
    _check("bsmm_multiply", rc)


def bsmm_filter(M, eps, stream=None):
    _check("bsmm_filter", lib().bsmm_filter(M, float(eps), _stream(stream)))


def bsmm_filter_noalloc(M, eps, stream=None):
    _check("bsmm_filter_noalloc", lib().bsmm_filter_noalloc(M, float(eps), _stream(stream)))


def bsmm_norms(M, out, stream=None):
    p, _ = _addr(out)
    _check("bsmm_norms", lib().bsmm_norms(M, p, _stream(stream)))


def bsmm_info(M):
    nbr, nbc, nnzb, nv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check("bsmm_info", lib().bsmm_info(M, ctypes.byref(nbr), ctypes.byref(nbc), ctypes.byref(nnzb),
                                         ctypes.byref(nv)))
    return nbr.value, nbc.value, nnzb.value, nv.value


def bsmm_export(M, row_ptr, col_idx, values, ptr_kind=None, stream=None):
    a, k = _addr(row_ptr)
    b, _ = _addr(col_idx)
    c, _ = _addr(values)
    _check("bsmm_export", lib().bsmm_export(M, a, b, c, int(k if ptr_kind is None else ptr_kind),
                                             _stream(stream)))


def bsmm_export_stack(C, st_c, st_a, st_b, ptr_kind=None, stream=None):
    a, k = _addr(st_c)
    b, _ = _addr(st_a)
    c, _ = _addr(st_b)
    n = ctypes.c_int64()
    _check("bsmm_export_stack", lib().bsmm_export_stack(C, a, b, c, ctypes.byref(n),
                                                         int(k if ptr_kind is None else ptr_kind),
                                                         _stream(stream)))
    return n.value


def bsmm_stats(C):
    s = MultStats()
    _check("bsmm_stats", lib().bsmm_stats(C, ctypes.byref(s)))
    return {f: (list(getattr(s, f)) if f == "variants" else getattr(s, f)) for f, _ in MultStats._fields_}


PHASES = ("norms", "count", "sizing", "fill", "numeric", "total")


def bsmm_timing(C, enable):
    _check("bsmm_timing", lib().bsmm_timing(C, int(enable)))


def bsmm_phase_times(C):
    ms = np.zeros(len(PHASES), dtype=np.float64)
    n = ctypes.c_int64()
    _check("bsmm_phase_times", lib().bsmm_phase_times(C, ms.ctypes.data, ctypes.byref(n)))
    return dict(zip(PHASES, ms.tolist())), n.value


def bsmm_last_error():
    return lib().bsmm_last_error().decode()


def bsmm_reserve(M, max_nnzb, max_nvals, max_products, stream=None):
    _check("bsmm_reserve", lib().bsmm_reserve(M, int(max_nnzb), int(max_nvals), int(max_products),
                                              _stream(stream)))


def bsmm_set_stack_limit(M, max_products):
    _check("bsmm_set_stack_limit", lib().bsmm_set_stack_limit(M, int(max_products)))


def bsmm_frobenius(M, out, stream=None):
    p, _ = _addr(out)
    _check("bsmm_frobenius", lib().bsmm_frobenius(M, p, _stream(stream)))


def bsmm_capture_begin(stream):
    _check("bsmm_capture_begin", lib().bsmm_capture_begin(_stream(stream)))


def bsmm_capture_end(stream):
    g = ctypes.c_void_p()
    _check("bsmm_capture_end", lib().bsmm_capture_end(_stream(stream), ctypes.byref(g)))
    return g


def bsmm_graph_launch(g, stream=None):
    _check("bsmm_graph_launch", lib().bsmm_graph_launch(g, _stream(stream)))


def bsmm_graph_destroy(g):
    _check("bsmm_graph_destroy", lib().bsmm_graph_destroy(g))


def bsmm_tune_small(alpha, A, B, beta, C_in, C_out, filter_eps, reps=5, stream=None):
    """Returns (chosen variant per class, a list of 4 (all -1 if another path
    serves the sizes), per variant and class milliseconds [BSMM_SMALL_VARIANTS, 4])."""
    v = np.zeros(4, dtype=np.int32)
    ms = np.zeros((BSMM_SMALL_VARIANTS, 4), dtype=np.float64)
    _check("bsmm_tune_small", lib().bsmm_tune_small(float(alpha), A, B, float(beta), C_in, C_out, float(filter_eps),
                                                    int(reps), v.ctypes.data, ms.ctypes.data, _stream(stream)))
    return v.tolist(), ms


def bsmm_small_variant(v):
    d = np.zeros(4, dtype=np.int32)
    _check("bsmm_small_variant", lib().bsmm_small_variant(int(v), d.ctypes.data))
    return d.tolist()


def bsmm_tune_key(A, B):
    k = ctypes.c_uint64()
    _check("bsmm_tune_key", lib().bsmm_tune_key(A, B, ctypes.byref(k)))
    return k.value


def bsmm_tune_set(key, variants):
    """Enter one variant per class (a sequence of 4), or remove the entry (None)."""
    if variants is None:
        _check("bsmm_tune_set", lib().bsmm_tune_set(int(key), None))
        return
    v = np.ascontiguousarray(variants, dtype=np.int32)
    if v.shape != (4,):
        raise ValueError("one variant per class: 4 values")
    _check("bsmm_tune_set", lib().bsmm_tune_set(int(key), v.ctypes.data))


def bsmm_tune_get(key):
    """The entry's variants per class (a list of 4), all -1 if there is none."""
    v = np.zeros(4, dtype=np.int32)
    _check("bsmm_tune_get", lib().bsmm_tune_get(int(key), v.ctypes.data))
    return v.tolist()


def bsmm_tune_entries():
    n = ctypes.c_int32()
    _check("bsmm_tune_entries", lib().bsmm_tune_entries(None, None, 0, ctypes.byref(n)))
    keys = np.zeros(max(n.value, 1), dtype=np.uint64)
    vs = np.zeros((max(n.value, 1), 4), dtype=np.int32)
    _check("bsmm_tune_entries", lib().bsmm_tune_entries(keys.ctypes.data, vs.ctypes.data, n.value, ctypes.byref(n)))
    return {k: v.tolist() for k, v in zip(keys[:n.value].tolist(), vs[:n.value])}


def bsmm_tune_mid(alpha, A, B, beta, C_in, C_out, filter_eps, reps=5, stream=None):
    """Returns (chosen variant of the generic path, -1 if another path serves
    the sizes; milliseconds per variant [BSMM_MID_VARIANTS])."""
    v = ctypes.c_int32()
    ms = np.zeros(BSMM_MID_VARIANTS, dtype=np.float64)
    _check("bsmm_tune_mid", lib().bsmm_tune_mid(float(alpha), A, B, float(beta), C_in, C_out, float(filter_eps),
                                                int(reps), ctypes.byref(v), ms.ctypes.data, _stream(stream)))
    return v.value, ms


def _masks(masks):
    m = np.ascontiguousarray(masks, dtype=np.uint32)
    if m.shape != (3,):
        raise ValueError("three edge masks: A rows, A columns, B columns")
    return m


def bsmm_mid_key(A, B):
    m = np.zeros(3, dtype=np.uint32)
    _check("bsmm_mid_key", lib().bsmm_mid_key(A, B, m.ctypes.data))
    return tuple(int(x) for x in m)


def bsmm_mid_set(masks, variant):
    """Enter `variant` for the edge masks, or remove the entry (variant -1 or None)."""
    m = _masks(masks)
    _check("bsmm_mid_set", lib().bsmm_mid_set(m.ctypes.data, -1 if variant is None else int(variant)))


def bsmm_mid_get(masks):
    m = _masks(masks)
    v = ctypes.c_int32()
    _check("bsmm_mid_get", lib().bsmm_mid_get(m.ctypes.data, ctypes.byref(v)))
    return v.value


def bsmm_mid_entries():
    n = ctypes.c_int32()
    _check("bsmm_mid_entries", lib().bsmm_mid_entries(None, None, 0, ctypes.byref(n)))
    ms = np.zeros((max(n.value, 1), 3), dtype=np.uint32)
    vs = np.zeros(max(n.value, 1), dtype=np.int32)
    _check("bsmm_mid_entries", lib().bsmm_mid_entries(ms.ctypes.data, vs.ctypes.data, n.value, ctypes.byref(n)))
    return {tuple(int(x) for x in m): int(v) for m, v in zip(ms[:n.value], vs[:n.value])}


# ------------------------------------------------------------ convenience

class Matrix:
    """Owning wrapper of a bsmm_mat handle."""

    def __init__(self, handle, row_sizes, col_sizes):
        self.handle = handle
        self.row_sizes = np.ascontiguousarray(row_sizes, dtype=np.int32)
        self.col_sizes = np.ascontiguousarray(col_sizes, dtype=np.int32)

    @classmethod
    def from_csr(cls, M, stream=None):
        """Upload a host block-CSR matrix (attributes row_sizes, col_sizes,
        row_ptr, col_idx, values)."""
        rp = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
        v = np.ascontiguousarray(M.values, dtype=np.float64)
        h = bsmm_create(len(M.row_sizes), len(M.col_sizes), M.row_sizes, M.col_sizes, len(ci), rp, ci, v,
                        BSMM_PTR_HOST, stream)
        return cls(h, M.row_sizes, M.col_sizes)

    @classmethod
    def empty(cls, row_sizes, col_sizes, stream=None):
        rp = np.zeros(len(row_sizes) + 1, dtype=np.int32)
        h = bsmm_create(len(row_sizes), len(col_sizes), row_sizes, col_sizes, 0, rp, None, None, BSMM_PTR_HOST,
                        stream)
        return cls(h, row_sizes, col_sizes)

    def info(self):
        return bsmm_info(self.handle)

    def to_host(self, stream=None):
        """(row_ptr, col_idx, values) as numpy arrays."""
        nbr, _, nnzb, nv = self.info()
        rp = np.zeros(nbr + 1, dtype=np.int32)
        ci = np.zeros(max(nnzb, 1), dtype=np.int32)
        v = np.zeros(max(nv, 1), dtype=np.float64)
        bsmm_export(self.handle, rp, ci if nnzb else None, v if nv else None, BSMM_PTR_HOST, stream)
        return rp, ci[:nnzb], v[:nv]

    def stack(self, stream=None):
        n = bsmm_export_stack(self.handle, None, None, None, BSMM_PTR_HOST, stream)
        out = np.zeros((3, max(n, 1)), dtype=np.int32)
        bsmm_export_stack(self.handle, out[0], out[1], out[2], BSMM_PTR_HOST, stream)
        return np.ascontiguousarray(out[:, :n].T)

    def close(self):
        if self.handle is not None:
            bsmm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def multiply(alpha, A, B, beta, C_in, C_out, eps, prec=BSMM_FP64, stream=None):
    bsmm_multiply(alpha, A.handle, B.handle, beta, C_in.handle if C_in is not None else None, C_out.handle, eps,
                  prec, stream)
