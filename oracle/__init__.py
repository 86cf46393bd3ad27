"""CPU FP64 oracle for the DBCSR block-sparse multiply -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It never imports the GPU library and the
GPU library never imports it.  The arithmetic lives in ``oracle.c`` (plain C,
FP64, ``-ffp-contract=off``); this file only marshals numpy arrays.

Matrices are passed duck-typed: any object with the numpy attributes
``row_sizes``, ``col_sizes``, ``row_ptr``, ``col_idx`` (int32) and ``values``
(float64, row-major blocks, contiguous in CSR order).

Paper: Bethune et al., "Porting of the DBCSR library for Sparse Matrix-Matrix
Multiplications to Intel Xeon Phi systems" (2017), Section 2 (blocked CSR
storage, pairwise block products C = C + A*B, on-the-fly norm filter) and
Section 1.1 (Gustavson's row-wise algorithm).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, E_ARG, E_SHAPE, E_PATTERN, E_NOMEM, E_CAPACITY = 0, 1, 2, 3, 5, 6


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


FLAGS = ["-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared"]


def build():
    """Compile oracle.c into liboracle.so (plain gcc, OpenMP over block rows)."""
    cmd = ["gcc"] + FLAGS + ["-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.check_call(cmd)


def use_native_build(directory):
    """Compile oracle.c for the CPU this process runs on (adds -march=native;
    still no FP contraction, so the results are the same bits) into
    `directory` and use that library from now on.  Returns the compile line."""
    global _lib
    path = os.path.join(directory, "liboracle_native.so")
    cmd = ["gcc"] + FLAGS + ["-march=native", "-o", path, _SRC, "-lm"]
    subprocess.check_call(cmd)
    _lib = None
    _load(path)
    return " ".join(cmd[:len(FLAGS) + 2])


def set_threads(n):
    """OpenMP threads of the oracle's row loop (the runtime it is linked with)."""
    import ctypes.util
    gomp = ctypes.CDLL(ctypes.util.find_library("gomp") or "libgomp.so.1")
    gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


class _Mat(ctypes.Structure):
    _fields_ = [
        ("nbrows", ctypes.c_int32),
        ("nbcols", ctypes.c_int32),
        ("row_sizes", ctypes.c_void_p),
        ("col_sizes", ctypes.c_void_p),
        ("nnzb", ctypes.c_int32),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("values", ctypes.c_void_p),
    ]


_lib = None


def _load(path=None):
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = _LIB_PATH
        stale = (not os.path.exists(_LIB_PATH)
                 or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC))
        if stale:
            build()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(_Mat)
    vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    lib.oracle_check.argtypes = [P]
    lib.oracle_check.restype = ctypes.c_int
    lib.oracle_norms.argtypes = [P, vp]
    lib.oracle_norms.restype = ctypes.c_int
    lib.oracle_value_count.argtypes = [P]
    lib.oracle_value_count.restype = i64
    lib.oracle_multiply.argtypes = [dbl, P, P, dbl, P, dbl, i64, i64, i64,
                                    vp, vp, vp, vp, vp, vp, vp]
    lib.oracle_multiply.restype = ctypes.c_int
    lib.oracle_filter.argtypes = [P, dbl, i64, i64, vp, vp, vp, vp]
    lib.oracle_filter.restype = ctypes.c_int
    lib.oracle_frobenius.argtypes = [P]
    lib.oracle_frobenius.restype = dbl
    _lib = lib
    return lib


class Matrix:
    """Plain container for a block-CSR matrix produced by the oracle."""

    def __init__(self, row_sizes, col_sizes, row_ptr, col_idx, values):
        self.row_sizes = np.ascontiguousarray(row_sizes, dtype=np.int32)
        self.col_sizes = np.ascontiguousarray(col_sizes, dtype=np.int32)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.values = np.ascontiguousarray(values, dtype=np.float64)

    @property
    def nbrows(self):
        return len(self.row_sizes)

    @property
    def nbcols(self):
        return len(self.col_sizes)

    @property
    def nnzb(self):
        return len(self.col_idx)


class Product(Matrix):
    """Result of ``multiply``: the matrix plus its product stack.

    ``stack`` is an int32 array of shape (nprod, 3): (C block, A block, B block)
    for every kept block product, sorted by C block and then inner index k.
    """

    def __init__(self, row_sizes, col_sizes, row_ptr, col_idx, values, stack):
        super().__init__(row_sizes, col_sizes, row_ptr, col_idx, values)
        self.stack = stack


def _as_struct(M, keep):
    arrs = [np.ascontiguousarray(M.row_sizes, dtype=np.int32),
            np.ascontiguousarray(M.col_sizes, dtype=np.int32),
            np.ascontiguousarray(M.row_ptr, dtype=np.int32),
            np.ascontiguousarray(M.col_idx, dtype=np.int32),
            np.ascontiguousarray(M.values, dtype=np.float64)]
    keep.extend(arrs)
    rs, cs, rp, ci, v = arrs
    # numpy returns NULL-ish pointers for empty arrays; give them a 1-element home
    def ptr(a):
        if a.size == 0:
            z = np.zeros(1, dtype=a.dtype)
            keep.append(z)
            return z.ctypes.data
        return a.ctypes.data
    return _Mat(len(rs), len(cs), ptr(rs), ptr(cs), len(ci), ptr(rp), ptr(ci), ptr(v))


def check(M):
    """Status code of the blocked-CSR well-formedness check (0 = valid)."""
    keep = []
    s = _as_struct(M, keep)
    return _load().oracle_check(ctypes.byref(s))


def norms(M):
    """Frobenius norm of every stored block, in the fixed summation order."""
    keep = []
    s = _as_struct(M, keep)
    out = np.zeros(max(s.nnzb, 1), dtype=np.float64)
    rc = _load().oracle_norms(ctypes.byref(s), out.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "norms")
    return out[: s.nnzb]


def multiply(alpha, A, B, beta=0.0, C_old=None, eps=0.0):
    """C = alpha*A*B + beta*C_old with on-the-fly filter eps (see oracle.c)."""
    lib = _load()
    keep = []
    sa = _as_struct(A, keep)
    sb = _as_struct(B, keep)
    so = _as_struct(C_old, keep) if C_old is not None else None
    po = ctypes.byref(so) if so is not None else None
    counts = np.zeros(3, dtype=np.int64)
    nbrows = sa.nbrows
    rp = np.zeros(nbrows + 1, dtype=np.int32)
    dummy_i = np.zeros(1, dtype=np.int32)
    dummy_d = np.zeros(1, dtype=np.float64)
    rc = lib.oracle_multiply(alpha, ctypes.byref(sa), ctypes.byref(sb), beta, po, eps, 0, 0, 0,
                             rp.ctypes.data, dummy_i.ctypes.data, dummy_d.ctypes.data,
                             dummy_i.ctypes.data, dummy_i.ctypes.data, dummy_i.ctypes.data,
                             counts.ctypes.data)
    if rc not in (OK, E_CAPACITY):
        raise OracleError(rc, "multiply")
    nnzb, nvals, nprod = (int(x) for x in counts)
    ci = np.zeros(max(nnzb, 1), dtype=np.int32)
    vals = np.zeros(max(nvals, 1), dtype=np.float64)
    st = np.zeros((3, max(nprod, 1)), dtype=np.int32)
    rc = lib.oracle_multiply(alpha, ctypes.byref(sa), ctypes.byref(sb), beta, po, eps,
                             nnzb, nvals, nprod, rp.ctypes.data, ci.ctypes.data,
                             vals.ctypes.data, st[0].ctypes.data, st[1].ctypes.data,
                             st[2].ctypes.data, counts.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "multiply")
    stack = np.ascontiguousarray(st[:, :nprod].T)
    return Product(A.row_sizes, B.col_sizes, rp, ci[:nnzb], vals[:nvals], stack)


def filter(M, eps):
    """Drop every block whose norm is not above eps (eps <= 0 keeps all)."""
    lib = _load()
    keep = []
    s = _as_struct(M, keep)
    counts = np.zeros(2, dtype=np.int64)
    rp = np.zeros(s.nbrows + 1, dtype=np.int32)
    ci = np.zeros(max(s.nnzb, 1), dtype=np.int32)
    nv = int(lib.oracle_value_count(ctypes.byref(s)))
    vals = np.zeros(max(nv, 1), dtype=np.float64)
    rc = lib.oracle_filter(ctypes.byref(s), eps, s.nnzb, nv, rp.ctypes.data, ci.ctypes.data,
                           vals.ctypes.data, counts.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "filter")
    nb, nvk = int(counts[0]), int(counts[1])
    return Matrix(M.row_sizes, M.col_sizes, rp, ci[:nb], vals[:nvk])


def frobenius(M):
    """Frobenius norm of the whole matrix (FP64 plain sum of squares)."""
    keep = []
    s = _as_struct(M, keep)
    return float(_load().oracle_frobenius(ctypes.byref(s)))
