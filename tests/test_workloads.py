"""Seeded input generators: determinism and the shapes the paper's workloads
prescribe (one 23-block per water molecule; O/H atom blocks of 13 and 5)."""
import numpy as np

from paper_1708_03604_amd import workloads as W


def _same(a, b):
    for f in ("row_sizes", "col_sizes", "row_ptr", "col_idx", "values"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_grid23_shape_and_determinism():
    w = W.grid23()
    assert w.A.nbrows == 64 and w.info["N"] == 1472
    assert np.all(w.A.row_sizes == 23)
    dens = w.A.nnzb / 64 ** 2
    assert 0.27 < dens < 0.33
    assert w.beta == 0.0 and w.eps == 0.0
    _same(w.A, W.grid23().A)
    assert np.all(np.abs(w.A.values) <= 1.0)


def test_molecules_shape():
    # full size is 2048 molecules (N = 47104); a smaller box keeps this CPU test fast
    w = W.molecules(nmol=512)
    A = w.A
    assert A.nbrows == 512 and w.info["N"] == 512 * 23
    per_row = np.diff(A.row_ptr)
    assert 15 < per_row.mean() < 30          # open box, 6 A cutoff at 0.033 / A^3
    # symmetric pattern with the diagonal present
    m = np.zeros((512, 512), dtype=bool)
    m[A.block_rows(), A.col_idx] = True
    assert np.array_equal(m, m.T) and m.diagonal().all()
    assert np.array_equal(w.B.col_idx, A.col_idx) and np.array_equal(w.C_old.col_idx, A.col_idx)
    assert not np.array_equal(w.A.values, w.B.values)
    assert w.beta == 1.0 and w.eps == 1e-6
    # values bounded by the decay envelope
    assert np.all(np.abs(A.values) <= 1.0)


def test_water_atoms_shape():
    w = W.water_atoms(nmol=300)
    A = w.A
    assert A.nbrows == 900
    assert np.array_equal(A.row_sizes[:6], [13, 5, 5, 13, 5, 5])
    assert w.info["N"] == 300 * 23
    # each molecule's three atoms see each other (O-H 0.96 A, H-H 1.5 A < 5 A)
    m = np.zeros((900, 900), dtype=bool)
    m[A.block_rows(), A.col_idx] = True
    for mol in range(300):
        assert m[3 * mol:3 * mol + 3, 3 * mol:3 * mol + 3].all()
    _same(A, W.water_atoms(nmol=300).A)


def test_symmetric_scaled_is_symmetric_and_bounded():
    H, info = W.symmetric_scaled(nmol=128)
    from helpers import dense
    D = dense(H)
    assert np.array_equal(D, D.T)
    assert np.abs(D).sum(axis=1).max() <= 1.0 + 1e-12
    assert np.max(np.abs(np.linalg.eigvalsh(D))) <= 1.0 + 1e-12


def test_random_matrix_int_values():
    M = W.random_matrix(3, [5, 13], [13, 5, 23], 0.7, kind="int")
    assert np.all(M.values == np.round(M.values)) and np.all(np.abs(M.values) <= 4)
    assert len(M.values) == M.nvals


def test_semi_empirical_shape():
    # full size is 186,624 molecules; a smaller box at the same density keeps this fast
    w = W.semi_empirical(nmol=12000)
    A = w.A
    assert A.nbrows == 12000 and np.all(A.row_sizes == 6) and w.info["N"] == 72000
    per_row = np.diff(A.row_ptr)
    # 8.7 A cutoff at 0.0334 / A^3: 92 neighbours in the bulk (0.05% of 186,624)
    L = w.info["box"]
    assert 60 < per_row.mean() < 92
    m = np.zeros((12000, 12000), dtype=bool)
    m[A.block_rows(), A.col_idx] = True
    assert np.array_equal(m, m.T) and m.diagonal().all()
    assert np.array_equal(w.B.col_idx, A.col_idx) and not np.array_equal(w.A.values, w.B.values)
    assert w.C_old is None and w.beta == 0.0 and w.eps == 0.07
    assert abs(L - (12000 / 0.0334) ** (1 / 3)) < 1e-9
    assert np.all(np.abs(A.values) <= 1.0)
    _same(A, W.semi_empirical(nmol=12000).A)


def test_mixed_dense_shape():
    w = W.mixed_dense()
    A = w.A
    assert A.nbrows == 64 and A.nnzb == 64 * 64 and w.info["N"] == 1332
    assert list(A.row_sizes[:6]) == [9, 22, 32, 9, 22, 32]
    assert np.array_equal(A.row_sizes, A.col_sizes)
    assert A.nvals == 1332 * 1332 and w.C_old.nnzb == 64 * 64
    assert w.beta == 1.0 and w.eps == 0.0
    _same(A, W.mixed_dense().A)


def test_block_stream_shape():
    w = W.block_stream(8005, 5, 7, 3, 11)
    assert w.A.nnzb == w.B.nnzb == w.C_old.nnzb == 11
    assert np.array_equal(w.A.col_idx, np.arange(11)) and np.array_equal(w.A.row_ptr, np.arange(12))
    assert np.all(w.A.row_sizes == 5) and np.all(w.A.col_sizes == 3)
    assert np.all(w.B.row_sizes == 3) and np.all(w.B.col_sizes == 7)
    assert w.A.nvals == 11 * 15 and w.B.nvals == 11 * 21 and w.C_old.nvals == 11 * 35
    assert w.beta == 1.0 and w.alpha == 1.0
