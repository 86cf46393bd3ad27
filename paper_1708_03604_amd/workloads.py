"""Seeded synthetic block-sparse inputs shaped like the paper's workloads.

This module only builds inputs (block sizes, sparsity patterns and values).
It holds no step of the multiply, so both the GPU path and the CPU oracle may
use it.  Every generator is a pure function of its seed
(``numpy.random.default_rng``, PCG64).

Shapes follow the paper's benchmark descriptions (Section 3.2, Table 1):
one 23x23 block per water molecule (H2O-DFT-LS), atom blocks of 13 (O) and
5 (H) (AMORPH), and an occupancy that comes from a real-space cutoff between
molecules, as in linear-scaling DFT matrices (Section 1).  The CP2K inputs
themselves are not available; these stand in for them.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class BlockCSR:
    """Blocked CSR matrix on the host.

    row_sizes[nbrows], col_sizes[nbcols] : block edge lengths (int32, >= 1)
    row_ptr[nbrows+1], col_idx[nnzb]     : CSR over blocks, columns ascending
    values[nvals]                        : FP64, each block row-major, blocks
                                           contiguous in CSR order
    """

    row_sizes: np.ndarray
    col_sizes: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray

    def __post_init__(self):
        self.row_sizes = np.ascontiguousarray(self.row_sizes, dtype=np.int32)
        self.col_sizes = np.ascontiguousarray(self.col_sizes, dtype=np.int32)
        self.row_ptr = np.ascontiguousarray(self.row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(self.col_idx, dtype=np.int32)
        self.values = np.ascontiguousarray(self.values, dtype=np.float64)

    @property
    def nbrows(self):
        return len(self.row_sizes)

    @property
    def nbcols(self):
        return len(self.col_sizes)

    @property
    def nnzb(self):
        return len(self.col_idx)

    def block_rows(self):
        """Block-row index of every stored block."""
        return np.repeat(np.arange(self.nbrows, dtype=np.int32), np.diff(self.row_ptr))

    def block_elems(self):
        """Element count of every stored block."""
        return (self.row_sizes[self.block_rows()].astype(np.int64)
                * self.col_sizes[self.col_idx].astype(np.int64))

    def block_offsets(self):
        """Offset of every block in ``values`` (length nnzb+1)."""
        off = np.zeros(self.nnzb + 1, dtype=np.int64)
        np.cumsum(self.block_elems(), out=off[1:])
        return off

    @property
    def nvals(self):
        return int(self.block_elems().sum())


@dataclass
class Workload:
    """One multiply C = alpha*A*B + beta*C_old with on-the-fly filter eps."""

    name: str
    A: BlockCSR
    B: BlockCSR
    C_old: BlockCSR = None
    alpha: float = 1.0
    beta: float = 0.0
    eps: float = 0.0
    info: dict = field(default_factory=dict)


# ---------------------------------------------------------------- patterns

def pattern_from_mask(mask):
    """CSR (row_ptr, col_idx) of a dense boolean block mask."""
    mask = np.asarray(mask, dtype=bool)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(mask.shape[0] + 1, dtype=np.int32)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = np.nonzero(mask)[1].astype(np.int32)
    return row_ptr, col_idx


def pattern_from_pairs(n, ii, jj):
    """CSR of an n x n pattern given (unsorted, duplicate-free) coordinates."""
    ii = np.asarray(ii, dtype=np.int64)
    jj = np.asarray(jj, dtype=np.int64)
    order = np.lexsort((jj, ii))
    ii, jj = ii[order], jj[order]
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(ii, minlength=n), out=row_ptr[1:])
    return row_ptr, jj.astype(np.int32)


def cutoff_pairs(pos, cutoff):
    """All ordered pairs (i, j) with |pos_i - pos_j| < cutoff (open box), with
    i == j included, and their distances.  Strict inequality."""
    from scipy.spatial import cKDTree

    tree = cKDTree(pos)
    pairs = tree.query_pairs(r=cutoff, output_type="ndarray")
    if len(pairs):
        d = np.linalg.norm(pos[pairs[:, 0]] - pos[pairs[:, 1]], axis=1)
        keep = d < cutoff
        pairs, d = pairs[keep], d[keep]
    else:
        d = np.zeros(0)
    n = len(pos)
    diag = np.arange(n)
    ii = np.concatenate([pairs[:, 0], pairs[:, 1], diag])
    jj = np.concatenate([pairs[:, 1], pairs[:, 0], diag])
    dd = np.concatenate([d, d, np.zeros(n)])
    return ii, jj, dd


def _csr_with_block_scalars(n, ii, jj, scal):
    """Sort coordinates into CSR and carry one scalar per block along."""
    order = np.lexsort((jj, ii))
    ii, jj, scal = ii[order], jj[order], scal[order]
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(ii, minlength=n), out=row_ptr[1:])
    return row_ptr, jj.astype(np.int32), scal


def values_uniform(seed, elems, scale=None):
    """U[-1,1] per element; optional per-block factor repeated over the block."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, int(np.sum(elems)))
    if scale is not None:
        v *= np.repeat(scale, elems)
    return v


def values_int(seed, nvals, lo=-4, hi=4):
    """Small integers in [lo, hi] stored as FP64 (every sum of products exact)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, int(nvals)).astype(np.float64)


def with_pattern(row_sizes, col_sizes, row_ptr, col_idx, values=None):
    M = BlockCSR(row_sizes, col_sizes, row_ptr, col_idx, np.zeros(0))
    M.values = np.zeros(M.nvals) if values is None else np.ascontiguousarray(values, dtype=np.float64)
    return M


def random_matrix(seed, row_sizes, col_sizes, density, kind="uniform", lo=-4, hi=4):
    """Blocks present i.i.d. with probability ``density``; values U[-1,1] or
    integers in [lo, hi]."""
    rng = np.random.default_rng(seed)
    row_sizes = np.asarray(row_sizes, dtype=np.int32)
    col_sizes = np.asarray(col_sizes, dtype=np.int32)
    mask = rng.random((len(row_sizes), len(col_sizes))) < density
    rp, ci = pattern_from_mask(mask)
    M = with_pattern(row_sizes, col_sizes, rp, ci)
    if kind == "uniform":
        M.values = values_uniform(seed + 7919, M.block_elems())
    elif kind == "int":
        M.values = values_int(seed + 7919, M.nvals, lo, hi)
    else:
        raise ValueError(kind)
    return M


def three_term_values(rng, n):
    """Values x = p + q 2^-9 + r 2^-18 with |p|, |q| in 5..7 and |r| in 1..7
    (random signs), returned as (x, [p, q 2^-9, r 2^-18]).  x is exact in FP64
    (21 significant bits), and its BF16 split by repeated rounding to nearest
    is exactly the three parts (each part stays inside one binade whose BF16
    rounding error bound exceeds the parts below it)."""
    def part(lo, hi):
        return rng.integers(lo, hi + 1, size=n) * rng.choice([-1.0, 1.0], size=n)
    parts = [part(5, 7), part(5, 7) * 2.0 ** -9, part(1, 7) * 2.0 ** -18]
    return parts[0] + parts[1] + parts[2], parts


def three_term_pair(seed, sizes, density=0.5):
    """A and B on random square block patterns with three-term values (see
    three_term_values); every A block has one nonzero per row (at a random
    column), B blocks are full.  Returns (A, B, A_parts, B_parts), the parts
    being three value arrays in A's (B's) layout that sum to its values."""
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int32)
    out = []
    for which in range(2):
        mask = rng.random((len(sizes), len(sizes))) < density
        rp, ci = pattern_from_mask(mask)
        M = with_pattern(sizes, sizes, rp, ci)
        vals, parts = three_term_values(rng, M.nvals)
        if which == 0:
            keep = np.zeros(M.nvals, dtype=bool)
            off = M.block_offsets()
            rows = M.block_rows()
            for b in range(M.nnzb):
                m, n = sizes[rows[b]], sizes[M.col_idx[b]]
                cols = rng.integers(0, n, size=m)
                keep[off[b] + np.arange(m) * n + cols] = True
            vals = np.where(keep, vals, 0.0)
            parts = [np.where(keep, x, 0.0) for x in parts]
        M.values = vals
        out.append((M, parts))
    return out[0][0], out[1][0], out[0][1], out[1][1]


def seven_digit_values(rng, n):
    """Values x = sum_s d_s 2^-(6 + 7(s-1)), s = 1..7, with |d_1| in 33..63 and
    d_2..d_7 in -63..63 (random signs and digits), returned as (x, digits),
    digits an int array of shape (7, n).  x is exact in FP64 (at most 49
    significant bits) and lies in [0.5, 1) in magnitude, so any row or column
    of such values has the power-of-two scale 1, and rounding to nearest
    recovers the digits one by one (every tail is below one half)."""
    d = rng.integers(-63, 64, size=(7, n))
    d[0] = rng.integers(33, 64, size=n) * rng.choice([-1, 1], size=n)
    x = np.zeros(n)
    for s in range(6, -1, -1):  # smallest first: every partial sum is exact
        x = x + d[s] * 2.0 ** -(6 + 7 * s)
    return x, d


def seven_digit_pair(seed, sizes, density=0.5):
    """A and B on random square block patterns, every value a seven-digit
    value (see seven_digit_values).  Returns (A, B, A_digits, B_digits), the
    digits as (7, nvals) arrays in A's (B's) value layout."""
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int32)
    out = []
    for _ in range(2):
        mask = rng.random((len(sizes), len(sizes))) < density
        rp, ci = pattern_from_mask(mask)
        M = with_pattern(sizes, sizes, rp, ci)
        M.values, digits = seven_digit_values(rng, M.nvals)
        out.append((M, digits))
    return out[0][0], out[1][0], out[0][1], out[1][1]


# ------------------------------------------------------- paper-shaped configs

def grid23(seed=1000, nb=64, p=0.3, bs=23):
    """64x64 grid of 23x23 blocks, each A and B block present i.i.d. with p=0.3,
    entries U[-1,1]; beta = 0, no filtering."""
    sizes = np.full(nb, bs, dtype=np.int32)
    A = random_matrix(seed, sizes, sizes, p)
    B = random_matrix(seed + 1, sizes, sizes, p)
    return Workload(f"grid{nb}x{nb}_b{bs}_p{p}", A, B, None, 1.0, 0.0, 0.0,
                    {"N": int(nb * bs)})


def box_side(count, density):
    return (count / density) ** (1.0 / 3.0)


def molecules(seed=2000, nmol=2048, density=0.033, cutoff=6.0, bs=23, eps=1e-6,
              beta=1.0):
    """Water-molecule-blocked matrix (one 23x23 block per molecule, as in
    H2O-DFT-LS): molecule centres uniform in an open cube at ``density``
    molecules per cubic angstrom; block (i,j) present iff the centres are
    closer than ``cutoff``; values U[-1,1]*exp(-0.5*d).  A and B share the
    pattern with independent values (seeds +0, +1); C_old has the same
    pattern (seed +2).  Positions come from seed +100."""
    L = box_side(nmol, density)
    pos = np.random.default_rng(seed + 100).uniform(0.0, L, (nmol, 3))
    ii, jj, dd = cutoff_pairs(pos, cutoff)
    rp, ci, dd = _csr_with_block_scalars(nmol, ii, jj, dd)
    sizes = np.full(nmol, bs, dtype=np.int32)
    decay = np.exp(-0.5 * dd)
    mats = []
    for off in (0, 1, 2):
        M = with_pattern(sizes, sizes, rp, ci)
        M.values = values_uniform(seed + off, M.block_elems(), decay)
        mats.append(M)
    A, B, C = mats
    return Workload(f"molecules{nmol}_b{bs}_cut{cutoff}", A, B, C if beta != 0 else None,
                    1.0, beta, eps, {"N": int(nmol * bs), "box": L, "positions": pos})


def water_atoms(seed=3000, nmol=3000, density=0.0334, cutoff=5.0, o_size=13, h_size=5):
    """Atom-blocked water (AMORPH-like block sizes 13 and 5): molecule centres
    uniform in an open cube; O at the centre, two H at 0.9572 A with an
    H-O-H angle of 104.52 degrees, random orientation; blocks ordered O,H,H
    per molecule; block (a,b) present iff the atoms are closer than
    ``cutoff``; values U[-1,1]*exp(-0.5*d); beta = 0, no filtering."""
    rng = np.random.default_rng(seed + 100)
    L = box_side(nmol, density)
    centres = rng.uniform(0.0, L, (nmol, 3))
    # random rotations from uniform unit quaternions
    q = rng.normal(size=(nmol, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)
    half = np.deg2rad(104.52) / 2.0
    r_oh = 0.9572
    local = np.array([[0.0, 0.0, 0.0],
                      [r_oh * np.sin(half), 0.0, r_oh * np.cos(half)],
                      [-r_oh * np.sin(half), 0.0, r_oh * np.cos(half)]])
    atoms = centres[:, None, :] + np.einsum("mij,aj->mai", R, local)
    pos = atoms.reshape(-1, 3)
    natom = len(pos)
    sizes = np.tile(np.array([o_size, h_size, h_size], dtype=np.int32), nmol)
    ii, jj, dd = cutoff_pairs(pos, cutoff)
    rp, ci, dd = _csr_with_block_scalars(natom, ii, jj, dd)
    decay = np.exp(-0.5 * dd)
    mats = []
    for off in (0, 1):
        M = with_pattern(sizes, sizes, rp, ci)
        M.values = values_uniform(seed + off, M.block_elems(), decay)
        mats.append(M)
    A, B = mats
    return Workload(f"water{nmol}_atoms_b{o_size}_{h_size}_cut{cutoff}", A, B, None, 1.0, 0.0, 0.0,
                    {"N": int(sizes.sum()), "box": L})


def symmetric_scaled(seed=5000, nmol=2048, density=0.033, cutoff=6.0, bs=23):
    """Symmetric H = (R + R^T)/2 on the molecule pattern with exp(-0.5 d)
    decay, divided by its Gershgorin bound max_i sum_j |H_ij| so that its
    spectral radius is at most 1 (input of the sign iteration)."""
    w = molecules(seed, nmol, density, cutoff, bs, 0.0, 0.0)
    R = w.A
    off = R.block_offsets()
    rows = R.block_rows()
    # position of the transposed block (j,i) for each block (i,j)
    key = rows.astype(np.int64) * R.nbcols + R.col_idx
    tkey = R.col_idx.astype(np.int64) * R.nbcols + rows
    pos_t = np.searchsorted(key, tkey)
    vals = np.empty_like(R.values)
    for b in range(R.nnzb):
        m = R.row_sizes[rows[b]]
        n = R.col_sizes[R.col_idx[b]]
        blk = R.values[off[b]:off[b + 1]].reshape(m, n)
        tb = pos_t[b]
        tblk = R.values[off[tb]:off[tb + 1]].reshape(n, m)
        vals[off[b]:off[b + 1]] = (0.5 * (blk + tblk.T)).ravel()
    H = with_pattern(R.row_sizes, R.col_sizes, R.row_ptr, R.col_idx, vals)
    # scalar row sums of |H|
    absrow = np.zeros(int(R.row_sizes.sum()))
    rstart = np.concatenate([[0], np.cumsum(R.row_sizes)])
    for b in range(R.nnzb):
        m = R.row_sizes[rows[b]]
        n = R.col_sizes[R.col_idx[b]]
        blk = np.abs(vals[off[b]:off[b + 1]].reshape(m, n)).sum(axis=1)
        absrow[rstart[rows[b]]:rstart[rows[b]] + m] += blk
    g = float(absrow.max())
    H.values = H.values / g
    return H, {"gershgorin": g, "N": int(R.row_sizes.sum())}


def identity_like(M, scale=1.0):
    """Block-diagonal scale*I with the block sizes of square matrix M."""
    n = M.nbrows
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    blocks = [scale * np.eye(int(s)).ravel() for s in M.row_sizes]
    vals = np.concatenate(blocks) if blocks else np.zeros(0)
    return with_pattern(M.row_sizes, M.col_sizes, rp, ci, vals)


def semi_empirical(seed=6000, nmol=186624, density=0.0334, cutoff=8.7, bs=6, eps=0.07):
    """S-E-shaped input (Section 3.2, Table 1: 6x6 blocks, 186,624 water
    molecules, occupancy about 0.05%): one 6x6 block per molecule, centres
    uniform in an open cube at liquid-water density; block (i,j) present iff
    the centres are closer than ``cutoff`` (8.7 A gives 0.05% occupancy at
    this size); values U[-1,1]*exp(-0.5*d); beta = 0; the on-the-fly filter
    at ``eps`` keeps about 1,300 products per block row, so the product has a
    pattern about as sparse as its operands.  Positions come from seed +100,
    values of A and B from seeds +0 and +1."""
    L = box_side(nmol, density)
    pos = np.random.default_rng(seed + 100).uniform(0.0, L, (nmol, 3))
    ii, jj, dd = cutoff_pairs(pos, cutoff)
    rp, ci, dd = _csr_with_block_scalars(nmol, ii, jj, dd)
    del ii, jj
    sizes = np.full(nmol, bs, dtype=np.int32)
    decay = np.exp(-0.5 * dd)
    mats = []
    for off in (0, 1):
        v = np.random.default_rng(seed + off).uniform(-1.0, 1.0, len(ci) * bs * bs)
        v.reshape(len(ci), bs * bs)[:] *= decay[:, None]
        mats.append(with_pattern(sizes, sizes, rp, ci, v))
    A, B = mats
    return Workload(f"semi_empirical{nmol}_b{bs}_cut{cutoff}_eps{eps}", A, B, None, 1.0, 0.0, eps,
                    {"N": int(nmol * bs), "box": L})


def mixed_dense(seed=7000, nb=64, sizes=(9, 22, 32)):
    """H2O-64-shaped input (Section 3.1: block sizes combining 9, 22 and 32,
    fully occupied matrices): nb x nb blocks, every block present, block
    edges cycling through ``sizes``; values U[-1,1]; C = A*B + C_old with a
    fully occupied C_old (seeds +0, +1, +2), no filtering."""
    edges = np.resize(np.asarray(sizes, dtype=np.int32), nb)
    full = np.ones((nb, nb), dtype=bool)
    rp, ci = pattern_from_mask(full)
    mats = []
    for off in (0, 1, 2):
        M = with_pattern(edges, edges, rp, ci)
        M.values = values_uniform(seed + off, M.block_elems())
        mats.append(M)
    A, B, C = mats
    return Workload(f"mixed_dense{nb}_b{'_'.join(map(str, sizes))}", A, B, C, 1.0, 1.0, 0.0,
                    {"N": int(edges.sum())})


def block_stream(seed, m, n, k, nblocks):
    """Independent block products C_i += A_i B_i, i < nblocks, as a
    block-diagonal multiply (the streaming micro-benchmark of Section 2 /
    Figure 1): A has m x k blocks, B k x n, C_old m x n on the diagonal;
    values U[-1,1] (seeds +0, +1, +2); beta = 1, no filtering."""
    rp = np.arange(nblocks + 1, dtype=np.int32)
    ci = np.arange(nblocks, dtype=np.int32)
    rs, ks, cs = (np.full(nblocks, x, dtype=np.int32) for x in (m, k, n))
    A = with_pattern(rs, ks, rp, ci, values_uniform(seed, np.full(nblocks, m * k)))
    B = with_pattern(ks, cs, rp, ci, values_uniform(seed + 1, np.full(nblocks, k * n)))
    C = with_pattern(rs, cs, rp, ci, values_uniform(seed + 2, np.full(nblocks, m * n)))
    return Workload(f"block_stream_m{m}_n{n}_k{k}_x{nblocks}", A, B, C, 1.0, 1.0, 0.0,
                    {"N": int(nblocks * max(m, n, k))})
