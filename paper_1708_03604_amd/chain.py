"""Newton-Schulz sign iteration as a chain of block-sparse multiplies.

Section 1 of the paper motivates the multiply by linear-scaling methods that
call it many times per step (density-matrix and matrix-sign iterations), with
sparsity that changes as the iteration proceeds.  This module runs the
Newton-Schulz iteration for sign(X0),

    T_k     = 3 I - X_k X_k
    X_{k+1} = 1/2 X_k T_k

with the on-the-fly filter in every multiply and a filter of every result at
the same threshold, then the residual ||X X - I||_F (always in FP64; the
iteration's multiplies may run in split precision).  All multiplies write
reserved (device-sized) matrices, so the whole sequence runs without a host
synchronisation and can be captured once in a HIP graph and replayed.

Argument marshalling only: every step is a call into libbsmm.
"""
import numpy as np

from . import bsmm
from .workloads import identity_like


def dense_caps(X0):
    """Capacities that always suffice: every block present."""
    nb = X0.nbrows
    n = int(np.asarray(X0.row_sizes, dtype=np.int64).sum())
    return nb * nb, n * n, nb * nb * nb


class SignChain:
    """Newton-Schulz chain on device.

    X0 (host BlockCSR, square, symmetric, spectral radius < 1) is uploaded
    once and never written, so every run starts from it.  `caps` =
    (max blocks, max values, max products per multiply) of the reserved work
    matrices (default: dense).  `prec` is the precision of the iteration's
    multiplies (bsmm.BSMM_FP64 or bsmm.BSMM_SPLIT_BF16X3); the residual
    multiply is FP64.  `stack_limit` (optional) caps the products one stack
    panel of the work matrices holds (bsmm_set_stack_limit): with the dense
    default capacities the multiplies then build their stacks in panels.
    """

    def __init__(self, X0, steps=12, eps=1e-7, caps=None, stream=None, prec=bsmm.BSMM_FP64, stack_limit=None):
        import torch
        self.steps = steps
        self.eps = eps
        self.prec = prec
        self.stream = stream if stream is not None else torch.cuda.Stream()
        st = self.stream
        nnzb, nvals, nprod = caps if caps is not None else dense_caps(X0)
        self.X0 = bsmm.Matrix.from_csr(X0, st)
        self.I3 = bsmm.Matrix.from_csr(identity_like(X0, 3.0), st)
        self.I1 = bsmm.Matrix.from_csr(identity_like(X0, 1.0), st)
        rs, cs = X0.row_sizes, X0.col_sizes
        self.X = [bsmm.Matrix.empty(rs, cs, st), bsmm.Matrix.empty(rs, cs, st)]
        self.T = bsmm.Matrix.empty(rs, cs, st)
        self.R = bsmm.Matrix.empty(rs, cs, st)
        for m in self.X + [self.T, self.R]:
            if stack_limit is not None:
                bsmm.bsmm_set_stack_limit(m.handle, stack_limit)
            bsmm.bsmm_reserve(m.handle, nnzb, nvals, nprod, st)
        self.residual = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.graph = None
        self.final = None

    def enqueue(self):
        """Enqueue the whole chain on the chain's stream (no host sync)."""
        st = self.stream
        cur = self.X0
        for k in range(self.steps):
            nxt = self.X[k % 2]
            bsmm.multiply(-1.0, cur, cur, 1.0, self.I3, self.T, self.eps, prec=self.prec, stream=st)
            bsmm.bsmm_filter(self.T.handle, self.eps, st)
            bsmm.multiply(0.5, cur, self.T, 0.0, None, nxt, self.eps, prec=self.prec, stream=st)
            bsmm.bsmm_filter(nxt.handle, self.eps, st)
            cur = nxt
        bsmm.multiply(1.0, cur, cur, -1.0, self.I1, self.R, 0.0, stream=st)
        bsmm.bsmm_frobenius(self.R.handle, self.residual, st)
        self.final = cur

    def count_flops(self, progress=None, after_multiply=None):
        """Run the chain eagerly, reading each multiply's counters (one host
        synchronisation per multiply); returns (useful flops of the whole
        chain, kept products, list of result block counts per step).
        progress(step, blocks), if given, is called after every step;
        after_multiply(step, args), if given, after every multiply and before
        its result is filtered, with args = (alpha, A, B, beta, C_in, C,
        filter_eps) as the multiply received them (step = self.steps for the
        residual multiply)."""
        st = self.stream
        cur = self.X0
        flops, prods, blocks = 0.0, 0, []
        for k in range(self.steps):
            nxt = self.X[k % 2]
            for args in ((-1.0, cur, cur, 1.0, self.I3, self.T), (0.5, cur, self.T, 0.0, None, nxt)):
                bsmm.multiply(*args, self.eps, prec=self.prec, stream=st)
                s = bsmm.bsmm_stats(args[5].handle)
                flops += s["useful_flops"]
                prods += s["products"]
                if after_multiply is not None:
                    after_multiply(k, args + (self.eps,))
                bsmm.bsmm_filter(args[5].handle, self.eps, st)
            blocks.append(nxt.info()[2])
            if progress is not None:
                progress(k, blocks[-1])
            cur = nxt
        bsmm.multiply(1.0, cur, cur, -1.0, self.I1, self.R, 0.0, stream=st)
        if after_multiply is not None:
            after_multiply(self.steps, (1.0, cur, cur, -1.0, self.I1, self.R, 0.0))
        s = bsmm.bsmm_stats(self.R.handle)
        flops += s["useful_flops"]
        prods += s["products"]
        bsmm.bsmm_frobenius(self.R.handle, self.residual, st)
        self.final = cur
        st.synchronize()
        return flops, prods, blocks

    def capture(self):
        """Run the chain once eagerly (sizes every scratch buffer), then
        capture it into one HIP graph."""
        self.enqueue()
        self.stream.synchronize()
        bsmm.bsmm_capture_begin(self.stream)
        try:
            self.enqueue()
        finally:
            g = bsmm.bsmm_capture_end(self.stream)
        self.graph = g
        return g

    def replay(self):
        bsmm.bsmm_graph_launch(self.graph, self.stream)

    def multiplies(self):
        return 2 * self.steps + 1

    def close(self):
        if self.graph is not None:
            bsmm.bsmm_graph_destroy(self.graph)
            self.graph = None
        for m in [self.X0, self.I3, self.I1, self.T, self.R] + self.X:
            m.close()
