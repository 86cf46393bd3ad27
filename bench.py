"""Benchmark: useful GFLOP/s of one block-sparse multiply C = alpha*A*B + beta*C
on one MI355X, FP64, on the molecule-blocked workload (2048 water molecules as
23x23 blocks, 6 A cutoff, filter_eps = 1e-6, beta = 1 with C on A's pattern).

    python bench.py [--steps K] [--warmup W]
                    [--workload molecules|grid|water|semi_empirical|mixed_dense|sweep|chain]

A step is one bsmm_multiply (norms, symbolic count, sizing, symbolic fill,
numeric with the alpha/beta epilogue) with inputs resident in HBM.  Prints one
JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "useful GFLOP/s of block-sparse C=A*B (23x23 blocks) FP64 vs split-prec, % roofline"
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (= FP64 matrix) peak
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(w, result_nvals):
    """Bytes the method must move: the FP64 values of A, B, C_in (when read)
    and of the result, each read or written once."""
    n = w.A.nvals + w.B.nvals + result_nvals
    if w.beta != 0 and w.C_old is not None:
        n += w.C_old.nvals
    return 8.0 * n


PROFILE = os.path.join(ROOT, "profiles", "numeric_mfma24_molecules2048.md")
NUMERIC_SRC = os.path.join(ROOT, "paper_1708_03604_amd", "csrc", "kernels_numeric.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def profile_record():
    """The machine-readable record of the committed rocprofv3 summary of the
    numeric kernel (HBM bytes per launch, average kernel duration), or {} if
    the numeric kernel source changed since the profile was taken."""
    import hashlib
    import re
    try:
        text = open(PROFILE).read()
        src = open(NUMERIC_SRC, "rb").read()
    except OSError:
        return {}
    m = re.search(r"^traffic_record: (\{.*\})$", text, re.M)
    if not m:
        return {}
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return {}
    return rec


def roofline_obj(workload, flops, numeric_ms, alg_bytes, path):
    """Roofline of the numeric kernel: `achieved` from the HIP events the
    library records around it on the multiply's stream; the committed
    rocprofv3 summary's average kernel duration gives a second figure (and the
    HBM traffic) while the kernel source is unchanged.  The 23x23 path runs on
    the FP64 matrix cores ("mfma"), the others on the FP64 vector units
    ("alu"); both peaks are 78.6 TFLOP/s."""
    achieved = flops / (numeric_ms * 1e-3) / 1e12
    mfma = path == 1
    out = {"bound": "mfma" if mfma else "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
           "kernel": ("k_numeric_mfma24 (FP64 matrix-core block products + alpha/beta epilogue)" if mfma else
                      "numeric (batched block products + alpha/beta epilogue)"),
           "algorithmic_bytes": alg_bytes, "flop_per_byte": round(flops / alg_bytes, 2)}
    if workload == "molecules":
        rec = profile_record()
        if rec:
            out["traffic"] = rec.get("hbm_bytes_per_launch")
            if rec.get("kernel_avg_us"):
                a2 = flops / (rec["kernel_avg_us"] * 1e-6) / 1e12
                out["achieved_rocprof"] = round(a2, 3)
                out["frac_rocprof"] = round(a2 / FP64_PEAK_TFLOPS, 4)
    return out


def make_workload(name):
    from paper_1708_03604_amd import workloads as W
    if name == "molecules":
        w = W.molecules()
        desc = ("molecules: 2048 water molecules as 23x23 blocks (N=47104), open box at 0.033/A^3, "
                "block iff centres < 6 A, values U[-1,1]*exp(-0.5 d), filter_eps=1e-6, beta=1, "
                "C on A's pattern")
    elif name == "grid":
        w = W.grid23()
        desc = "grid: 64x64 blocks of 23x23 (N=1472), p=0.3, U[-1,1], beta=0, no filter"
    elif name == "water":
        w = W.water_atoms()
        desc = ("water: 3000 molecules as O(13),H(5),H(5) atom blocks (N=69000), 5 A cutoff, "
                "U[-1,1]*exp(-0.5 d), beta=0, no filter")
    elif name == "semi_empirical":
        w = W.semi_empirical()
        desc = ("semi_empirical: 186,624 molecules as 6x6 blocks (N=1,119,744), 8.7 A cutoff (0.05% occupancy), "
                "U[-1,1]*exp(-0.5 d), beta=0, filter_eps=0.07")
    elif name == "mixed_dense":
        w = W.mixed_dense()
        desc = ("mixed_dense: 64x64 blocks with edges cycling 9,22,32 (N=1332), fully occupied, U[-1,1], "
                "beta=1, no filter")
    else:
        raise SystemExit(f"unknown workload {name}")
    return w, desc


SWEEP_EDGES = (4, 5, 6, 8, 9, 12, 13, 16, 20, 22, 23, 24, 26, 32, 40, 45, 48, 55, 64, 78)


def sweep_leg(steps, warmup, working_set=2 << 30):
    """Streaming block products C_i += A_i B_i with m = n = k = s for each
    edge s, the operands of one multiply about `working_set` bytes; returns
    per-edge rates and their geometric mean."""
    import torch
    from paper_1708_03604_amd import bsmm
    from paper_1708_03604_amd import workloads as W
    stream = torch.cuda.current_stream()
    rows = []
    for s in SWEEP_EDGES:
        nblocks = max(1, working_set // (8 * 4 * s * s))
        w = W.block_stream(8000 + s, s, s, s, nblocks)
        dA, dB, dCin = (bsmm.Matrix.from_csr(x, stream) for x in (w.A, w.B, w.C_old))
        dC = bsmm.Matrix.empty(w.A.row_sizes, w.B.col_sizes, stream)
        # the autotuner picks the small-block variant for this edge (untimed)
        variants = bsmm.bsmm_tune_small(1.0, dA.handle, dB.handle, 1.0, dCin.handle, dC.handle, 0.0, 2, stream)[0]
        # and the tile shape and form of the generic path (untimed)
        midv, mid_ms = bsmm.bsmm_tune_mid(1.0, dA.handle, dB.handle, 1.0, dCin.handle, dC.handle, 0.0, 2, stream)
        if midv >= 0:
            variants = [midv]
        for _ in range(warmup):
            bsmm.multiply(1.0, dA, dB, 1.0, dCin, dC, 0.0, stream=stream)
        torch.cuda.synchronize()
        bsmm.bsmm_timing(dC.handle, 1)
        t0 = time.perf_counter()
        for _ in range(steps):
            bsmm.multiply(1.0, dA, dB, 1.0, dCin, dC, 0.0, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        ph, n = bsmm.bsmm_phase_times(dC.handle)
        st = bsmm.bsmm_stats(dC.handle)
        num_ms = ph["numeric"] / max(n, 1)
        flops = st["useful_flops"]
        row = {"edge": s, "blocks": nblocks, "path": PATH_NAMES.get(st["path"], st["path"]), "variants": variants,
               "ms": round(ms, 4), "gflops": round(flops / ms / 1e6, 1),
               "numeric_ms": round(num_ms, 4), "numeric_gflops": round(flops / num_ms / 1e6, 1),
               "numeric_gbs": round(8 * 4 * s * s * nblocks / num_ms / 1e6, 1)}
        log(f"[sweep] {row}")
        rows.append(row)
        for m in (dA, dB, dCin, dC):
            m.close()
        del w
    gm = math.exp(sum(math.log(r["gflops"]) for r in rows) / len(rows))
    return gm, rows


PATH_NAMES = {0: "generic", 1: "tile23", 2: "small", 3: "split23", 4: "slice23"}


def take_rows(M, rows):
    from paper_1708_03604_amd.workloads import BlockCSR
    off = M.block_offsets()
    rp = [0]
    ci, vals = [], []
    for i in rows:
        b0, b1 = M.row_ptr[i], M.row_ptr[i + 1]
        ci.append(M.col_idx[b0:b1])
        vals.append(M.values[off[b0]:off[b1]])
        rp.append(rp[-1] + b1 - b0)
    return BlockCSR(M.row_sizes[rows], M.col_sizes, rp, np.concatenate(ci), np.concatenate(vals))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, gpu_flops_per_step, target_s=12.0):
    """Time the CPU oracle (compiled for this host: gcc -O3 -march=native
    -ffp-contract=off, OpenMP over block rows) on a bounded sample of block
    rows of the same workload, on all the cores this process may use and on
    one core; report useful GFLOP/s."""
    import tempfile
    import oracle
    build_dir = tempfile.mkdtemp(prefix="oracle_native_")
    compile_line = oracle.use_native_build(build_dir)
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS") or ncores)
    threads = oracle.set_threads(threads)
    res = _time_oracle(w, target_s)
    res.update({"cores": threads, "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": ncores,
                "build": compile_line})
    oracle.set_threads(1)
    one = _time_oracle(w, target_s / 2)
    res["one_core"] = {"value": one["value"], "unit": "GFLOP/s", "sample": one["sample"]}
    oracle.set_threads(threads)
    return res


def _time_oracle(w, target_s):
    import oracle
    rng = np.random.default_rng(123)
    order = rng.permutation(w.A.nbrows)
    nrows = min(32, w.A.nbrows)
    spent = 0.0
    while True:
        rows = np.sort(order[:nrows])
        Asub = take_rows(w.A, rows)
        Csub = take_rows(w.C_old, rows) if w.C_old is not None else None
        t0 = time.perf_counter()
        ref = oracle.multiply(w.alpha, Asub, w.B, w.beta, Csub, w.eps)
        dt = time.perf_counter() - t0
        spent += dt
        # useful flops of the sample: 2*m*n*k over its kept products
        a_k = w.A.col_sizes[Asub.col_idx[ref.stack[:, 1]]] if len(ref.stack) else np.zeros(0)
        c_rows = np.repeat(np.arange(len(rows)), np.diff(ref.row_ptr))
        m = Asub.row_sizes[c_rows[ref.stack[:, 0]]] if len(ref.stack) else np.zeros(0)
        n = w.B.col_sizes[ref.col_idx[ref.stack[:, 0]]] if len(ref.stack) else np.zeros(0)
        flops = float(np.sum(2.0 * m * n * a_k))
        if dt >= target_s or nrows >= w.A.nbrows or spent > 3 * target_s:
            break
        nrows = min(w.A.nbrows, max(nrows * 2, int(nrows * target_s / max(dt, 1e-3))))
    runs = [dt]
    if nrows >= w.A.nbrows and dt < target_s / 2:
        # the whole workload is a short sample: repeat it for about target_s
        # and take the median run
        while sum(runs) < target_s and len(runs) < 200:
            t0 = time.perf_counter()
            oracle.multiply(w.alpha, Asub, w.B, w.beta, Csub, w.eps)
            runs.append(time.perf_counter() - t0)
    dt = float(np.median(runs))
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s",
            "sample": f"{len(rows)} of {w.A.nbrows} block rows (random, seed 123), same B and filter; "
                      f"{flops / 1e9:.2f} GFLOP in {dt:.2f} s (median of {len(runs)} runs, "
                      f"{sum(runs):.1f} s of CPU work)",
            "seconds": dt}


def small_class_leg(w, dA, dB, dCin, dC, stream, reps=5):
    """Per shape class (and per (m, n, k) triple) breakdown of the small-block
    path: the tuner times each class alone with every pipeline variant; the
    class's useful flops come from the exported product stack.  Leaves C as
    the plain multiply computes it."""
    from paper_1708_03604_amd import bsmm
    v, ms = bsmm.bsmm_tune_small(w.alpha, dA.handle, dB.handle, w.beta, dCin.handle if dCin is not None else None,
                                 dC.handle, w.eps, reps, stream)
    if v[0] < 0:
        return None
    st = dC.stack(stream)
    rp, ci, _ = dC.to_host(stream)
    crow = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    m = w.A.row_sizes[crow[st[:, 0]]].astype(np.int64)
    n = w.B.col_sizes[ci[st[:, 0]]].astype(np.int64)
    k = w.A.col_sizes[w.A.col_idx[st[:, 1]]].astype(np.int64)
    cls = (m > 8).astype(np.int64) * 2 + (n > 8).astype(np.int64)
    names = ("8x8", "8x16", "16x8", "16x16")
    classes = []
    for c in range(4):
        sel = cls == c
        fl = float(np.sum(2 * m[sel] * n[sel] * k[sel]))
        t = ms[v[c], c] / reps
        triples = {}
        for mm, nn, kk in set(zip(m[sel].tolist(), n[sel].tolist(), k[sel].tolist())):
            s2 = sel & (m == mm) & (n == nn) & (k == kk)
            triples[f"{mm}x{nn}x{kk}"] = {"products": int(s2.sum()), "gflop": round(2 * mm * nn * kk * int(s2.sum()) / 1e9, 4)}
        classes.append({"class": names[c], "products": int(sel.sum()), "gflop": round(fl / 1e9, 4),
                        "ms": round(t, 4), "gflops": round(fl / t / 1e6, 1) if t > 0 else None,
                        "triples": dict(sorted(triples.items()))})
    return {"variants": [int(x) for x in v], "depths": [bsmm.bsmm_small_variant(x)[c] for c, x in enumerate(v)],
            "note": "each class timed alone with its tuned variant (launch of the whole grid over that class's "
                    "list), mean of the tuner's launches; depth 16 + d is the FP64 matrix-core form",
            "classes": classes}


def _time_precision(w, dA, dB, dCin, stream, steps, warmup, prec):
    """Time the multiply in precision `prec` into a fresh C; returns
    (ms per step, numeric-phase ms, stats, values)."""
    from paper_1708_03604_amd import bsmm
    import torch
    dS = bsmm.Matrix.empty(w.A.row_sizes, w.B.col_sizes, stream)

    def step():
        bsmm.multiply(w.alpha, dA, dB, w.beta, dCin, dS, w.eps, prec=prec, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    bsmm.bsmm_timing(dS.handle, 1)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    phases, nrec = bsmm.bsmm_phase_times(dS.handle)
    bsmm.bsmm_timing(dS.handle, 0)
    stats = bsmm.bsmm_stats(dS.handle)
    _, _, got = dS.to_host()
    dS.close()
    return ms, phases["numeric"] / max(nrec, 1), stats, got


def _error_record(got, ref):
    err = got - ref
    return {"rel_frobenius_vs_fp64": float(np.linalg.norm(err) / np.linalg.norm(ref)),
            "max_abs_err": float(np.max(np.abs(err))),
            "max_abs_err_over_max_abs_c": float(np.max(np.abs(err)) / np.max(np.abs(ref)))}


def split_leg(w, dA, dB, dCin, dC, stream, steps, warmup, fp64_ms, fp64_numeric_ms):
    """Same multiply with the operands split into three BF16 terms on matrix
    cores; error against the FP64 result (which matches the oracle within
    1e-12, see the parity tests)."""
    from paper_1708_03604_amd import bsmm
    _, _, ref = dC.to_host()
    ms, numeric, stats, got = _time_precision(w, dA, dB, dCin, stream, steps, warmup, bsmm.BSMM_SPLIT_BF16X3)
    # roofline of the split form: matrix-core peak over the six BF16 term
    # products, against the algorithmic FP64 bytes at the HBM peak
    flops = stats["useful_flops"]
    mfma_eq = BF16_MFMA_PEAK_TFLOPS / 6.0
    ab = algorithmic_bytes(w, stats["nvals"])
    hbm_eq = flops / ab * HBM_PEAK_GBS / 1e3
    peak = min(mfma_eq, hbm_eq)
    achieved = flops / (numeric * 1e-3) / 1e12
    roof = {"bound": "hbm" if hbm_eq < mfma_eq else "mfma", "achieved": round(achieved, 3),
            "peak": round(peak, 2), "unit": "TFLOP/s (FP64-equivalent)", "frac": round(achieved / peak, 4),
            "traffic": None, "peak_note": f"min(2.5 PFLOP/s BF16 / 6 terms = {mfma_eq:.0f}, "
            f"{flops / ab:.1f} flop/B x 8 TB/s = {hbm_eq:.0f})",
            "kernel": "split pre-pass + split numeric kernel (numeric phase)"}
    out = {"value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "roofline": roof,
           "ms_per_step": round(ms, 4), "numeric_ms": round(numeric, 4),
           "speedup_vs_fp64": round(fp64_ms / ms, 3), "numeric_speedup_vs_fp64": round(fp64_numeric_ms / numeric, 3)}
    out.update(_error_record(got, ref))
    out.update({"stated_bound": "per element 2^-15 |alpha| (|A||B|)_ij + FP64 rounding (rigorous); the tests "
                                "also assert relative Frobenius <= 1e-7 and max-abs <= 1e-6 max|C| (dropping any "
                                "one of the six BF16 term products gives >= 2e-6)",
                "equal_accuracy": False,
                "note": "numeric_ms includes splitting A and B into BF16 terms"})
    return out


# INT8 matrix-core work of one exact-slice 23x23 block product: 28 digit
# products, each one 32x32x32 INT8 MFMA (the 23x23x23 product padded)
SLICE_MFMA_OPS_PER_PRODUCT = 28 * 2 * 32 ** 3
INT8_MFMA_PEAK_TOPS = 5000.0


def slice_leg(w, dA, dB, dCin, dC, stream, steps, warmup, fp64_ms, fp64_numeric_ms):
    """Same multiply in exact-slice precision (seven INT8 digits per value,
    the 28 digit products of combined order <= 8 on INT8 matrix cores, exact
    INT32 sums): FP64-level accuracy, timed next to FP64."""
    from paper_1708_03604_amd import bsmm
    _, _, ref = dC.to_host()
    ms, numeric, stats, got = _time_precision(w, dA, dB, dCin, stream, steps, warmup, bsmm.BSMM_SLICE_INT8X7)
    flops = stats["useful_flops"]
    # matrix-core bound in FP64-equivalent flops: the INT8 peak times useful
    # flops per executed INT8 op (2*23^3 per 28 padded 32x32x32 products)
    useful_per_op = 2.0 * 23 ** 3 / SLICE_MFMA_OPS_PER_PRODUCT
    mfma_eq = INT8_MFMA_PEAK_TOPS * useful_per_op
    ab = algorithmic_bytes(w, stats["nvals"])
    hbm_eq = flops / ab * HBM_PEAK_GBS / 1e3
    peak = min(mfma_eq, hbm_eq)
    achieved = flops / (numeric * 1e-3) / 1e12
    int8_tops = stats["products"] * SLICE_MFMA_OPS_PER_PRODUCT / (numeric * 1e-3) / 1e12
    roof = {"bound": "hbm" if hbm_eq < mfma_eq else "mfma", "achieved": round(achieved, 3),
            "peak": round(peak, 2), "unit": "TFLOP/s (FP64-equivalent)", "frac": round(achieved / peak, 4),
            "traffic": None, "peak_note": f"min(5.0 POP/s INT8 x {useful_per_op:.4f} useful flop per INT8 op = "
            f"{mfma_eq:.1f}, {flops / ab:.1f} flop/B x 8 TB/s = {hbm_eq:.0f})",
            "int8_tops_executed": round(int8_tops, 1),
            "kernel": "slice pre-pass + slice numeric kernel (numeric phase)"}
    out = {"value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "roofline": roof,
           "ms_per_step": round(ms, 4), "numeric_ms": round(numeric, 4),
           "speedup_vs_fp64": round(fp64_ms / ms, 3), "numeric_speedup_vs_fp64": round(fp64_numeric_ms / numeric, 3)}
    out.update(_error_record(got, ref))
    out.update({"stated_bound": "per element 2^-39 |alpha| n_ij MA(i,r) MB(j,q) + FP64 rounding (rigorous); the "
                                "tests assert relative Frobenius <= 1e-13 and bit equality with the CPU model of "
                                "the scheme",
                "equal_accuracy": True,
                "note": "numeric_ms includes the exponent and digit pre-passes over A and B"})
    return out


def chain_leg(nmol, steps=12, eps=1e-7, replays=3, prec=None):
    """Newton-Schulz sign chain (12 steps, filter 1e-7) on a symmetric,
    Gershgorin-scaled molecule matrix, captured in one HIP graph; returns the
    graph replay throughput and the FP64 residual, and the open chain (its
    final X stays on the device for comparison)."""
    from paper_1708_03604_amd import bsmm
    from paper_1708_03604_amd import workloads as W
    from paper_1708_03604_amd.chain import SignChain
    prec = bsmm.BSMM_FP64 if prec is None else prec
    X0, info = W.symmetric_scaled(nmol=nmol)
    ch = SignChain(X0, steps=steps, eps=eps, prec=prec)
    t0 = time.perf_counter()
    flops, prods, blocks = ch.count_flops(
        progress=lambda k, nb: log(f"[bench] counting run: step {k + 1} done, X has {nb} blocks, "
                                   f"{time.perf_counter() - t0:.1f} s"))
    # the same chain enqueued call by call (no graph), for comparison
    t0 = time.perf_counter()
    ch.enqueue()
    ch.stream.synchronize()
    dt_eager = time.perf_counter() - t0
    log(f"[bench] eager chain: {dt_eager:.2f} s")
    ch.capture()
    ch.stream.synchronize()
    log("[bench] chain captured")
    t0 = time.perf_counter()
    for r in range(replays):
        ch.replay()
        if replays > 1:
            ch.stream.synchronize()
            log(f"[bench] replay {r + 1} done")
    ch.stream.synchronize()
    dt = (time.perf_counter() - t0) / replays
    res = float(ch.residual.cpu()[0])
    n = int(info["N"])
    out = {"workload": f"sign chain: {nmol} molecules as 23x23 blocks (N={n}), {steps} Newton-Schulz steps, "
                       f"filter_eps={eps}, {ch.multiplies()} multiplies + {2 * steps} filters + residual, "
                       f"one HIP graph",
           "value": round(flops / dt / 1e9, 2), "unit": "GFLOP/s", "ms_per_chain": round(dt * 1e3, 3),
           "useful_gflop_per_chain": round(flops / 1e9, 3), "products_per_chain": int(prods),
           "x_blocks_per_step": blocks, "residual_fro": res,
           "residual_rel": res / math.sqrt(n), "replays": replays, "ms_per_chain_eager": round(dt_eager * 1e3, 3)}
    return out, ch


def chain_difference(ch_split, ch_fp64):
    """||X_split - X_fp64||_F / ||X_fp64||_F of the two chains' final X, on the
    device: D = 1 * X_split * I - 1 * X_fp64 (an FP64 multiply by the identity)."""
    import torch
    from paper_1708_03604_amd import bsmm
    ch_split.stream.synchronize()
    ch_fp64.stream.synchronize()
    xs, xf = ch_split.final, ch_fp64.final
    D = bsmm.Matrix.empty(xs.row_sizes, xs.col_sizes)
    bsmm.multiply(1.0, xs, ch_split.I1, -1.0, xf, D, 0.0)
    t = torch.zeros(2, dtype=torch.float64, device="cuda")
    bsmm.bsmm_frobenius(D.handle, t[0:1], None)
    bsmm.bsmm_frobenius(xf.handle, t[1:2], None)
    torch.cuda.synchronize()
    d, ref = (float(x) for x in t.cpu())
    D.close()
    return d / ref if ref > 0 else d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="molecules")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chain-nmol", type=int, default=512,
                    help="molecules of the sign chain (--workload chain)")
    ap.add_argument("--chain-replays", type=int, default=3)
    ap.add_argument("--chain-no-split", action="store_true",
                    help="skip the split-precision chain (--workload chain)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB device to device three times (calibrates the HBM traffic counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = 256 << 20
        a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_launch": n}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1708_03604_amd import bsmm

    assert torch.cuda.is_available(), "needs a GPU"
    if args.workload == "chain":
        torch.cuda.set_device(0)
        log(f"[bench] sign chain on {args.chain_nmol} molecules")
        ch, chain_f = chain_leg(args.chain_nmol, replays=args.chain_replays)
        out = {"metric": "useful GFLOP/s of the Newton-Schulz sign chain (block-sparse 23x23 FP64 multiplies, "
                         "one HIP graph)",
               "value": ch.pop("value"), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.chain_replays, "warmup": 1,
               "ms_per_step": ch["ms_per_chain"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic", "config": {"workload": ch.pop("workload")}, "chain": ch}
        log(f"[bench] chain: {ch['ms_per_chain']} ms, {out['value']} GFLOP/s, residual {ch['residual_fro']:.3e}")
        if args.chain_no_split:
            chain_f.close()
            print(json.dumps(out), flush=True)
            return
        log("[bench] the same chain with split-precision iteration multiplies (residual in FP64)")
        sp, chain_s = chain_leg(args.chain_nmol, replays=args.chain_replays, prec=bsmm.BSMM_SPLIT_BF16X3)
        sp.pop("workload")
        sp["speedup_vs_fp64"] = round(ch["ms_per_chain"] / sp["ms_per_chain"], 3)
        sp["x_rel_fro_diff_vs_fp64"] = chain_difference(chain_s, chain_f)
        out["chain_split_bf16x3"] = sp
        log(f"[bench] split chain: {sp['ms_per_chain']} ms ({sp['speedup_vs_fp64']}x), residual "
            f"{sp['residual_fro']:.3e}, final X differs from the FP64 chain's by {sp['x_rel_fro_diff_vs_fp64']:.2e}")
        chain_s.close()
        chain_f.close()
        print(json.dumps(out), flush=True)
        return
    if args.workload == "sweep":
        torch.cuda.set_device(0)
        gm, rows = sweep_leg(args.steps, args.warmup)
        out = {"metric": "geometric mean of useful GFLOP/s of streaming block products C_i += A_i B_i "
                         "(m=n=k=s), FP64",
               "value": round(gm, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": round(sum(r["ms"] for r in rows), 4),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic",
               "config": {"workload": f"block_stream sweep, s in {list(SWEEP_EDGES)}, 2 GiB of operands per s"},
               "sweep": rows}
        print(json.dumps(out), flush=True)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] building workload {args.workload}")
    t0 = time.time()
    w, desc = make_workload(args.workload)
    log(f"[bench] workload ready in {time.time() - t0:.1f} s: A {w.A.nnzb} blocks, B {w.B.nnzb} blocks")
    stream = torch.cuda.current_stream()
    dA = bsmm.Matrix.from_csr(w.A, stream)
    dB = bsmm.Matrix.from_csr(w.B, stream)
    dCin = bsmm.Matrix.from_csr(w.C_old, stream) if w.C_old is not None else None
    dC = bsmm.Matrix.empty(w.A.row_sizes, w.B.col_sizes, stream)
    torch.cuda.synchronize()

    def step():
        bsmm.multiply(w.alpha, dA, dB, w.beta, dCin, dC, w.eps, stream=stream)

    mid_tune = None
    if args.workload == "mixed_dense":
        # the autotuner picks the generic path's tile shape and form for these
        # block edges before the timed steps (the tuning is not timed)
        midv, mid_ms = bsmm.bsmm_tune_mid(w.alpha, dA.handle, dB.handle, w.beta,
                                          dCin.handle if dCin is not None else None, dC.handle, w.eps, 5, stream)
        if midv >= 0:
            mid_tune = {"variant": midv, "t16": bool(midv & 1), "matrix_cores": bool(midv & 2),
                        "cin_prefetch": bool(midv & 4),
                        "ms_per_launch": [round(x / 5, 5) for x in mid_ms.tolist()],
                        "note": "variant bit 0: one 16x16 sub-tile for C blocks with both edges <= 16; bit 1: FP64 "
                                "matrix-core form (0 ms: not allowed for these inner edges); bit 2: C_in loaded before "
                                "each sub-tile's last chunk"}
            log(f"[bench] generic path tuned: {mid_tune}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    bsmm.bsmm_timing(dC.handle, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phases, nrec = bsmm.bsmm_phase_times(dC.handle)
    bsmm.bsmm_timing(dC.handle, 0)
    stats = bsmm.bsmm_stats(dC.handle)
    ms_per_step = elapsed * 1e3 / args.steps
    flops = stats["useful_flops"]
    value = flops / (ms_per_step * 1e-3) / 1e9
    phase_avg = {k: v / max(nrec, 1) for k, v in phases.items()}
    numeric_ms = phase_avg["numeric"]
    achieved = flops / (numeric_ms * 1e-3) / 1e12
    log(f"[bench] {ms_per_step:.3f} ms/step, {value:.1f} GFLOP/s; numeric kernel {numeric_ms:.3f} ms "
        f"({achieved:.2f} TFLOP/s)")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "prec": "fp64", "products": stats["products"],
                   "result_blocks": stats["nnzb"], "useful_gflop_per_step": round(flops / 1e9, 4),
                   "kernel_path": PATH_NAMES.get(stats["path"], stats["path"])},
        "roofline": roofline_obj(args.workload, flops, numeric_ms, algorithmic_bytes(w, stats["nvals"]), stats["path"]),
        "whole_step_frac_of_fp64_peak": round(value / 1e3 / FP64_PEAK_TFLOPS, 4),
        "phases_ms": {k: round(v, 4) for k, v in phase_avg.items()},
    }
    if args.workload == "molecules":
        log("[bench] split precision (three BF16 terms on matrix cores)")
        out["split_bf16x3"] = split_leg(w, dA, dB, dCin, dC, stream, args.steps, args.warmup, ms_per_step,
                                        numeric_ms)
        sp = out["split_bf16x3"]
        log(f"[bench] split: {sp['ms_per_step']} ms/step ({sp['speedup_vs_fp64']}x), rel Frobenius error "
            f"{sp['rel_frobenius_vs_fp64']:.2e}")
        log("[bench] exact-slice precision (seven INT8 digits on matrix cores)")
        out["slice_int8x7"] = slice_leg(w, dA, dB, dCin, dC, stream, args.steps, args.warmup, ms_per_step,
                                        numeric_ms)
        sl = out["slice_int8x7"]
        log(f"[bench] slice: {sl['ms_per_step']} ms/step ({sl['speedup_vs_fp64']}x), rel Frobenius error "
            f"{sl['rel_frobenius_vs_fp64']:.2e}")
    if mid_tune is not None:
        out["mid_tune"] = mid_tune
    if args.workload == "water":
        log("[bench] per shape class timing of the small-block kernel")
        out["small_classes"] = small_class_leg(w, dA, dB, dCin, dC, stream)
        for c in out["small_classes"]["classes"]:
            log(f"[bench]   class {c['class']}: {c['products']} products, {c['ms']} ms, {c['gflops']} GFLOP/s")
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(w, flops)
    for m in (dA, dB, dCin, dC):
        if m is not None:
            m.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
