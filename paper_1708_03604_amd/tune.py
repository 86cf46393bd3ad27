"""Autotuners of the small-block and generic paths and their table.

The small-block kernel pads every block to one of four shape classes
(8 or 16 rows by 8 or 16 columns); a variant fixes per class the form of the
block product (FP64 vector units or FP64 matrix cores) and how many block
products each wave keeps in flight.  Section 2 of the paper tunes the batched
multiply for each set of block dimensions; here the tuner times every variant
on each class of a real product (bsmm_tune_small) and keeps, per class, the
fastest in a table keyed by the block edges of A's rows, A's columns and B's
columns; the classes then run each with its own variant.

The table is saved as JSON, one entry per edge set:

    {"arch": "gfx950", "entries": [{"rows": [5, 13], "inner": [5, 13],
      "cols": [5, 13], "variants": [6, 6, 6, 7], "depths": [18, 18, 18, 19],
      "ms": [...]}]}

(`depths[c]` is bsmm_small_variant(variants[c])[c].)

The generic path (blocks neither all <= 16 nor all 23x23) has its own
variants (bsmm_tune_mid: 32x32 sub-tiles, or one 16x16 sub-tile for C
blocks with both edges <= 16, and the FP64 vector or matrix-core form), kept
per set of block edges under "mid_entries":

    {"masks": [rows, inner, cols], "rows": [9, 22, 32], ..., "variant": 1,
     "ms": [...]}

(the masks have bit e-1 set for edge e, bit 31 for every edge >= 32; the
edge lists show them, 32 standing for ">= 32").

`load()` enters a saved table into the library; the package loads
tune_gfx950.json next to this file, if present, when the library is first
used.

    python -m paper_1708_03604_amd.tune [--nmol 3000] [--se-nmol 40000] [--reps 5]

tunes the atom-blocked water product (O: 13, H: 5) and a semi-empirical-shaped
product (6x6 blocks) and writes the table.
"""
import argparse
import json
import os

from . import bsmm

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.json")


def key_edges(key):
    """Tuning key -> (row edges, inner edges, column edges)."""
    return tuple([e + 1 for e in range(16) if (key >> (16 * part + e)) & 1] for part in range(3))


def edges_key(rows, inner, cols):
    key = 0
    for part, edges in enumerate((rows, inner, cols)):
        for e in edges:
            if not 1 <= int(e) <= 16:
                raise ValueError(f"block edge {e} outside 1..16")
            key |= 1 << (16 * part + int(e) - 1)
    return key


def tune(alpha, A, B, beta, C_in, C_out, eps, reps=5, stream=None):
    """Tune on one product (Matrix wrappers); C_out receives the product.
    Returns the table entry (None if the small-block path does not serve it)."""
    v, ms = bsmm.bsmm_tune_small(alpha, A.handle, B.handle, beta, C_in.handle if C_in is not None else None,
                                 C_out.handle, eps, reps, stream)
    if v[0] < 0:
        return None
    rows, inner, cols = key_edges(bsmm.bsmm_tune_key(A.handle, B.handle))
    return {"rows": rows, "inner": inner, "cols": cols, "variants": [int(x) for x in v],
            "depths": [bsmm.bsmm_small_variant(x)[c] for c, x in enumerate(v)],
            "ms": [[round(x / reps, 5) for x in r] for r in ms.tolist()]}


def mask_edges(mask):
    """Edge mask of the generic path's key -> edges (32 stands for >= 32)."""
    return [e + 1 for e in range(32) if (int(mask) >> e) & 1]


def tune_mid(alpha, A, B, beta, C_in, C_out, eps, reps=5, stream=None):
    """Tune the generic path on one product (Matrix wrappers); C_out receives
    the product.  Returns the table entry (None if another path serves it)."""
    v, ms = bsmm.bsmm_tune_mid(alpha, A.handle, B.handle, beta, C_in.handle if C_in is not None else None,
                               C_out.handle, eps, reps, stream)
    if v < 0:
        return None
    masks = bsmm.bsmm_mid_key(A.handle, B.handle)
    return {"masks": list(masks), "rows": mask_edges(masks[0]), "inner": mask_edges(masks[1]),
            "cols": mask_edges(masks[2]), "variant": int(v), "ms": [round(x / reps, 5) for x in ms.tolist()]}


def load(path=TABLE):
    """Enter a saved table into the library; returns its small-block entries."""
    with open(path) as f:
        table = json.load(f)
    entries = table.get("entries", [])
    for e in entries:
        bsmm.bsmm_tune_set(edges_key(e["rows"], e["inner"], e["cols"]), [int(x) for x in e["variants"]])
    for e in table.get("mid_entries", []):
        bsmm.bsmm_mid_set([int(x) for x in e["masks"]], int(e["variant"]))
    return entries


def save(entries, path=TABLE, note="", mid_entries=()):
    with open(path, "w") as f:
        json.dump({"arch": "gfx950", "note": note, "entries": entries, "mid_entries": list(mid_entries)}, f,
                  indent=1)
        f.write("\n")


def main():
    import torch
    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--nmol", type=int, default=3000)
    ap.add_argument("--se-nmol", type=int, default=40000)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    entries, names = [], []
    for w in (W.water_atoms(nmol=args.nmol), W.semi_empirical(nmol=args.se_nmol)):
        st = torch.cuda.Stream()
        dA = bsmm.Matrix.from_csr(w.A, st)
        dB = bsmm.Matrix.from_csr(w.B, st)
        dC = bsmm.Matrix.empty(w.A.row_sizes, w.B.col_sizes, st)
        entry = tune(w.alpha, dA, dB, w.beta, None, dC, w.eps, args.reps, st)
        if entry is None:
            raise SystemExit(f"the small-block path does not serve {w.name}")
        print(w.name, json.dumps(entry), flush=True)
        entries.append(entry)
        names.append(w.name)
        for m in (dA, dB, dC):
            m.close()
    mid_entries = []
    for w in (W.mixed_dense(),):
        st = torch.cuda.Stream()
        dA, dB, dCin = (bsmm.Matrix.from_csr(x, st) for x in (w.A, w.B, w.C_old))
        dC = bsmm.Matrix.empty(w.A.row_sizes, w.B.col_sizes, st)
        entry = tune_mid(w.alpha, dA, dB, w.beta, dCin, dC, w.eps, args.reps, st)
        if entry is None:
            raise SystemExit(f"the generic path does not serve {w.name}")
        print(w.name, json.dumps(entry), flush=True)
        mid_entries.append(entry)
        names.append(w.name)
        for m in (dA, dB, dCin, dC):
            m.close()
    save(entries, args.out, note=f"tuned on {', '.join(names)}; {args.reps} launches per variant and class; "
                                 "ms per launch", mid_entries=mid_entries)


if __name__ == "__main__":
    main()
