"""Autotune the flexibility-product schedules of a workload on the GPU and record them.

    python -m paper_1208_6387_amd.tune --config 3 --forms fp64,bf16x3 [--reps 10]

For every form and every block width the solver uses on the workload (n_rhs * n_perm for the
inner products, n_rhs for the FP64 residual products), problem_tune times every candidate
schedule on the structure itself and installs the fastest; the measured table is merged into
schedules.json next to this file, keyed by the structure's signature (see signature()).
structure.install_schedules() reads it back when a structure is created.
"""
from __future__ import annotations

import argparse
import datetime
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TABLE = os.path.join(HERE, "schedules.json")
FORMS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16": 3}


def signature(n_b, n_occ, m: int, form: str) -> str:
    """Key of a schedule: the form, the block width and each pattern's (n_b, occurrences)."""
    return f"{form}|m={m}|" + ";".join(f"{b}x{q}" for b, q in zip(n_b, n_occ))


def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def main() -> None:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import paper_1208_6387_amd as R
    from paper_1208_6387_amd import structure as ST
    import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, required=True)
    ap.add_argument("--forms", default="fp64,bf16x3")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    R.load()
    p = W.config(args.config)
    pats = ST.factor_patterns(p)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    ST.condense_patterns(pats, tuple(sorted({R.FP64} | {FORMS[f] for f in forms})))
    pb = ST.create_problem(p)
    n_occ = list(np.bincount(p.occ_pattern, minlength=len(p.patterns)))
    n_b = [pat.n_b for pat in p.patterns]
    widths = sorted({p.n_rhs * p.n_perm, p.n_rhs})
    dev = torch.cuda.get_device_name(0)
    table = load_table(args.out)
    for form in forms:
        for m in widths:
            if form != "fp64" and m != p.n_rhs * p.n_perm:
                continue  # the low-precision products only run at the inner width
            print(f"[tune] {p.name} {form} m={m}", flush=True)
            res = R.problem_tune(pb, pats, m, FORMS[form], reps=args.reps)
            best = next(r for r in res if r["chosen"])
            for r in res:
                print(f"[tune]   tile {r['tile']:3d} work {r['work']:5d}: {r['ms']:.4f} ms"
                      f"{'  <- chosen' if r['chosen'] else ''}", flush=True)
            table[signature(n_b, n_occ, m, form)] = {
                "workload": p.name, "tile": best["tile"], "work": best["work"], "reps": args.reps,
                "device": dev, "date": datetime.date.today().isoformat(),
                "measured_ms": [{"tile": r["tile"], "work": r["work"], "ms": round(r["ms"], 5)} for r in res]}
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(f"[tune] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
