"""Project autotuner for the BILU kernels on the current GPU.

For each update precision and each workload given, it times the full step
(bilu_factor + bilu_fgmres_solve to 1e-8) under candidate kernel settings
and keeps, per (precision, block-width class, reproducibility requirement),
the settings with the smallest mean time relative to the library's
defaults over the workloads of that class.  The search is coordinate
descent from the defaults over:

  workers_per_cu   0 (as many as fit, two) or 1
  update_mfma      0 (scalar update terms) or 1 (16x16 matrix-core tiles)
  factor_path      0 (LDS staging where it fits) or 2 (global staging)
  apply_path       0 (dataflow, workgroup order), 1 (per level), 2 (ticket)
  deterministic    1, or 0 for the entries of handles that do not require
                   reproducible results (--allow-nondeterministic)

A setting replaces the current one only when it is faster by more than the
noise margin (1%).  The table is written as JSON for bilu_load_tuning.

  python -m paper_1908_10169_amd.tune --workload el3d_80_b3 \\
      --workload cd3d_64_b4 --out paper_1908_10169_amd/tuning/gfx950.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KNOBS = [("workers_per_cu", [0, 1]), ("update_mfma", [0, 1]), ("factor_path", [0, 2]),
         ("apply_path", [0, 1, 2])]
DEFAULTS = dict(workers_per_cu=0, update_mfma=0, factor_path=0, apply_path=0, deterministic=1)
MARGIN = 0.01


def step_time(w, prec, settings, steps, warmup):
    """Seconds per step (factor + FGMRES to 1e-8) under explicit settings."""
    import numpy as np
    import torch

    from paper_1908_10169_amd import bilu
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, update_precision=prec, use_tuning=0, **settings)
    h.analyze(w.a, pre_perm=w.perm)
    b = torch.from_numpy(w.a.matvec(np.ones(w.a.n))).cuda()
    x = torch.zeros_like(b)
    for _ in range(warmup):
        h.factor(w.tau)
        x.zero_()
        h.fgmres(b, x, restart=w.restart, rtol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.factor(w.tau)
        x.zero_()
        info = h.fgmres(b, x, restart=w.restart, rtol=1e-8)
        if not info["converged"]:
            h.close()
            return float("inf"), None
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    st = h.stats()
    assert st["apply_faults"] == 0
    h.close()
    return t, st


def tune_class(ws, prec, reproducible, steps, warmup, log):
    """Coordinate descent over the knobs for the workloads ws of one class."""
    cur = dict(DEFAULTS)
    knobs = list(KNOBS) + ([] if reproducible else [("deterministic", [1, 0])])
    base = {}
    for w in ws:
        base[w.name], _ = step_time(w, prec, cur, steps, warmup)
    log(f"  defaults: " + ", ".join(f"{k} {v * 1e3:.2f} ms" for k, v in base.items()))

    def score(settings):
        tot = 0.0
        for w in ws:
            t, _ = step_time(w, prec, settings, steps, warmup)
            tot += t / base[w.name]
        return tot / len(ws)

    best = 1.0
    for name, values in knobs:
        for v in values:
            if v == cur[name]:
                continue
            cand = dict(cur, **{name: v})
            sc = score(cand)
            log(f"  {name}={v}: {sc:.4f} of the defaults")
            if sc < best * (1.0 - MARGIN):
                best, cur = sc, cand
    return cur, best, base


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--workload", action="append", default=[])
    p.add_argument("--precisions", default="f64,f32,bf16")
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--allow-nondeterministic", action="store_true")
    p.add_argument("--out", default=os.path.join(HERE, "tuning", "gfx950.json"))
    args = p.parse_args()
    import torch

    from paper_1908_10169_amd import bilu, matgen as mg
    torch.cuda.set_device(0)
    log = lambda m: print(m, flush=True)  # noqa: E731
    names = args.workload or ["el3d_80_b3", "cd3d_64_b4"]
    ws = [mg.workload(n) for n in names]
    precs = {"f64": 0, "f32": 1, "bf16": 2}
    entries, notes = [], []
    for pname in [s for s in args.precisions.split(",") if s]:
        prec = precs[pname]
        # block-width class of each workload's initial partition
        classes = {}
        for w in ws:
            _, st = step_time(w, prec, DEFAULTS, 1, 0)
            classes.setdefault(1 if st["max_width_initial"] > 16 else 0, []).append(w)
        for wc, group in sorted(classes.items()):
            for reproducible in ([1, 0] if args.allow_nondeterministic else [1]):
                log(f"[tune] {pname} width class {wc} reproducible={reproducible}: "
                    f"{[w.name for w in group]}")
                best, score, base = tune_class(group, prec, reproducible, args.steps, args.warmup,
                                               log)
                log(f"[tune] chosen {best} ({score:.4f} of the defaults)")
                # entries are flat numeric objects (the library's reader);
                # what they were measured on goes to the notes
                entries.append(dict(precision=prec, width_class=wc, reproducible=reproducible,
                                    **best, relative_time=round(score, 4)))
                notes.append(dict(precision=pname, width_class=wc, reproducible=reproducible,
                                  workloads=[w.name for w in group],
                                  default_ms={k: round(v * 1e3, 3) for k, v in base.items()}))
    out = {"version": 1, "device": torch.cuda.get_device_name(0),
           "measured": time.strftime("%Y-%m-%d"), "steps": args.steps,
           "noise_margin": MARGIN, "entries": entries, "notes": notes}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    log(f"[tune] wrote {len(entries)} entries to {args.out}")
    assert bilu.load_tuning(args.out) == len(entries)


if __name__ == "__main__":
    main()
