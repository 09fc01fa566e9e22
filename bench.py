"""Benchmark: BILU factor + FGMRES(1e-8) wall time on one MI355X.

One step = bilu_factor(tau) (ILU(1,tau) block guess, GPU block Crout sweep
with dropping, perturbation and aggregation, apply plan) followed by
bilu_fgmres_solve to a relative residual of 1e-8 with b = A * ones, x0 = 0.
The matrix is analyzed (cosine blocking, ordering, upload) once before the
timed region, so every input is resident in HBM when timing starts.

Prints one JSON line.  Extra fields: the roofline of the dominant kernel
(device time from HIP events on the library's stream), the Schur-update
rate, and the FP64 CPU oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="cd3d_64_b4")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--ordering", choices=["caller", "project"], default="caller",
                   help="caller: the workload's geometric nested dissection as pre_perm, groups "
                        "in that order; project: the library's nested dissection of the "
                        "compressed graph (no cpu_baseline)")
    p.add_argument("--aggregation", type=int, default=-1,
                   help="1/0 forces progressive aggregation on/off (default: library default)")
    p.add_argument("--update-precision", choices=["f64", "f32", "bf16"], default="f64",
                   help="arithmetic of the Schur-complement updates (pivots, drop test and "
                        "FGMRES are FP64 in every form)")
    p.add_argument("--apply-path", type=int, default=0, choices=[0, 1, 2],
                   help="0: dataflow apply, slots in dispatch order; 1: one launch per level; "
                        "2: dataflow apply, slots by ticket")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                   help="only copy BYTES between two device buffers twice (reference for the "
                        "HBM byte counters of a profiler) and exit")
    return p.parse_args()


def calibrate_copy(nbytes):
    """A plain device-to-device copy of known size, for scaling FETCH_SIZE /
    WRITE_SIZE counters: each copy reads and writes nbytes once."""
    import torch
    torch.cuda.set_device(0)
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes // 8 * 8, "copies": 2}), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: "
              f"sharding one factorization over several GPUs is not built.", flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1908_10169_amd import bilu, matgen as mg

    torch.cuda.set_device(0)
    w = mg.workload(args.workload)
    a = w.a
    prec = {"f64": bilu.PREC_F64, "f32": bilu.PREC_F32, "bf16": bilu.PREC_BF16}[args.update_precision]
    project = args.ordering == "project"
    opts = dict(ordering=bilu.ORDER_ND if project else bilu.ORDER_NATURAL, collect_timing=1,
                update_precision=prec, apply_path=args.apply_path)
    agg = AGGREGATION_DEFAULT if args.aggregation < 0 else bool(args.aggregation)
    opts["use_aggregation"] = agg
    h = bilu.Bilu(**opts)
    t0 = time.perf_counter()
    h.analyze(a, pre_perm=None if project else w.perm)
    t_analyze = time.perf_counter() - t0
    b_host = a.matvec(np.ones(a.n))
    b = torch.from_numpy(b_host).cuda()
    x = torch.zeros_like(b)
    restart, rtol = w.restart, 1e-8

    def step():
        h.factor(w.tau)
        x.zero_()
        return h.fgmres(b, x, restart=restart, rtol=rtol, maxit=2000)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dev = dict(factor_ms=0.0, apply_ms=0.0, spmv_ms=0.0, n_apply=0, n_spmv=0,
               factor_launches=0)
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(step())
        st = h.stats()   # resolves this step's events (the solve has synchronized)
        dev["factor_ms"] += st["dev_ms_factor"]
        dev["apply_ms"] += st["dev_ms_apply"]
        dev["spmv_ms"] += st["dev_ms_spmv"]
        dev["n_apply"] += st["n_apply"]
        dev["n_spmv"] += st["n_spmv"]
        dev["factor_launches"] += st["n_factor_launches"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sec_per_step = elapsed / args.steps
    st = h.stats()
    info = infos[-1]
    res = np.linalg.norm(b_host - a.matvec(x.cpu().numpy())) / np.linalg.norm(b_host)

    # roofline of the dominant kernel: algorithmic bytes / device time
    fac_bytes = st["bytes_factor"] * args.steps
    app_bytes = st["bytes_apply"] * dev["n_apply"]
    kernels = {
        "factor": dict(ms=dev["factor_ms"], bytes=fac_bytes, launches=dev["factor_launches"]),
        "apply": dict(ms=dev["apply_ms"], bytes=app_bytes, launches=dev["n_apply"]),
    }
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    achieved = kd["bytes"] / (kd["ms"] * 1e-3) / 1e9 if kd["ms"] > 0 else 0.0
    roofline = {"kernel": {"factor": "factor_worker_kernel",
                           "apply": "forward_level+backward_level"}[dom],
                "bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                "traffic": measured_traffic(roofline_kernel_name(dom), w.name)}
    other = "apply" if dom == "factor" else "factor"
    ko = kernels[other]
    other_gbs = ko["bytes"] / (ko["ms"] * 1e-3) / 1e9 if ko["ms"] > 0 else 0.0
    upd_tflops = (st["flops_update"] * args.steps) / (dev["factor_ms"] * 1e-3) / 1e12 \
        if dev["factor_ms"] > 0 else 0.0
    # FP32 vector peak for the FP32-accumulated forms (the products are FMAs)
    upd_peak = FP64_PEAK_TFLOPS if args.update_precision == "f64" else FP32_PEAK_TFLOPS

    # bilu_refactor with the same values, outside the timed region (its
    # statistics are not read after this point)
    vd = torch.from_numpy(a.val).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.refactor(w.tau, vd)
    t_refactor = time.perf_counter() - t0

    out = {
        "metric": "BILU factor+FGMRES(1e-8) time",
        "value": round(sec_per_step, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_per_step * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.update_precision == "f64" else f"f64 ({args.update_precision} updates)",
        "data": "synthetic",
        "config": {
            "workload": w.name, "n": a.n, "nnz": a.nnz, "tau": w.tau, "restart": restart,
            "rtol": rtol,
            "ordering": "nested dissection of the compressed graph (library)" if project
            else "geometric nested dissection (caller permutation)",
            "update_precision": args.update_precision, "aggregation": agg,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "other_kernel": {"kernel": other, "achieved_gbs": round(other_gbs, 3),
                         "frac": round(other_gbs / HBM_PEAK_GBS, 6),
                         "device_ms_per_step": round(ko["ms"] / args.steps, 3)},
        "schur_update": {"tflops": round(upd_tflops, 6), "peak": upd_peak,
                         "frac": round(upd_tflops / upd_peak, 8)},
        "phases_s": {"analyze": round(t_analyze, 4), "refactor": round(t_refactor, 4),
                     "ilu1t": round(st["t_ilu1t"], 4),
                     "factor": round(st["t_factor"], 4),
                     "factor_host_phases": dict(zip(
                         ["ilu1t_sets", "ilu1t_growth", "launch_prep", "factor_kernel",
                          "aggregation", "apply_plan", "statistics"],
                         [round(x, 4) for x in st["t_phase"][:7]])),
                     "factor_device_ms": round(dev["factor_ms"] / args.steps, 3),
                     "solve": round(info["seconds"], 4),
                     "apply_device_ms_each": round(dev["apply_ms"] / max(1, dev["n_apply"]), 4)},
        "solve": {"iterations": info["iterations"], "rel_residual": res,
                  "converged": info["converged"]},
        "factor": {"nblocks": st["nblocks"], "nblocks_initial": st["nblocks_initial"],
                   "max_width": st["max_width"], "avg_width": round(st["avg_width"], 3),
                   "fill": round((st["nnz_l"] + st["nnz_w"] + st["nnz_d"]) / a.nnz, 4),
                   "dependency_depth": st["factor_levels"],
                   "apply_levels": [st["apply_levels_fwd"], st["apply_levels_bwd"]]},
    }
    if not args.no_cpu_baseline and not project:
        out["cpu_baseline"] = cpu_baseline(w, agg, restart, rtol)
    print(json.dumps(out), flush=True)


def roofline_kernel_name(dom):
    return {"factor": "factor_worker_kernel", "apply": "forward_level+backward_level"}[dom]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE profile
    of this kernel and workload (scaled by a plain copy), or None when there
    is none or the kernel's sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_{kernel}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("{"):
            rec = json.loads(line)
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return rec["traffic_bytes"] if h.hexdigest() == rec["sources_sha256"] else None


def cpu_baseline(w, agg, restart, rtol):
    """The FP64 oracle on the host: ILU(1,tau) + sequential sweep + FGMRES."""
    import numpy as np

    from oracle import Oracle, OracleOptions
    o = Oracle()
    o.run(w.a, OracleOptions(tau=w.tau, use_aggregation=agg), pre_perm=w.perm)
    t = o.times()
    b = w.a.matvec(np.ones(w.a.n))
    t0 = time.perf_counter()
    _, info = o.fgmres(b, restart=restart, rtol=rtol)
    t_solve = time.perf_counter() - t0
    total = t["ilu1t"] + t["factor"] + t_solve
    return {"value": round(total, 4), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"the full {w.name} workload (ILU(1,tau) + block Crout sweep + "
                      f"FGMRES, {info['iterations']} iterations), one thread",
            "phases_s": {"ilu1t": round(t["ilu1t"], 4), "factor": round(t["factor"], 4),
                         "solve": round(t_solve, 4)}}


AGGREGATION_DEFAULT = True  # the full method: cosine + ILU(1,tau) blocking + progressive aggregation

if __name__ == "__main__":
    main()
