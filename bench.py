"""Benchmark: BILU factor + FGMRES(1e-8) wall time on one MI355X.

One step = bilu_factor(tau) (ILU(1,tau) block guess, GPU block Crout sweep
with dropping, perturbation and aggregation, apply plan) followed by
bilu_fgmres_solve to a relative residual of 1e-8 with b = A * ones, x0 = 0.
The matrix is analyzed (cosine blocking, ordering, upload) once before the
timed region, so every input is resident in HBM when timing starts.

The main workload is the 80^3 x 3 elasticity operator (n = 1,536,000,
121M nonzeros, tau = 5e-3, FGMRES(30)), timed in the plain FP64 form (the
line's value) and, on the same GPU with the same K steps, in the mixed
forms (FP32 and BF16 Schur updates with L and W stored in that precision;
pivot blocks, drop test and FGMRES in FP64).  Each form reports its factor
and solve times, iterations, the true final residual and the kept-pattern
residual ||(L S U - A)_Omega||/||A||, and the mixed/FP64 time ratio.  The
form f64_atomic is FP64 with the Schur terms subtracted by atomic adds
(deterministic = 0): faster, but the summation order, and so the last bits,
vary from run to run; the line's value stays the reproducible FP64 form.
The 64^3 x 4 convection-diffusion workload in FP64 is a second figure, and
the symmetric variant (symmetric matching, SQMR) on a saddle-point matrix a
third.

Prints one JSON line.  Extra fields: the roofline of the dominant kernel
(device time from HIP events on the library's stream), the Schur-update
rate, and the FP64 CPU oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector
AGGREGATION_DEFAULT = True  # the full method: cosine + ILU(1,tau) blocking + progressive aggregation
FORM_PREC = {"f64": 0, "f32": 1, "bf16": 2, "f64_atomic": 0}
FORM_DET = {"f64_atomic": 0}   # forms that override --deterministic


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="el3d_80_b3")
    p.add_argument("--forms", default="f64,f32,bf16,f64_atomic",
                   help="comma-separated update precisions; the first is the line's value")
    p.add_argument("--second-workload", default="cd3d_64_b4",
                   help="a second workload timed in FP64 ('none' to skip)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--symmetric-workload", default="kkt_32",
                   help="the symmetric variant (Sec. 5) on a saddle-point matrix kkt_<side> "
                        "(elasticity side^3 plus side^3/2 constraints): symmetric matching, "
                        "factor and SQMR to a backward error of 1e-6; 'none' skips it")
    p.add_argument("--ordering", choices=["caller", "project", "multilevel"], default="caller",
                   help="caller: the workload's geometric nested dissection as pre_perm, groups "
                        "in that order; project: the library's nested dissection of the "
                        "compressed graph by level structures; multilevel: its multilevel "
                        "nested dissection (both without cpu_baseline)")
    p.add_argument("--aggregation", type=int, default=-1,
                   help="1/0 forces progressive aggregation on/off (default: library default)")
    p.add_argument("--apply-path", type=int, default=0, choices=[0, 1, 2],
                   help="0: dataflow apply, slots in dispatch order; 1: one launch per level; "
                        "2: dataflow apply, slots by ticket")
    p.add_argument("--update-mfma", type=int, default=0, choices=[0, 1],
                   help="1: Schur-update terms as matrix-core tiles; 0: scalar FMAs")
    p.add_argument("--deterministic", type=int, default=1, choices=[0, 1],
                   help="1: update terms subtracted in a fixed order (bit-identical runs); "
                        "0: with atomic adds")
    p.add_argument("--tuning", default="",
                   help="load this tuning table (paper_1908_10169_amd/tune.py) before timing; "
                        "handles use its entries for their precision and width class")
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


def time_form(w, prec, args, project, agg, det=None):
    """K timed steps of one form on workload w; returns its record."""
    import numpy as np
    import torch

    from paper_1908_10169_amd import bilu
    order = {"caller": bilu.ORDER_NATURAL, "project": bilu.ORDER_ND,
             "multilevel": bilu.ORDER_ND_MULTILEVEL}[args.ordering]
    opts = dict(ordering=order, collect_timing=1,
                update_precision=prec, apply_path=args.apply_path,
                update_mfma=args.update_mfma, use_aggregation=agg,
                deterministic=args.deterministic if det is None else det)
    h = bilu.Bilu(**opts)
    t0 = time.perf_counter()
    h.analyze(w.a, pre_perm=None if project else w.perm)
    t_analyze = time.perf_counter() - t0
    b_host = w.a.matvec(np.ones(w.a.n))
    b = torch.from_numpy(b_host).cuda()
    x = torch.zeros_like(b)
    restart, rtol = w.restart, 1e-8
    phase = dict(factor=0.0, solve=0.0)

    def step():
        t1 = time.perf_counter()
        h.factor(w.tau)
        t2 = time.perf_counter()
        x.zero_()
        info = h.fgmres(b, x, restart=restart, rtol=rtol, maxit=2000)
        t3 = time.perf_counter()
        return info, t2 - t1, t3 - t2

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dev = dict(factor_ms=0.0, apply_ms=0.0, spmv_ms=0.0, n_apply=0, n_spmv=0, factor_launches=0)
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, tf, ts = step()
        infos.append(info)
        phase["factor"] += tf
        phase["solve"] += ts
        st = h.stats()   # resolves this step's events (the solve has synchronized)
        dev["factor_ms"] += st["dev_ms_factor"]
        dev["apply_ms"] += st["dev_ms_apply"]
        dev["spmv_ms"] += st["dev_ms_spmv"]
        dev["n_apply"] += st["n_apply"]
        dev["n_spmv"] += st["n_spmv"]
        dev["factor_launches"] += st["n_factor_launches"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = h.stats()
    assert st["apply_faults"] == 0, "a dataflow apply timed out"
    assert st["ilu1t_host"] == 0, "the ILU(1,tau) partition was computed on the host"
    info = infos[-1]
    res = float(np.linalg.norm(b_host - w.a.matvec(x.cpu().numpy())) / np.linalg.norm(b_host))
    r_kept = h.kept_residual()   # outside the timed region
    h.close()
    return dict(sec_per_step=elapsed / args.steps, t_analyze=t_analyze, stats=st, dev=dev,
                info=info, residual=res, r_kept=r_kept,
                factor_s=phase["factor"] / args.steps, solve_s=phase["solve"] / args.steps)


def time_symmetric(name, args, agg):
    """K timed steps of the symmetric variant: the factor of the saddle-point
    matrix kkt_<side> under the symmetric matching (use_mwm = 2, the
    library's multilevel nested dissection of the compressed graph) and
    SQMR to the paper's backward error of 1e-6 (Sec. 5)."""
    import numpy as np
    import torch

    from paper_1908_10169_amd import bilu, matgen as mg
    side = int(name.split("_")[1])
    a, order, ncon = mg.kkt_elasticity(side)
    tau, tol = 1e-2, 1e-6
    h = bilu.Bilu(ordering=bilu.ORDER_ND_MULTILEVEL, use_mwm=2, use_aggregation=agg,
                  deterministic=args.deterministic)
    t0 = time.perf_counter()
    h.analyze(a, pre_perm=order)
    t_analyze = time.perf_counter() - t0
    b_host = a.matvec(np.ones(a.n))
    b = torch.from_numpy(b_host).cuda()
    x = torch.zeros_like(b)
    phase = dict(factor=0.0, solve=0.0)

    def step():
        t1 = time.perf_counter()
        h.factor(tau)
        t2 = time.perf_counter()
        x.zero_()
        info = h.sqmr(b, x, tol=tol, maxit=2000)
        return info, t2 - t1, time.perf_counter() - t2

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, tf, ts = step()
        phase["factor"] += tf
        phase["solve"] += ts
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = h.stats()
    assert st["apply_faults"] == 0, "a dataflow apply timed out"
    xs = x.cpu().numpy()
    r = b_host - a.matvec(xs)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    anorm = np.bincount(rows, weights=np.abs(a.val), minlength=a.n).max()
    eta = float(np.abs(r).max() / (anorm * np.abs(xs).max() + np.abs(b_host).max()))
    h.close()
    return {"workload": name, "matrix": f"[[K, B^T], [B, 0]]: unperturbed elasticity {side}^3 "
                                        f"plus {ncon} two-node constraints, empty diagonal block",
            "n": a.n, "nnz": a.nnz, "tau": tau, "solver": "SQMR, backward error 1e-6",
            "ordering": "symmetric matching, multilevel nested dissection (library)",
            "dtype": "f64", "ms_per_step": round(elapsed / args.steps * 1e3, 3),
            "factor_ms": round(phase["factor"] / args.steps * 1e3, 3),
            "solve_ms": round(phase["solve"] / args.steps * 1e3, 3),
            "iterations": info["iterations"], "eta": eta, "converged": info["converged"],
            "perturbed_blocks": st["perturbed_blocks"], "nblocks": st["nblocks"],
            "analyze_s": round(t_analyze, 4)}


def roofline_of(rec, w, steps):
    """Roofline of the dominant kernel: algorithmic bytes / device time."""
    st, dev = rec["stats"], rec["dev"]
    kernels = {
        "factor": dict(ms=dev["factor_ms"], bytes=st["bytes_factor"] * steps),
        "apply": dict(ms=dev["apply_ms"], bytes=st["bytes_apply"] * dev["n_apply"]),
    }
    name = {"factor": "factor_worker_kernel", "apply": "apply_flow"}
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    achieved = kd["bytes"] / (kd["ms"] * 1e-3) / 1e9 if kd["ms"] > 0 else 0.0
    roof = {"kernel": name[dom], "bound": "hbm", "achieved": round(achieved, 3),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
            "traffic": measured_traffic(name[dom], w.name)}
    other = "apply" if dom == "factor" else "factor"
    ko = kernels[other]
    other_gbs = ko["bytes"] / (ko["ms"] * 1e-3) / 1e9 if ko["ms"] > 0 else 0.0
    return roof, {"kernel": name[other], "achieved_gbs": round(other_gbs, 3),
                  "frac": round(other_gbs / HBM_PEAK_GBS, 6),
                  "device_ms_per_step": round(ko["ms"] / steps, 3)}


def form_summary(rec, steps, prec):
    st, dev, info = rec["stats"], rec["dev"], rec["info"]
    upd_tflops = (st["flops_update"] * steps) / (dev["factor_ms"] * 1e-3) / 1e12 \
        if dev["factor_ms"] > 0 else 0.0
    # FP32 vector peak for the FP32-accumulated forms (the products are FMAs)
    upd_peak = FP64_PEAK_TFLOPS if prec == 0 else FP32_PEAK_TFLOPS
    return {
        "ms_per_step": round(rec["sec_per_step"] * 1e3, 3),
        "factor_ms": round(rec["factor_s"] * 1e3, 3),
        "solve_ms": round(rec["solve_s"] * 1e3, 3),
        "factor_kernel_device_ms": round(dev["factor_ms"] / steps, 3),
        "apply_device_ms_each": round(dev["apply_ms"] / max(1, dev["n_apply"]), 4),
        "iterations": info["iterations"],
        "rel_residual": rec["residual"],
        "converged": info["converged"],
        "r_kept": rec["r_kept"],
        "schur_update": {"tflops": round(upd_tflops, 6), "peak": upd_peak,
                         "frac": round(upd_tflops / upd_peak, 8)},
        "apply_faults": st["apply_faults"],
        "ilu1t_host": st["ilu1t_host"],
    }


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: "
              f"sharding one factorization over several GPUs is not built.", flush=True)
        sys.exit(2)
    import torch

    from paper_1908_10169_amd import bilu, matgen as mg
    torch.cuda.set_device(0)
    if args.tuning:
        bilu.load_tuning(args.tuning)
    forms = [f for f in args.forms.split(",") if f]
    project = args.ordering != "caller"
    agg = AGGREGATION_DEFAULT if args.aggregation < 0 else bool(args.aggregation)
    w = mg.workload(args.workload)
    recs = {f: time_form(w, FORM_PREC[f], args, project, agg, FORM_DET.get(f)) for f in forms}
    main_rec = recs[forms[0]]
    st = main_rec["stats"]
    roofline, other = roofline_of(main_rec, w, args.steps)
    summaries = {f: form_summary(recs[f], args.steps, FORM_PREC[f]) for f in forms}
    base = main_rec["sec_per_step"]
    ratios = {f: round(recs[f]["sec_per_step"] / base, 4) for f in forms[1:]}
    out = {
        "metric": "BILU factor+FGMRES(1e-8) time",
        "value": round(base, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(base * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": forms[0].split("_")[0],
        "data": "synthetic",
        "config": {
            "workload": w.name, "n": w.a.n, "nnz": w.a.nnz, "tau": w.tau, "restart": w.restart,
            "rtol": 1e-8,
            "ordering": {"caller": "geometric nested dissection (caller permutation)",
                         "project": "nested dissection of the compressed graph (library, level "
                                    "structures)",
                         "multilevel": "multilevel nested dissection of the compressed graph "
                                       "(library)"}[args.ordering],
            "update_precision": forms[0].split("_")[0], "aggregation": agg,
            "update_mfma": args.update_mfma,
            "deterministic": FORM_DET.get(forms[0], args.deterministic),
            "tuning": os.path.relpath(args.tuning, ROOT) if args.tuning else None,
            "tuning_applied": bool(st["tuning_applied"]),
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "other_kernel": other,
        "forms": summaries,
        "time_ratio_vs_first_form": ratios,
        "phases_s": {"analyze": round(main_rec["t_analyze"], 4),
                     "ilu1t": round(st["t_ilu1t"], 4),
                     "factor": round(st["t_factor"], 4),
                     "factor_host_phases": dict(zip(
                         ["ilu1t_sets", "ilu1t_growth", "launch_prep", "factor_kernel",
                          "aggregation", "apply_plan", "statistics"],
                         [round(x, 4) for x in st["t_phase"][:7]]))},
        "factor": {"nblocks": st["nblocks"], "nblocks_initial": st["nblocks_initial"],
                   "max_width": st["max_width"], "avg_width": round(st["avg_width"], 3),
                   "fill": round((st["nnz_l"] + st["nnz_w"] + st["nnz_d"]) / w.a.nnz, 4),
                   "dependency_depth": st["factor_levels"],
                   "apply_levels": [st["apply_levels_fwd"], st["apply_levels_bwd"]]},
    }
    if args.second_workload and args.second_workload != "none":
        w2 = mg.workload(args.second_workload)
        r2 = time_form(w2, 0, args, project, agg)
        roof2, _ = roofline_of(r2, w2, args.steps)
        out["second_workload"] = {"workload": w2.name, "n": w2.a.n, "nnz": w2.a.nnz,
                                  "tau": w2.tau, "restart": w2.restart, "dtype": "f64",
                                  **form_summary(r2, args.steps, 0), "roofline": roof2}
        del w2
    if args.symmetric_workload and args.symmetric_workload != "none":
        out["symmetric_workload"] = time_symmetric(args.symmetric_workload, args, agg)
    if not args.no_cpu_baseline and not project:
        out["cpu_baseline"] = cpu_baseline(w, agg)
    print(json.dumps(out), flush=True)


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


def host_cpu():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(w, agg):
    """The FP64 oracle on the host, one thread, on a bounded sample of the
    workload: the same operator family on a smaller grid (the full 80^3
    sweep takes minutes in the oracle), ILU(1,tau) + sequential sweep +
    FGMRES, scaled to the full workload by the ratio of nonzeros."""
    import numpy as np

    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import matgen as mg
    if w.name.startswith("el3d_") and w.a.n > 400_000:
        sample = "el3d_32_b3"
    else:
        sample = w.name
    ws = mg.workload(sample) if sample != w.name else w
    o = Oracle()
    o.run(ws.a, OracleOptions(tau=ws.tau, use_aggregation=agg), pre_perm=ws.perm)
    t = o.times()
    b = ws.a.matvec(np.ones(ws.a.n))
    t0 = time.perf_counter()
    _, info = o.fgmres(b, restart=ws.restart, rtol=1e-8)
    t_solve = time.perf_counter() - t0
    total = t["ilu1t"] + t["factor"] + t_solve
    scale = w.a.nnz / ws.a.nnz
    model, nproc = host_cpu()
    if ws is w:
        what = (f"the full {w.name} workload (ILU(1,tau) + block Crout sweep + FGMRES, "
                f"{info['iterations']} iterations), one thread")
    else:
        what = (f"{ws.name} (n = {ws.a.n}, {ws.a.nnz} nonzeros; the same operator, tau and "
                f"ordering rule): ILU(1,tau) + block Crout sweep + FGMRES "
                f"({info['iterations']} iterations) on one thread in {round(total, 3)} s, "
                f"scaled by nonzeros x{round(scale, 2)}; the oracle's time grows faster than "
                f"its nonzeros, so this understates a full run")
    return {"value": round(total * scale, 4), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": what, "sample_seconds": round(total, 4),
            "phases_s": {"ilu1t": round(t["ilu1t"], 4), "factor": round(t["factor"], 4),
                         "solve": round(t_solve, 4)},
            "host_cpu": model, "host_nproc": nproc}


if __name__ == "__main__":
    main()
