#!/usr/bin/env python3
"""Benchmark of the EO-preconditioned domain-wall CG on one MI355X.

One step = one full solve D x = b (source preparation, mixed-precision
CG with FP64 defect correction and reliable updates, reconstruction and the
FP64 true-residual check) on the 16^3 x 32, Ns = 16 optimal-DWF workload,
with b and x resident in HBM.  Prints one JSON line: CG Gflops (the paper's
counting convention) as `value`, plus algorithmic HBM GB/s, the
roofline of the dominant kernel (HIP-event timed on the solver's stream) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CG Gflops & HBM GB/s (16^3x32, Ns=16) + served solves/s, p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "fp32": ("odwf_16x16x16x32_ns16", 1, 0),
    "fp16": ("odwf_16x16x16x32_ns16_fp16", 2, 1),
    "fp64": ("odwf_16x16x16x32_ns16", 0, 0),
}
KERNEL_SOURCES = ["paper_1101_0423_amd/csrc/dwf_device.h", "paper_1101_0423_amd/csrc/solver.hip"]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, workload):
    """Counter-measured HBM bytes per launch from profiles/, or None when absent
    or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, U, b, n1=1, n2=5):
    """The FP64 oracle, as it stands, on the same workload: per-iteration time
    from two bounded runs (n1 and n2 CG iterations)."""
    import oracle
    args = (U, w["dims"], w["ns"], w["m0"], w["mq"], w["sigma"], w["omega"])
    t = []
    for n in (n1, n2):
        t0 = time.perf_counter()
        oracle.solve(*args, b, tol=1e-12, maxiter=n)
        t.append(time.perf_counter() - t0)
    per_it = (t[1] - t[0]) / (n2 - n1)
    lx, ly, lz, lt = w["dims"]
    v5h = lx * ly * lz * lt * w["ns"] // 2
    flops = v5h * (5280.0 + 192.0 * w["ns"] + 288.0)
    return dict(value=round(flops / per_it * 1e-9, 3), unit="Gflops", cores=oracle.num_threads(), kind="oracle",
                sample=f"FP64 CPU oracle, CG iterations {n1}..{n2} of the same solve (per-iteration time from "
                       f"the difference of two runs; {sum(t):.1f} s of CPU work)",
                seconds_per_iteration=per_it)


KERNEL_KEYS = [("ProCgE", "cg_dir_m5t"), ("EpiCgD", "hop_oe_m5_cgupd"), ("EpiCgB", "hop_oe_g5_sub"),
               ("k_finish", "finish_reduction"), ("EpiOuter", "outer_residual_fp64")]


def kernel_label(name):
    for key, label in KERNEL_KEYS:
        if key in name:
            return label
    if "k_dwf" in name and "true, 3, dwf::ProLoad<dwf::FS>, dwf::EpiStore<dwf::FS" in name:
        return "hop_eo_m5t"
    if "k_dwf" in name and "true, 2, dwf::ProLoad<dwf::FS>, dwf::EpiStore<dwf::FS" in name:
        return "hop_eo_m5"
    return name[:90]


def summarize_rocpd(path):
    import sqlite3
    db = sqlite3.connect(path)
    tabs = {r[0] for r in db.execute("select name from sqlite_master")}
    if "pmc_events" in tabs and db.execute("select count(*) from pmc_events").fetchone()[0] > 0:
        rows = db.execute("select name, counter_name, count(*), avg(counter_value), avg(duration) "
                          "from pmc_events group by name, counter_name order by avg(duration) desc").fetchall()
        print(f"{'kernel':40s} {'counter':12s} {'dispatches':>10s} {'avg value':>14s} {'avg us':>9s}")
        for name, ctr, n, val, dur in rows:
            print(f"{kernel_label(name):40s} {ctr:12s} {n:10d} {val:14.1f} {dur / 1e3:9.1f}")
        return
    rows = db.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                      "group by name order by sum(duration) desc").fetchall()
    tot = sum(r[2] for r in rows)
    print(f"{'kernel':40s} {'calls':>8s} {'total ms':>10s} {'avg us':>9s} {'share':>6s}")
    for name, n, s, a in rows[:20]:
        print(f"{kernel_label(name):40s} {n:8d} {s / 1e6:10.2f} {a / 1e3:9.2f} {100 * s / tot:5.1f}%")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=sorted(WORKLOADS), default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-launches", type=int, default=20)
    ap.add_argument("--mode", choices=["solve", "kernels"], default="solve",
                    help="kernels: one short solve without graphs, then each inner kernel timed "
                         "(the driver for counter runs)")
    ap.add_argument("--summarize-rocpd", metavar="DB", help="print per-kernel statistics of a rocprofv3 "
                    "results database (kernel trace or --pmc) and exit")
    args = ap.parse_args()
    if args.summarize_rocpd:
        summarize_rocpd(args.summarize_rocpd)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; there is no multi-GPU path "
              "(a single solve would shard by 4D domain decomposition, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import dwf_inputs as inp
    import paper_1101_0423_amd as dwf

    wname, prec, lc = WORKLOADS[args.prec]
    w = inp.workload(wname)
    dims, ns = w["dims"], w["ns"]
    print(f"[bench] generating {wname}", file=sys.stderr, flush=True)
    U = inp.gauge_field(dims, w["eps"], seed=w["seed_gauge"])
    b = inp.gaussian_spinor(dims, ns, seed=w["seed_rhs"])
    torch.cuda.set_device(0)
    ctx = dwf.Context(U, dims, ns, w["m0"], w["mq"], w["sigma"], w["omega"], device=0)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    params = dwf.default_params(inner_prec=prec, link_compress=lc, tol=1e-10)
    if args.mode == "kernels":
        kp = dwf.default_params(inner_prec=prec, link_compress=lc, use_graph=0, maxiter=40)
        st, rc = ctx.solve_dev(bd, xd, params=kp)
        ms, by = ctx.time_kernels(params=kp, launches=5)
        print(json.dumps(dict(mode="kernels", workload=wname, ms={k: ms[k] for k in ms},
                              bytes={k: by[k] for k in by})), flush=True)
        ctx.close()
        return
    for i in range(args.warmup):
        st, rc = ctx.solve_dev(bd, xd, params=params)
        print(f"[bench] warmup {i}: rc={rc} {st[0]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        st, rc = ctx.solve_dev(bd, xd, params=params)
        stats.append((st[0], rc))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, (s, rc) in enumerate(stats):
        print(f"[bench] step {i}: rc={rc} iters={s['iters']} res={s['true_residual']:.3e} "
              f"t={s['seconds']:.4f}s {s['gflops']:.1f} Gflops", file=sys.stderr, flush=True)
    flops = sum(s["gflops"] * s["seconds"] for s, _ in stats) * 1e9
    gbytes = sum(s["hbm_gbytes"] for s, _ in stats)
    value = flops / elapsed * 1e-9
    ok = all(rc == dwf.DWF_OK for _, rc in stats)

    # per-kernel device time on the solver's stream (HIP events), same process
    ms, by = ctx.time_kernels(params=params, launches=args.kernel_launches)
    dom = max(ms, key=ms.get)
    names = {"E": "cg_dir_m5t", "A": "hop_eo_m5t", "B": "hop_oe_g5_sub", "C": "hop_eo_m5", "D": "hop_oe_m5_cgupd"}
    achieved = by[dom] / (ms[dom] * 1e-3) * 1e-9
    traffic = counter_traffic(names[dom], wname)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=names[dom],
                    algorithmic_bytes_per_launch=by[dom], avg_launch_ms=round(ms[dom], 5))
    kernels = {names[k]: dict(ms=round(ms[k], 5), gbs=round(by[k] / (ms[k] * 1e-3) * 1e-9, 1)) for k in ms}

    line = dict(metric=METRIC, value=round(value, 2), unit="Gflops", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(elapsed / args.steps * 1e3, 3), higher_is_better=True,
                scaling="weak", vs_baseline=None,
                dtype={0: "f64", 1: "f32 inner / f64 outer", 2: "f16 storage, f32 arithmetic / f64 outer"}[prec],
                data="synthetic",
                config=dict(workload=f"{wname}: 16^3x32 lattice, Ns=16, m0=1.8, mq=0.01, sigma=omega~U[0.5,1.5], "
                                     f"SU(3) links eps=0.5, Gaussian RHS, tol 1e-10",
                            lattice=list(dims), Ns=ns, inner_prec=["fp64", "fp32", "fp16"][prec],
                            link_real=12 if lc else 18, reliable_updates=True),
                hbm_gbs=round(gbytes / elapsed, 1), iters=stats[-1][0]["iters"],
                true_residual=stats[-1][0]["true_residual"], converged=ok,
                roofline=roofline, kernels=kernels)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, U, b)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
