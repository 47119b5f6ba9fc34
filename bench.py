#!/usr/bin/env python3
"""Benchmark of the EO-preconditioned domain-wall CG on one MI355X.

One step = one full solve D x = b (source preparation, mixed-precision
CG with FP64 defect correction and reliable updates, reconstruction and the
FP64 true-residual check) on the 16^3 x 32, Ns = 16 optimal-DWF workload,
with b and x resident in HBM.  Prints one JSON line: CG Gflops (the paper's
counting convention: 1320 flops per 5D site per hop, 48 Ns per site per dense
fifth-dimension matrix, 24 per subtraction, per-real BLAS) as `value`, plus
algorithmic HBM GB/s, the forward error of the timed solve against the FP64
oracle's stored samples, the roofline of the dominant kernel (HIP-event timed
on the solver's stream), the same workload with FP16 storage (`precision`),
the 12-point-source batched workload against 12 single solves (`batched`), a
200-request served stream against a FIFO single-solve server (`served`) and
the FP64 CPU oracle timed on a bounded sample of the workload.
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
WORKLOADS = {  # name, inner precision, link_compress (-1: the library's default, 12-real)
    "fp32": ("odwf_16x16x16x32_ns16", 1, -1),
    "fp32-18real": ("odwf_16x16x16x32_ns16", 1, 0),
    "fp16": ("odwf_16x16x16x32_ns16_fp16", 2, -1),
    "fp64": ("odwf_16x16x16x32_ns16", 0, 0),
}
# every choice above runs on this lattice; the counter-traffic summaries in
# profiles/ are named after it and the --prec choice
LATTICE = "odwf_16x16x16x32_ns16"
KERNEL_SOURCES = ["paper_1101_0423_amd/csrc/dwf_device.h", "paper_1101_0423_amd/csrc/solver.hip"]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, workload, variant):
    """Counter-measured HBM bytes per launch from profiles/, or None when absent
    or taken on different kernel sources.  variant: the --prec choice
    (precision and link format)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{variant}.txt")
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


def golden_samples(name):
    """Sampled entries of the FP64 oracle's solution (tests/golden, written by
    tests/golden/make_oracle_samples.py from the oracle alone), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_oracle_samples.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def sampled_forward_error(x_dev, g, unbiased=False):
    """Relative forward error of a device solution on the oracle's samples:
    |x_S - xo_S| / |xo_S|, or for a solution concentrated near its source
    (point sources) the unbiased estimate sqrt(N / |S|) |x_S - xo_S| / |xo|."""
    import numpy as np
    import torch
    idx = torch.as_tensor(np.asarray(g["indices"], dtype=np.int64), device=x_dev.device)
    got = x_dev.reshape(-1)[idx].cpu().numpy()
    exp = np.asarray(g["values"])
    e = float(np.linalg.norm(got - exp))
    if unbiased:
        return float(np.sqrt(x_dev.numel() / idx.numel()) * e / g["norm_x"])
    return e / float(np.linalg.norm(exp))


def cpu_baseline(w, U, b, n1=2, n2=12, reps=3):
    """The FP64 oracle, as it stands, on the same workload: the per-iteration
    time is the difference of the median times of runs capped at n1 and n2 CG
    iterations (reps runs each), which removes the set-up and reconstruction."""
    import numpy as np

    import oracle
    args = (U, w["dims"], w["ns"], w["m0"], w["mq"], w["sigma"], w["omega"])
    t = {n1: [], n2: []}
    for _ in range(reps):
        for n in (n1, n2):
            t0 = time.perf_counter()
            oracle.solve(*args, b, tol=1e-12, maxiter=n)
            t[n].append(time.perf_counter() - t0)
    per_it = (float(np.median(t[n2])) - float(np.median(t[n1]))) / (n2 - n1)
    lx, ly, lz, lt = w["dims"]
    v5h = lx * ly * lz * lt * w["ns"] // 2
    flops = v5h * (5280.0 + 192.0 * w["ns"] + 288.0)
    work = sum(sum(v) for v in t.values())
    # one hop (D_w^OE) and one application of C (Eq. (11)) on the same field,
    # median of 5 each: 1320 flops per 5D site per hop, C = two hops, two
    # dense M5 and the subtraction
    th, tc = [], []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.hop(U, w["dims"], w["ns"], 1, b)
        th.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        oracle.schur_c(*args, b)
        tc.append(time.perf_counter() - t0)
    hop_s, c_s = float(np.median(th)), float(np.median(tc))
    # the whole FP64 solve of the small case (4^4, Ns = 8 Shamir), median of 3
    import dwf_inputs as inp
    w0 = inp.workload("shamir_4x4x4x4_ns8")
    U0 = inp.gauge_field(w0["dims"], w0["eps"], seed=w0["seed_gauge"])
    b0 = inp.gaussian_spinor(w0["dims"], w0["ns"], seed=w0["seed_rhs"])
    ts, info = [], None
    for _ in range(3):
        t0 = time.perf_counter()
        _, info = oracle.solve(U0, w0["dims"], w0["ns"], w0["m0"], w0["mq"], w0["sigma"], w0["omega"], b0,
                               tol=1e-10)
        ts.append(time.perf_counter() - t0)
    work += sum(th) + sum(tc) + sum(ts)
    return dict(value=round(flops / per_it * 1e-9, 3), unit="Gflops", cores=oracle.num_threads(), kind="oracle",
                sample=f"FP64 CPU oracle on the same 16^3x32x16 solve: median of {reps} runs capped at {n1} and "
                       f"at {n2} CG iterations, per-iteration time from their difference, converted with the "
                       f"same flop convention; also one hop and one C (median of 5) and the whole 4^4 x 8 solve "
                       f"(median of 3); {work:.1f} s of CPU work in all",
                seconds_per_iteration=per_it,
                hop=dict(seconds=hop_s, gflops=round(1320.0 * v5h / hop_s * 1e-9, 3)),
                schur_c=dict(seconds=c_s, gflops=round((2640.0 + 96.0 * w["ns"] + 24.0) * v5h / c_s * 1e-9, 3)),
                small_solve=dict(workload="shamir_4x4x4x4_ns8", tol=1e-10, seconds=float(np.median(ts)),
                                 iters=info["iters"], converged=info["converged"]))


# the inner kernels of dwf_time_kernels (T once per cycle, then one iteration A B C D)
KERNEL_NAMES = {"T": "cycle_start_m5t", "A": "hop_eo_m5t", "B": "hop_oe_g5_dir", "C": "hop_eo_m5",
                "D": "hop_oe_m5_cgupd_m5t"}
KERNEL_KEYS = [("EpiCgD", "hop_oe_m5_cgupd_m5t"), ("EpiCgB", "hop_oe_g5_dir"),
               ("k_finish", "finish_reduction"), ("EpiOuter", "outer_residual_fp64"),
               ("k_stream_copy<true>", "copy_nontemporal_1GiB"), ("k_stream_copy<false>", "copy_cached_1GiB")]


def kernel_label(name):
    for key, label in KERNEL_KEYS:
        if key in name:
            return label
    if "k_dwf<" in name:
        # k_dwf<Real, F, LF, NSMAX, HOP, MIXM, REGMIX, Pro, Epi>: the low-precision
        # kernels A (hop, M5^T: mode 3), C (hop, M5: mode 2) and T (no hop, M5^T
        # gamma_5: mode 3) store their result
        args = [a.strip() for a in name.split("k_dwf<", 1)[1].split(",")]
        if len(args) >= 9 and args[0] == "float" and "EpiStore" in name:
            if args[4] == "true" and args[5] == "3":
                return "hop_eo_m5t"
            if args[4] == "true" and args[5] == "2":
                return "hop_eo_m5"
            if args[4] == "false" and args[5] == "3":
                return "cycle_start_m5t"
    return name[:90]


def summarize_rocpd(path):
    import sqlite3
    db = sqlite3.connect(path)
    tabs = {r[0] for r in db.execute("select name from sqlite_master")}
    if "pmc_events" in tabs and db.execute("select count(*) from pmc_events").fetchone()[0] > 0:
        # averages over the full dispatches (at least half as long as the
        # kernel's longest): a dispatch of stopped right-hand sides exits at once
        by = {}
        for name, ctr, val, dur in db.execute("select name, counter_name, counter_value, duration from pmc_events"):
            by.setdefault((kernel_label(name), ctr), []).append((dur, val))
        print(f"{'kernel':40s} {'counter':12s} {'dispatches':>10s} {'full':>5s} {'avg value (full)':>17s} "
              f"{'avg us (full)':>14s}")
        for (k, ctr), v in sorted(by.items(), key=lambda kv: -max(d for d, _ in kv[1])):
            full = [(d, x) for d, x in v if d >= 0.5 * max(d for d, _ in v)]
            print(f"{k[:40]:40s} {ctr:12s} {len(v):10d} {len(full):5d} {sum(x for _, x in full) / len(full):17.1f} "
                  f"{sum(d for d, _ in full) / len(full) / 1e3:14.1f}")
        return
    import statistics
    trace = [(kernel_label(n), s, e) for n, s, e in
             db.execute("select name, start, end from kernels order by start").fetchall()]
    by = {}
    for k, s, e in trace:
        by.setdefault(k, []).append(e - s)
    tot = sum(sum(v) for v in by.values())
    # "full": dispatches at least half as long as the kernel's longest; a
    # dispatch whose right-hand sides have all stopped exits at once
    print(f"{'kernel':40s} {'calls':>8s} {'total ms':>10s} {'avg us':>9s} {'full':>6s} {'median us':>10s} "
          f"{'share':>6s}")
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1]))[:20]:
        full = [d for d in v if d >= 0.5 * max(v)]
        print(f"{k[:40]:40s} {len(v):8d} {sum(v) / 1e6:10.2f} {statistics.mean(v) / 1e3:9.2f} {len(full):6d} "
              f"{statistics.median(full) / 1e3:10.2f} {100 * sum(v) / tot:5.1f}%")
    # inner iterations inside the solves: A B C D finish, followed by A
    pat = ["hop_eo_m5t", "hop_oe_g5_dir", "hop_eo_m5", "hop_oe_m5_cgupd_m5t", "finish_reduction"]
    n = len(pat)
    its = [i for i in range(len(trace) - n)
           if [trace[i + j][0] for j in range(n + 1)] == pat + ["hop_eo_m5t"]]
    if its:
        longest = max(trace[i][2] - trace[i][1] for i in its)
        its = [i for i in its if trace[i][2] - trace[i][1] >= 0.5 * longest]
        per = statistics.median(trace[i + n][1] - trace[i][1] for i in its)
        busy = statistics.median(sum(trace[i + j][2] - trace[i + j][1] for j in range(n)) for i in its)
        print(f"\ninner iterations inside the solves ({len(its)} with every kernel live): median period "
              f"{per / 1e3:.2f} us start to start, kernels busy {busy / 1e3:.2f} us of it")
        for j, k in enumerate(pat):
            print(f"  {k:24s} median {statistics.median(trace[i + j][2] - trace[i + j][1] for i in its) / 1e3:8.2f} us")


def _ctx(dwf, U, w, **kw):
    return dwf.Context(U, w["dims"], w["ns"], w["m0"], w["mq"], w["sigma"], w["omega"], device=0, **kw)


def run_batch(nrhs=12, log=True):
    """24^3 x 48, Ns = 16 Shamir, 12 point sources: one 12-right-hand-side
    solve against 12 single-right-hand-side solves of the same sources, each
    timed alone; every true residual from the solver's FP64 check, source 0's
    forward error against the oracle's stored samples."""
    import torch

    import dwf_inputs as inp
    import paper_1101_0423_amd as dwf

    def say(msg):
        if log:
            print(msg, file=sys.stderr, flush=True)

    wname = "shamir_24x24x24x48_ns16_12pt"
    w = inp.workload(wname)
    dims, ns = w["dims"], w["ns"]
    say(f"[bench] generating {wname}")
    U = inp.gauge_field(dims, w["eps"], seed=w["seed_gauge"])
    torch.cuda.set_device(0)
    ctx = _ctx(dwf, U, w)
    B = torch.empty((nrhs,) + ctx.spinor_shape(), dtype=torch.float64, device="cuda")
    for k in range(nrhs):
        B[k].copy_(torch.from_numpy(inp.point_source(dims, ns, k, seed=w["seed_rhs"])))
    X = torch.zeros_like(B)
    X1 = torch.zeros_like(B[0])
    params = dwf.default_params(inner_prec=1, tol=1e-10)
    # build both engines (and their graphs) outside the timed region
    warm = dwf.default_params(inner_prec=1, tol=1e-10, maxiter=8)
    ctx.solve_dev(B, X, nrhs=nrhs, params=warm)
    ctx.solve_dev(B[0], X1, nrhs=1, params=warm)
    X.zero_()
    X1.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_b, rc_b = ctx.solve_dev(B, X, nrhs=nrhs, params=params)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    say(f"[bench] batched {nrhs}: rc={rc_b} {t_batch:.2f}s iters={[s['iters'] for s in st_b]}")
    g = golden_samples(wname + "_rhs0")
    fwd0 = sampled_forward_error(X[0], g, unbiased=True) if g is not None else None
    ms_b, by_b = ctx.time_kernels(params=params, nrhs=nrhs, launches=5)
    t_seq, st_s, diff = 0.0, [], 0.0
    for k in range(nrhs):
        X1.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rc = ctx.solve_dev(B[k], X1, nrhs=1, params=params)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        st_s.append((st[0], rc))
        diff = max(diff, float(torch.linalg.vector_norm(X[k] - X1) / torch.linalg.vector_norm(X1)))
        say(f"[bench] single {k}: rc={rc} {st[0]['seconds']:.2f}s iters={st[0]['iters']}")
    ms_1, by_1 = ctx.time_kernels(params=params, nrhs=1, launches=5)
    flops = sum(s["gflops"] for s in st_b[:1]) * st_b[0]["seconds"] * 1e9
    gbytes = st_b[0]["hbm_gbytes"]
    names = KERNEL_NAMES
    kern = {names[k]: dict(ms_batch=round(ms_b[k], 4), ms_single=round(ms_1[k], 4),
                           gbs_batch=round(by_b[k] / (ms_b[k] * 1e-3) * 1e-9, 1),
                           gbs_single=round(by_1[k] / (ms_1[k] * 1e-3) * 1e-9, 1)) for k in ms_b}
    ctx.close()
    del B, X, X1
    torch.cuda.empty_cache()
    return dict(workload=f"{wname}: 24^3x48 lattice, Ns=16 Shamir, m0=1.8, mq=0.005, SU(3) links eps=0.5, "
                         f"{nrhs} point sources at one seeded 5D site, tol 1e-10, FP32 inner / FP64 outer",
                nrhs=nrhs, solves_per_s=round(nrhs / t_batch, 4), seconds=round(t_batch, 3),
                sequential_solves_per_s=round(nrhs / t_seq, 4), sequential_seconds=round(t_seq, 3),
                speedup=round(t_seq / t_batch, 3), gflops=round(flops / t_batch * 1e-9, 1),
                hbm_gbs=round(gbytes / t_batch, 1),
                converged=all(s["status"] == 0 for s in st_b) and all(rc == 0 for _, rc in st_s),
                max_true_residual=max(s["true_residual"] for s in st_b),
                forward_error_source0=fwd0,
                forward_error_kind="unbiased estimate sqrt(N/|S|) |x_S - xo_S| / |xo| from 4096 uniform samples of "
                                   "the FP64 oracle's solution of source 0 (solved to 1e-12)",
                batch_vs_single_max_rel_diff=diff, iters=[s["iters"] for s in st_b],
                rhs_per_workgroup=st_b[0]["rhs_per_block"], kernels=kern)


def run_batch_small(nrhs=12, reps=3, log=True):
    """8^3 x 16, Ns = 16, 12 Gaussian sources: the batched form where one
    solve is too small to fill the GPU.  Median of reps batched solves against
    the median of reps rounds of 12 single solves; every true residual from the
    solver's FP64 check."""
    import torch

    import dwf_inputs as inp
    import paper_1101_0423_amd as dwf

    wname = "odwf_8x8x8x16_ns16_12rhs"
    w = inp.workload(wname)
    dims, ns = w["dims"], w["ns"]
    U = inp.gauge_field(dims, w["eps"], seed=w["seed_gauge"])
    torch.cuda.set_device(0)
    ctx = _ctx(dwf, U, w)
    B = torch.from_numpy(inp.gaussian_spinor(dims, ns, seed=w["seed_rhs"], nrhs=nrhs)).cuda()
    X = torch.zeros_like(B)
    X1 = torch.zeros_like(B[0])
    params = dwf.default_params(inner_prec=1, tol=1e-10)
    ctx.solve_dev(B, X, nrhs=nrhs, params=params)  # engines, tuning and graphs outside the timing
    ctx.solve_dev(B[0], X1, nrhs=1, params=params)
    tb, ts, stb, sts = [], [], None, []
    for _ in range(reps):
        X.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stb, rcb = ctx.solve_dev(B, X, nrhs=nrhs, params=params)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        t = 0.0
        sts = []
        for k in range(nrhs):
            X1.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, rc = ctx.solve_dev(B[k], X1, nrhs=1, params=params)
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            sts.append((st[0], rc))
        ts.append(t)
    diff = float(torch.linalg.vector_norm(X[nrhs - 1] - X1) / torch.linalg.vector_norm(X1))
    ctx.close()
    del B, X, X1
    torch.cuda.empty_cache()
    t_b, t_s = sorted(tb)[reps // 2], sorted(ts)[reps // 2]
    if log:
        print(f"[bench] small batched {nrhs}: {t_b:.3f} s vs {t_s:.3f} s sequential", file=sys.stderr, flush=True)
    return dict(workload=f"{wname}: 8^3x16 lattice, Ns=16, m0=1.8, mq=0.01, sigma=omega~U[0.5,1.5], SU(3) links "
                         f"eps=0.5, {nrhs} Gaussian sources, tol 1e-10, FP32 inner / FP64 outer",
                nrhs=nrhs, seconds=round(t_b, 4), sequential_seconds=round(t_s, 4),
                solves_per_s=round(nrhs / t_b, 2), sequential_solves_per_s=round(nrhs / t_s, 2),
                speedup=round(t_s / t_b, 3), timing=f"median of {reps} batched solves and of {reps} rounds of "
                                                      f"{nrhs} single solves",
                converged=all(s["status"] == 0 for s in stb) and all(rc == 0 for _, rc in sts),
                max_true_residual=max(s["true_residual"] for s in stb),
                batch_vs_single_rel_diff_last=diff, iters=[s["iters"] for s in stb],
                rhs_per_workgroup=stb[0]["rhs_per_block"])


def batch_bench(args):
    r = run_batch(args.nrhs)
    r["small_lattice"] = run_batch_small(args.nrhs)
    line = dict(metric="batched solves/s (24^3x48, Ns=16, 12 point sources)", value=r["solves_per_s"],
                unit="solves/s", n_gpus=1, steps=1, warmup=1, ms_per_step=round(r["seconds"] * 1e3, 1),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32 inner / f64 outer",
                data="synthetic", config=dict(workload=r["workload"], nrhs=r["nrhs"]),
                **{k: v for k, v in r.items() if k not in ("workload", "nrhs", "solves_per_s")})
    print(json.dumps(line), flush=True)


def run_serve(n_requests, load, log=True, fifo_run=False):
    """Poisson stream of independent solves on four resident fields (every
    (field, Ns) pair is one context), served by dwf_submit/dwf_poll, against a
    FIFO server of plain single-right-hand-side solves (dwf_solve, one request
    at a time in arrival order) on the same stream: simulated from each request
    type's service time measured here (median of 3 solves), and with fifo_run
    also run for real.  Latencies are from arrival to completion, p50 and p99
    by the same definition (numpy's interpolated percentile) for both servers.
    Returns the measurements as a dict."""
    import threading

    import numpy as np
    import torch

    import dwf_inputs as inp
    import paper_1101_0423_amd as dwf

    def say(msg):
        if log:
            print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    reqs = inp.serve_stream(n_requests)
    used = sorted({(r["field"], r["ns"]) for r in reqs})
    ctxs, rhs, gauges = {}, {}, {}
    for f, ns in used:
        o = inp.serve_operator(f, ns)
        if f not in gauges:
            gauges[f] = inp.gauge_field(o["dims"], o["eps"], seed=o["seed_gauge"])
        ctxs[(f, ns)] = dwf.Context(gauges[f], o["dims"], ns, o["m0"], inp.SERVE_MQ[0], o["sigma"], o["omega"],
                                    device=0)
        for k in range(inp.SERVE_RHS_PER_OPERATOR):
            rhs[(f, ns, k)] = inp.gaussian_spinor(o["dims"], ns, seed=inp.serve_rhs_seed(f, ns, k))
    say(f"[serve] {len(ctxs)} operators resident")
    params = dwf.default_params(inner_prec=1, tol=1e-10)
    # plain single-right-hand-side service time of every request type (a
    # context per mass, so that dwf_solve runs that mass)
    svc, fctx = {}, {}
    for r in reqs:
        key = (r["field"], r["ns"], r["mq"])
        if key in svc:
            continue
        o = inp.serve_operator(r["field"], r["ns"])
        c = dwf.Context(gauges[r["field"]], o["dims"], r["ns"], o["m0"], r["mq"], o["sigma"], o["omega"], device=0)
        b = rhs[(r["field"], r["ns"], 0)]
        c.solve(b, params=dwf.default_params(inner_prec=1, tol=1e-10, maxiter=8))  # engine and graph
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            x, st, rc = c.solve(b, params=params)
            ts.append(time.perf_counter() - t0)
        svc[key] = float(np.median(ts))
        if fifo_run:
            fctx[key] = c
        else:
            c.close()
        say(f"[serve] plain service {key}: {svc[key]:.3f}s iters={st[0]['iters']}")
    mean_svc = float(np.mean([svc[(r["field"], r["ns"], r["mq"])] for r in reqs]))
    if load > 0:
        rate = load / mean_svc
        arrivals = np.cumsum([r["gap"] for r in reqs]) / rate
        arrivals -= arrivals[0]
    else:  # saturated: every request is there at the start
        arrivals = np.zeros(len(reqs))
    # FIFO single-right-hand-side server: each request starts when it has
    # arrived and the previous one is done
    done, fifo_lat = 0.0, []
    for r, a in zip(reqs, arrivals):
        done = max(done, a) + svc[(r["field"], r["ns"], r["mq"])]
        fifo_lat.append(done - a)
    fifo_span = done
    fifo_real = None
    if fifo_run:
        say(f"[serve] FIFO run of {len(reqs)} requests")
        lat_f, ok_f = [], True
        t_start = time.perf_counter()
        for i, (r, a) in enumerate(zip(reqs, arrivals)):
            delay = t_start + a - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            x, st, rc = fctx[(r["field"], r["ns"], r["mq"])].solve(rhs[(r["field"], r["ns"], r["rhs"])],
                                                                   params=params)
            ok_f &= rc == dwf.DWF_OK
            lat_f.append(time.perf_counter() - t_start - a)
            if (i + 1) % 50 == 0:
                say(f"[serve] FIFO: {i + 1} of {len(reqs)} requests done")
        span_f = time.perf_counter() - t_start
        for c in fctx.values():
            c.close()
        fifo_real = dict(solves_per_s=round(len(reqs) / span_f, 4),
                         p50_latency_s=round(float(np.percentile(lat_f, 50)), 4),
                         p99_latency_s=round(float(np.percentile(lat_f, 99)), 4), converged=bool(ok_f),
                         kind="plain single-RHS dwf_solve calls in arrival order, run on this GPU")
    # warm the server: one request per operator builds its lane
    warm = [ctxs[k].submit(rhs[k + (0,)], mq=inp.SERVE_MQ[-1], params=params) for k in ctxs]
    for t, k in zip(warm, ctxs):
        while dwf.poll(t, ctxs[k].spinor_shape(), timeout_us=100000)[0] == dwf.DWF_PENDING:
            pass
    dwf.server_stats(reset=True)
    tickets = [None] * len(reqs)
    t_start = time.perf_counter()

    def submitter():
        for i, (r, a) in enumerate(zip(reqs, arrivals)):
            delay = t_start + a - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            k = (r["field"], r["ns"])
            tickets[i] = ctxs[k].submit(rhs[k + (r["rhs"],)], mq=r["mq"], params=params)

    th = threading.Thread(target=submitter)
    th.start()
    pending = set(range(len(reqs)))
    results = [None] * len(reqs)
    last_report = time.perf_counter()
    while pending:
        for i in list(pending):
            if tickets[i] is None:
                continue
            r = reqs[i]
            rc, x, st = dwf.poll(tickets[i], ctxs[(r["field"], r["ns"])].spinor_shape(), timeout_us=0)
            if rc != dwf.DWF_PENDING:
                results[i] = (rc, st["true_residual"], time.perf_counter() - t_start - arrivals[i])
                pending.discard(i)
        if time.perf_counter() - last_report > 10:
            last_report = time.perf_counter()
            say(f"[serve] {len(reqs) - len(pending)} of {len(reqs)} requests done")
        time.sleep(0.002)
    span = time.perf_counter() - t_start
    th.join()
    s = dwf.server_stats()
    lat = np.array([l for _, _, l in results])
    for c in ctxs.values():
        c.close()
    out = dict(requests=len(reqs), load=load, solves_per_s=round(len(reqs) / span, 4),
               solves_per_busy_s=round(s["completed"] / s["busy_seconds"], 4) if s["busy_seconds"] > 0 else None,
               p50_latency_s=round(float(np.percentile(lat, 50)), 4),
               p99_latency_s=round(float(np.percentile(lat, 99)), 4),
               latency_kind="arrival to completion, numpy percentile (the same for the FIFO server)",
               server_p50_p99_s=[round(s["p50_latency"], 4), round(s["p99_latency"], 4)],
               peak_batch=s["peak_batch"], waits_for_memory=s["waits_for_memory"],
               busy_s=round(s["busy_seconds"], 3),
               fifo=dict(solves_per_s=round(len(reqs) / fifo_span, 4), solves_per_busy_s=round(1.0 / mean_svc, 4),
                         p50_latency_s=round(float(np.percentile(fifo_lat, 50)), 4),
                         p99_latency_s=round(float(np.percentile(fifo_lat, 99)), 4),
                         kind="simulated: plain single-RHS solves in arrival order, each request type's service "
                              "time measured on this GPU (median of 3 dwf_solve calls)"),
               mean_plain_service_s=round(mean_svc, 4),
               converged=all(rc == dwf.DWF_OK for rc, _, _ in results),
               max_true_residual=max(r for _, r, _ in results))
    if fifo_real is not None:
        out["fifo_run"] = fifo_real
    return out


SERVE_WORKLOAD = ("fields 8^3x16, 12^3x24, 2x 16^3x32 (eps 0.5); per request Ns in {8,16,32}, "
                  "mq in {0.01,0.03,0.1}, sigma=omega~U[0.5,1.5], m0=1.8, Gaussian RHS, tol 1e-10")


def serve_bench(args):
    r = run_serve(args.requests, args.load, fifo_run=args.fifo_run)
    arrivals = (f"Poisson arrivals at {args.load} x the plain single-RHS service rate" if args.load > 0
                else "all submitted at once (saturated)")
    line = dict(metric="served solves/s, p99 latency (Poisson stream, 4 resident fields)",
                value=r["solves_per_s"], unit="solves/s", n_gpus=1, steps=r["requests"], warmup=0,
                ms_per_step=round(1e3 / r["solves_per_s"], 2), higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32 inner / f64 outer", data="synthetic",
                config=dict(workload=f"{r['requests']} requests, {arrivals}; {SERVE_WORKLOAD}",
                            requests=r["requests"], load=args.load), **{k: v for k, v in r.items()
                                                                         if k not in ("requests", "load")})
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=sorted(WORKLOADS), default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-launches", type=int, default=20)
    ap.add_argument("--mode", choices=["solve", "kernels", "batch", "serve"], default="solve",
                    help="kernels: one short solve without graphs, then each inner kernel timed "
                         "(the program the counter runs profile); batch: 12 point sources on 24^3x48, Ns=16, "
                         "batched vs sequential; serve: Poisson request stream, served vs FIFO")
    ap.add_argument("--nrhs", type=int, default=12, help="batch mode: right-hand sides")
    ap.add_argument("--requests", type=int, default=200, help="serve mode: requests in the stream")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="solve mode: requests of the served stream measured after the solves (0: none)")
    ap.add_argument("--no-extra", action="store_true",
                    help="solve mode: skip the precision (FP16) and batched blocks")
    ap.add_argument("--fifo-run", action="store_true",
                    help="serve mode: also run the FIFO single-solve server on the stream (not only simulate it)")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serve mode: arrival rate / plain service rate (0: all requests at once)")
    ap.add_argument("--summarize-rocpd", metavar="DB", help="print per-kernel statistics of a rocprofv3 "
                    "results database (kernel trace or --pmc) and exit")
    args = ap.parse_args()
    if args.summarize_rocpd:
        summarize_rocpd(args.summarize_rocpd)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; there is no multi-GPU path "
              "(a single solve would shard by 4D domain decomposition of the lattice)", file=sys.stderr)
        sys.exit(2)

    if args.mode == "batch":
        return batch_bench(args)
    if args.mode == "serve":
        return serve_bench(args)

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
    if args.mode == "kernels":
        kp = dwf.default_params(inner_prec=prec, link_compress=lc, use_graph=0, maxiter=40)
        st, rc = ctx.solve_dev(bd, xd, params=kp)
        ms, by = ctx.time_kernels(params=kp, launches=5)
        # counter calibration: plain copies of a known size (1 GiB, four times
        # the Infinity Cache), with cached and with non-temporal accesses
        n = 1 << 30
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        side = torch.cuda.Stream()  # the library never uses the legacy null stream
        torch.cuda.synchronize()
        copy_gbs = {}
        for nt in (False, True):
            t = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(side)
                dwf.stream_copy(src, dst, nontemporal=nt, stream=side.cuda_stream)
                e1.record(side)
                e1.synchronize()
                t.append(e0.elapsed_time(e1) * 1e-3)
            # bytes read plus bytes written, per second, median of three
            copy_gbs["nontemporal" if nt else "cached"] = round(2 * n / sorted(t)[1] * 1e-9, 1)
        del src, dst
        print(json.dumps(dict(mode="kernels", workload=wname, ms={k: ms[k] for k in ms},
                              bytes={k: by[k] for k in by}, copy_bytes_read=n, copy_bytes_written=n,
                              copy_read_plus_write_gbs=copy_gbs)), flush=True)
        ctx.close()
        return

    def say(msg):
        print(msg, file=sys.stderr, flush=True)

    r = run_solve(dwf, ctx, bd, xd, prec, lc, args.steps, args.warmup, args.kernel_launches, say)
    g = golden_samples("odwf_16x16x16x32_ns16")
    fwd = sampled_forward_error(xd, g) if g is not None else None
    traffic = counter_traffic(r["dominant"], LATTICE, args.prec)
    roofline = dict(r["roofline"], traffic=traffic)
    line = dict(metric=METRIC, value=r["gflops"], unit="Gflops", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=r["ms_per_step"], higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype=r["dtype"], data="synthetic",
                config=dict(workload=f"{wname}: 16^3x32 lattice, Ns=16, m0=1.8, mq=0.01, sigma=omega~U[0.5,1.5], "
                                     f"SU(3) links eps=0.5, Gaussian RHS, tol 1e-10",
                            lattice=list(dims), Ns=ns, inner_prec=["fp64", "fp32", "fp16"][prec],
                            link_real=18 if (lc == 0 or prec == 0) else 12, reliable_updates=True),
                hbm_gbs=r["hbm_gbs"], iters=r["iters"], true_residual=r["true_residual"],
                forward_error=fwd,
                forward_error_kind="|x_S - xo_S| / |xo_S| over 4096 uniform samples of the FP64 oracle's solution "
                                   "(solved to 1e-12), for the last timed solve",
                converged=r["converged"], roofline=roofline, kernels=r["kernels"])
    if args.prec == "fp32" and not args.no_extra:
        # the precision form: the same workload with FP16 storage and FP32 arithmetic
        say("[bench] precision form: FP16 storage")
        r16 = run_solve(dwf, ctx, bd, xd, 2, -1, max(3, args.steps // 4), 1, args.kernel_launches, say)
        line["precision"] = dict(
            workload=f"{wname} with FP16 storage (binary16 spinors with one FP32 scale per 5D site, 12-real "
                     f"binary16 links), FP32 arithmetic, FP64 outer residual / solution / reductions",
            steps=max(3, args.steps // 4), gflops=r16["gflops"], hbm_gbs=r16["hbm_gbs"],
            ms_per_step=r16["ms_per_step"], iters=r16["iters"], true_residual=r16["true_residual"],
            forward_error=sampled_forward_error(xd, g) if g is not None else None, converged=r16["converged"],
            dominant_kernel=dict(r16["roofline"], kernel=r16["dominant"],
                                 traffic=counter_traffic(r16["dominant"], LATTICE, "fp16")),
            kernels=r16["kernels"])
    ctx.close()
    del bd, xd
    torch.cuda.empty_cache()
    if args.prec == "fp32" and not args.no_extra:
        say("[bench] batched form: 24^3x48, 12 point sources")
        line["batched"] = run_batch(12)
        say("[bench] batched form on a small lattice: 8^3x16, 12 sources")
        line["batched"]["small_lattice"] = run_batch_small(12)
    if args.serve_requests > 0:
        say(f"[bench] served stream of {args.serve_requests} requests")
        sv = run_serve(args.serve_requests, 0.8)
        line["served"] = dict(workload=f"{sv['requests']} requests, Poisson arrivals at 0.8 x the plain "
                                       f"single-RHS service rate; {SERVE_WORKLOAD}", **sv)
    if not args.no_cpu_baseline:
        say("[bench] timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(w, U, b)
    print(json.dumps(line), flush=True)


def run_solve(dwf, ctx, bd, xd, prec, lc, steps, warmup, launches, say):
    """Timed solves of D x = b with b and x resident in HBM, then each inner
    kernel timed with HIP events on the solver's stream."""
    import torch
    params = dwf.default_params(inner_prec=prec, link_compress=lc, tol=1e-10)
    for i in range(warmup):
        st, rc = ctx.solve_dev(bd, xd, params=params)
        say(f"[bench] warmup {i}: rc={rc} {st[0]}")
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(steps):
        st, rc = ctx.solve_dev(bd, xd, params=params)
        stats.append((st[0], rc))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, (s, rc) in enumerate(stats):
        say(f"[bench] step {i}: rc={rc} iters={s['iters']} res={s['true_residual']:.3e} "
            f"t={s['seconds']:.4f}s {s['gflops']:.1f} Gflops")
    flops = sum(s["gflops"] * s["seconds"] for s, _ in stats) * 1e9
    gbytes = sum(s["hbm_gbytes"] for s, _ in stats)
    ms, by = ctx.time_kernels(params=params, launches=launches)
    dom = max(ms, key=ms.get)
    names = KERNEL_NAMES
    achieved = by[dom] / (ms[dom] * 1e-3) * 1e-9
    return dict(gflops=round(flops / elapsed * 1e-9, 2), hbm_gbs=round(gbytes / elapsed, 1),
                ms_per_step=round(elapsed / steps * 1e3, 3), iters=stats[-1][0]["iters"],
                true_residual=stats[-1][0]["true_residual"], converged=all(rc == dwf.DWF_OK for _, rc in stats),
                dtype={0: "f64", 1: "f32 inner / f64 outer", 2: "f16 storage, f32 arithmetic / f64 outer"}[prec],
                dominant=names[dom],
                roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(achieved / HBM_PEAK_GBS, 4), kernel=names[dom],
                              algorithmic_bytes_per_launch=by[dom], avg_launch_ms=round(ms[dom], 5)),
                kernels={names[k]: dict(ms=round(ms[k], 5), gbs=round(by[k] / (ms[k] * 1e-3) * 1e-9, 1))
                         for k in ms})


if __name__ == "__main__":
    main()
