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
WORKLOADS = {  # name, inner precision, link_compress (-1: the library's default, 12-real)
    "fp32": ("odwf_16x16x16x32_ns16", 1, -1),
    "fp32-18real": ("odwf_16x16x16x32_ns16", 1, 0),
    "fp16": ("odwf_16x16x16x32_ns16_fp16", 2, -1),
    "fp64": ("odwf_16x16x16x32_ns16", 0, 0),
}
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


def cpu_baseline(w, U, b, n1=1, n2=30):
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
    if "k_dwf<" in name:
        # k_dwf<Real, F, LF, NSMAX, HOP, MIXM, REGMIX, Pro, Epi>: the low-precision
        # hop-only kernels A (M5^T, mode 3) and C (M5, mode 2) store their result
        args = [a.strip() for a in name.split("k_dwf<", 1)[1].split(",")]
        if len(args) >= 9 and args[0] == "float" and args[4] == "true" and "EpiStore" in name:
            if args[5] == "3":
                return "hop_eo_m5t"
            if args[5] == "2":
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


def _ctx(dwf, U, w, **kw):
    return dwf.Context(U, w["dims"], w["ns"], w["m0"], w["mq"], w["sigma"], w["omega"], device=0, **kw)


def batch_bench(args):
    """24^3 x 48, Ns = 16 Shamir, 12 point sources: one 12-right-hand-side
    solve against 12 single-right-hand-side solves of the same sources."""
    import numpy as np
    import torch

    import dwf_inputs as inp
    import paper_1101_0423_amd as dwf

    wname = "shamir_24x24x24x48_ns16_12pt"
    w = inp.workload(wname)
    dims, ns = w["dims"], w["ns"]
    nrhs = args.nrhs
    print(f"[bench] generating {wname}", file=sys.stderr, flush=True)
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
    print(f"[bench] batched {nrhs}: rc={rc_b} {t_batch:.2f}s iters={[s['iters'] for s in st_b]}",
          file=sys.stderr, flush=True)
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
        print(f"[bench] single {k}: rc={rc} {st[0]['seconds']:.2f}s iters={st[0]['iters']}", file=sys.stderr,
              flush=True)
    ms_1, by_1 = ctx.time_kernels(params=params, nrhs=1, launches=5)
    flops = sum(s["gflops"] for s in st_b[:1]) * st_b[0]["seconds"] * 1e9
    names = {"E": "cg_dir_m5t", "A": "hop_eo_m5t", "B": "hop_oe_g5_sub", "C": "hop_eo_m5", "D": "hop_oe_m5_cgupd"}
    kern = {names[k]: dict(ms_batch=round(ms_b[k], 4), ms_single=round(ms_1[k], 4),
                           gbs_batch=round(by_b[k] / (ms_b[k] * 1e-3) * 1e-9, 1),
                           gbs_single=round(by_1[k] / (ms_1[k] * 1e-3) * 1e-9, 1)) for k in ms_b}
    line = dict(metric="batched solves/s (24^3x48, Ns=16, 12 point sources)", value=round(nrhs / t_batch, 4),
                unit="solves/s", n_gpus=1, steps=1, warmup=1, ms_per_step=round(t_batch * 1e3, 1),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32 inner / f64 outer",
                data="synthetic",
                config=dict(workload=f"{wname}: 24^3x48 lattice, Ns=16 Shamir, m0=1.8, mq=0.005, SU(3) links "
                                     f"eps=0.5, {nrhs} point sources at one seeded 5D site, tol 1e-10",
                            nrhs=nrhs),
                sequential_solves_per_s=round(nrhs / t_seq, 4), speedup=round(t_seq / t_batch, 3),
                batch_gflops=round(flops / t_batch * 1e-9, 1),
                converged=all(s["status"] == 0 for s in st_b) and all(rc == 0 for _, rc in st_s),
                max_true_residual=max(s["true_residual"] for s in st_b),
                batch_vs_single_max_rel_diff=diff, iters=[s["iters"] for s in st_b],
                rhs_per_workgroup=st_b[0]["rhs_per_block"], kernels=kern)
    ctx.close()
    print(json.dumps(line), flush=True)


def run_serve(n_requests, load, log=True):
    """Poisson stream of independent solves on four resident fields (every
    (field, Ns) pair is one context), served by dwf_submit/dwf_poll, against a
    FIFO server of plain single-right-hand-side solves on the same stream.
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
    svc = {}
    for r in reqs:
        key = (r["field"], r["ns"], r["mq"])
        if key in svc:
            continue
        o = inp.serve_operator(r["field"], r["ns"])
        c = dwf.Context(gauges[r["field"]], o["dims"], r["ns"], o["m0"], r["mq"], o["sigma"], o["omega"], device=0)
        b = rhs[(r["field"], r["ns"], 0)]
        c.solve(b, params=dwf.default_params(inner_prec=1, tol=1e-10, maxiter=8))  # engine and graph
        t0 = time.perf_counter()
        x, st, rc = c.solve(b, params=params)
        svc[key] = time.perf_counter() - t0
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
    return dict(requests=len(reqs), load=load, solves_per_s=round(len(reqs) / span, 4),
                solves_per_busy_s=round(s["completed"] / s["busy_seconds"], 4) if s["busy_seconds"] > 0 else None,
                p50_latency_s=round(s["p50_latency"], 4), p99_latency_s=round(s["p99_latency"], 4),
                p50_latency_from_arrival_s=round(float(np.percentile(lat, 50)), 4),
                p99_latency_from_arrival_s=round(float(np.percentile(lat, 99)), 4),
                peak_batch=s["peak_batch"], waits_for_memory=s["waits_for_memory"],
                busy_s=round(s["busy_seconds"], 3),
                fifo=dict(solves_per_s=round(len(reqs) / fifo_span, 4), solves_per_busy_s=round(1.0 / mean_svc, 4),
                          p50_latency_s=round(float(np.percentile(fifo_lat, 50)), 4),
                          p99_latency_s=round(float(np.percentile(fifo_lat, 99)), 4),
                          kind="plain single-RHS solves in arrival order; service time of each request type "
                               "measured on this GPU"),
                mean_plain_service_s=round(mean_svc, 4),
                converged=all(rc == dwf.DWF_OK for rc, _, _ in results),
                max_true_residual=max(r for _, r, _ in results))


SERVE_WORKLOAD = ("fields 8^3x16, 12^3x24, 2x 16^3x32 (eps 0.5); per request Ns in {8,16,32}, "
                  "mq in {0.01,0.03,0.1}, sigma=omega~U[0.5,1.5], m0=1.8, Gaussian RHS, tol 1e-10")


def serve_bench(args):
    r = run_serve(args.requests, args.load)
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
                         "(the driver for counter runs); batch: 12 point sources on 24^3x48, Ns=16, "
                         "batched vs sequential; serve: Poisson request stream, served vs FIFO")
    ap.add_argument("--nrhs", type=int, default=12, help="batch mode: right-hand sides")
    ap.add_argument("--requests", type=int, default=200, help="serve mode: requests in the stream")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="solve mode: requests of the served stream measured after the solves (0: none)")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serve mode: arrival rate / plain service rate (0: all requests at once)")
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

    if args.mode == "batch":
        return batch_bench(args)
    if args.mode == "serve":
        return serve_bench(args)

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
        # counter calibration: the layout conversions of an M5 application move
        # known bytes in each storage format (k_host_to_half / k_half_to_host)
        for pr in (dwf.PREC_FP64, dwf.PREC_FP32, dwf.PREC_FP16):
            ctx.apply_dev(dwf.OP_M5, bd, xd, prec=pr)
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
    traffic = counter_traffic(names[dom], wname, args.prec)
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
                            link_real=18 if (lc == 0 or prec == 0) else 12, reliable_updates=True),
                hbm_gbs=round(gbytes / elapsed, 1), iters=stats[-1][0]["iters"],
                true_residual=stats[-1][0]["true_residual"], converged=ok,
                roofline=roofline, kernels=kernels)
    ctx.close()
    if args.serve_requests > 0:
        print(f"[bench] served stream of {args.serve_requests} requests", file=sys.stderr, flush=True)
        sv = run_serve(args.serve_requests, 0.8)
        line["served"] = dict(workload=f"{sv['requests']} requests, Poisson arrivals at 0.8 x the plain "
                                       f"single-RHS service rate; {SERVE_WORKLOAD}", **sv)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, U, b)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
