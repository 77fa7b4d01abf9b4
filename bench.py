"""Throughput benchmark of the phi-combination solver on one MI355X.

Workload: the 2-D advection-diffusion-reaction operator
A = 1e-2 L5 - 10 (Dx + Dy) + diag(r), r ~ U[-1, 0], on a 2048 x 2048 periodic
grid (N = 4,194,304, h = 1/2048), p = 3 with b_0..b_3 ~ N(0, 1), FP64, IOP
window q = 2, tol = 1e-8, m_init = 10.  One step is one sweep over the five
step sizes tau in {1e-3, 10^-2.5, 1e-2, 10^-1.5, 1e-1}: five solves.
Inputs are resident in device memory before the timed region.

Output: one JSON line (see README of the run contract): solves/s, the
roofline record of the persistent solve kernel (algorithmic bytes from the
solver's own count / kernel time measured with HIP events on the launch
stream), and a CPU baseline of the oracle on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "φ-combination solves/s at tol 1e-8; HBM GB/s vs peak; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side", type=int, default=2048)
    ap.add_argument("--taus", type=str, default="")
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--estimate", type=int, default=0, choices=(0, 1, 2),
                    help="error estimate (Section 3.4): 0 Eq. (36), 1 two terms of Eq. (35), 2 corrected scheme")
    ap.add_argument("--precision", type=str, default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-substeps", type=int, default=1,
                    help="substeps of the one-thread CPU oracle sample")
    ap.add_argument("--traffic-json", type=str, default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--workload", choices=("adr2d", "diff3d", "batch", "serve", "small", "probe", "epirk"),
                    default="adr2d",
                    help="adr2d: the 2048^2 tau sweep (default); diff3d: the 256^3 variable-"
                         "coefficient solve; batch: 256 2-D problems in one launch vs a per-solve loop; "
                         "probe: the streaming ceiling of the device (the library's plain streaming kernel); "
                         "epirk: EPIRK4s3A on the paper's nonlinear 2-D ADR problem (400^2, t in [0, 0.1])")
    ap.add_argument("--epirk-side", type=int, default=400)
    ap.add_argument("--epirk-steps", type=str, default="10,20,40,80", help="step counts over [0, 0.1] (epirk)")
    ap.add_argument("--probe-mib", type=int, default=1024, help="MiB per array (probe)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--serve-count", type=int, default=48, help="requests per arrival rate (serve)")
    ap.add_argument("--serve-lams", type=str, default="100,1000,5000", help="arrival rates, req/s (serve)")
    ap.add_argument("--serve-group", type=int, default=16, help="workgroups per server group (serve)")
    ap.add_argument("--serve-pool-gb", type=float, default=64.0, help="HBM budget of the server (serve)")
    ap.add_argument("--traffic-from", type=str, default="", metavar="FETCH_CSV,WRITE_CSV",
                    help="no GPU work: turn the rocprofv3 counter files of two bench runs (--pmc FETCH_SIZE, "
                         "--pmc WRITE_SIZE, each with --calibrate-copy) into the traffic record --traffic-out")
    ap.add_argument("--traffic-key", type=str, default="", help="workload key of the traffic record")
    ap.add_argument("--traffic-out", type=str, default="", help="traffic record to write (JSON)")
    ap.add_argument("--print-maps", action="store_true",
                    help="print /proc/self/maps to stderr at exit (to resolve addresses of a crash in teardown)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, run one plain device copy of MIB MiB (a known-size "
                         "kernel that HBM traffic counters are scaled by)")
    return ap.parse_args()


def _host_info():
    """nproc and the CPU model of the host (lscpu), for the baseline record."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    return info


def cpu_baseline(pr_sample, sweep_taus, one_thread_substeps):
    """Time the oracle's exact-result route (full-Arnoldi Krylov, oracle/arnoldi.py,
    as it stands) on one whole solve of the smallest-tau point of the sweep, on
    the host's cores, and once more on one thread over its first substeps.

    The oracle's stencil products are single-threaded NumPy; its orthogonal-
    isation (tall-skinny products) runs on the BLAS thread pool.  The sweep rate
    is the whole solve's time scaled by sum(tau) / tau_sample (the oracle's
    substep count grows linearly in tau: each substep covers a bounded tau||A||);
    the factor is stated in the record."""
    import numpy as np  # noqa: F401
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import operators
    from oracle.arnoldi import phi_combination_arnoldi
    ap = operators.make_apply(pr_sample.op)
    blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    st = {}
    t0 = time.perf_counter()
    phi_combination_arnoldi(ap, pr_sample.tau, pr_sample.vectors, tol_o=1e-3 * pr_sample.tol, m=48, stats=st)
    t_solve = time.perf_counter() - t0
    st1 = {}
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        phi_combination_arnoldi(ap, pr_sample.tau, pr_sample.vectors, tol_o=1e-3 * pr_sample.tol, m=48,
                                stats=st1, stop_after=one_thread_substeps)
        t_one = time.perf_counter() - t1
    factor = sum(sweep_taus) / pr_sample.tau
    t_sweep = t_solve * factor
    one_solve_est = t_one * pr_sample.tau / max(st1["t"], 1e-300)
    return {
        "value": len(sweep_taus) / t_sweep,
        "unit": "solves/s",
        "cores": int(blas_threads),
        "kind": "oracle",
        "sample": (f"one whole solve of the same problem (N={pr_sample.n}) at tau={pr_sample.tau:g} by the oracle's full-Arnoldi "
                   f"route (m=48, CGS2, tol_o=1e-11): {st['substeps']} substeps, {st['matvecs']} products, "
                   f"{t_solve:.1f} s measured on {blas_threads} BLAS threads (stencil products single-threaded); "
                   f"sweep rate = 5 / (that time x sum(tau)/tau = {factor:.1f})"),
        "measured_solve_s": t_solve,
        "measured_solves_per_s_at_tau": 1.0 / t_solve,
        "sweep_extrapolation_factor": factor,
        "one_thread": {"substeps": st1["substeps"], "products": st1["matvecs"], "seconds": t_one,
                       "t_covered": st1["t"], "solve_s_estimate": one_solve_est},
        "host": _host_info(),
    }


def main():
    args = parse()
    if args.traffic_from:
        return _write_traffic(args)
    if args.print_maps:
        import atexit
        atexit.register(lambda: sys.stderr.write(open("/proc/self/maps").read()))
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(instances shard by GPU with no exchange; see the design notes).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    import paper_1804_05126_amd as K

    if args.workload == "diff3d":
        return bench_diff3d(args, W, K, np, torch)
    if args.workload == "batch":
        return bench_batch(args, W, K, np, torch)
    if args.workload == "serve":
        return bench_serve(args, W, K, np, torch)
    if args.workload == "small":
        return bench_small(args, W, K, np, torch)
    if args.workload == "probe":
        return bench_probe(args, K, torch)
    if args.workload == "epirk":
        return bench_epirk(args, K, torch)
    taus = [float(t) for t in args.taus.split(",")] if args.taus else W.cfg2_tau_grid()
    side = args.side
    pr = W.cfg2(side, taus[0], q=args.q)       # operator and vectors shared by the sweep
    dev = torch.device("cuda:0")
    op = K.Operator.from_desc(pr.op, precision=args.precision)
    vecs = [torch.as_tensor(v, device=dev) for v in pr.vectors]
    w = torch.empty(pr.n, dtype=torch.float64, device=dev)
    tol = 1e-8 if args.precision == "fp64" else 1e-6
    stream = torch.cuda.current_stream()
    elem = "double" if args.precision == "fp64" else "float"

    def one_solve(tau):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        _, st, _ = K.phi_combination(op, tau, vecs, tol=tol, m_init=10, q=args.q, out=w, estimate=args.estimate)
        ev1.record(stream)
        return ev0, ev1, st

    for i in range(args.warmup):
        for tau in taus:
            one_solve(tau)
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    records = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        for tau in taus:
            ev0, ev1, st = one_solve(tau)
            records.append((tau, ev0, ev1, st))
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    times_ms = [ev0.elapsed_time(ev1) for _, ev0, ev1, _ in records]
    total_bytes = sum(st["alg_bytes"] for *_, st in records)
    total_ms = sum(times_ms)
    achieved = total_bytes / (total_ms * 1e-3) / 1e9
    n_solves = len(records)
    per_tau = {}
    for (tau, _, _, st), ms in zip(records, times_ms):
        d = per_tau.setdefault(f"{tau:.4g}", {"ms": [], "matvecs": st["matvecs"], "substeps": st["substeps"],
                                              "rejections": st["rejections"], "m_last": st["m_last"],
                                              "alg_GB": st["alg_bytes"] / 1e9})
        d["ms"].append(ms)
    for d in per_tau.values():
        d["ms"] = float(np.median(d["ms"]))
    traffic = _traffic(args.traffic_json, f"adr2d-{side}-{args.precision}-q{args.q}")
    lat = sorted(times_ms)
    out = {
        "metric": METRIC,
        "value": n_solves / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-basis/f64-accumulate",
        "data": "synthetic",
        "config": {
            "workload": (f"2D ADR {side}^2 periodic (N={pr.n}), A=1e-2 L5 - 10(Dx+Dy) + diag(r), "
                         f"r~U[-1,0], p=3, b_k~N(0,1), tau sweep {taus}, tol {tol:g}, IOP q={args.q}, "
                         f"m_init=10, m_max={records[0][3]['m_max']}"),
            "solves_per_step": len(taus),
            "precision": args.precision, "estimate": args.estimate,
            "seed": pr.seed,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": (f"kiops_solve_kernel<{K._lib.PASS_NAMES.get(records[0][3]['pass_kind'], '?')}<{elem}>, {elem}> "
                       f"(one persistent launch per solve)"),
            "algorithmic_bytes_per_launch": total_bytes / n_solves,
            "avg_launch_ms": total_ms / n_solves,
        },
        "latency_ms": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]},
        "matvecs_per_s": sum(st["matvecs"] for *_, st in records) / wall,
        "per_tau": per_tau,
    }
    _calibrate_copy(args, torch, out)
    # release the device objects before the host-side baseline and the exit
    torch.cuda.synchronize()
    op.close()
    del op, vecs, w
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        sample = W.cfg2(side, taus[0], q=args.q)
        print("[bench] timing the CPU oracle (one whole solve)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sample, taus, args.cpu_sample_substeps)
    print(json.dumps(out), flush=True)


def bench_epirk(args, K, torch):
    """EPIRK4s3A (Eq. (51)) on the paper's 2-D ADR problem at --epirk-side^2
    over t in [0, 0.1] with constant steps (two solver calls per step, m warm
    start across steps); for each step count: wall time, products with the
    Jacobian, and the error against the run with the most steps at tol 1e-12
    (the reference is that self-run, as no independent solver of this size is
    at hand)."""
    from paper_1804_05126_amd.epirk import ADR2D, EPIRK4s3A
    prob = ADR2D(args.epirk_side)
    u0 = prob.initial_condition()
    counts = [int(c) for c in args.epirk_steps.split(",")]
    T = 0.1
    ref = EPIRK4s3A(prob, tol=1e-12).integrate(u0, T / (2 * max(counts)), 2 * max(counts))
    rows = []
    for k in counts:
        for warm in (True, False):
            integ = EPIRK4s3A(prob, tol=1e-8, warm_start=warm)
            integ.integrate(u0, T / k, 1)          # untimed: builds workspaces
            integ = EPIRK4s3A(prob, tol=1e-8, warm_start=warm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u = integ.integrate(u0, T / k, k)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            err = float(torch.linalg.norm(u - ref) / torch.linalg.norm(ref))
            mv = [sum(s.matvecs[c] for s in integ.history) for c in (0, 1)]
            rows.append({"steps": k, "h": T / k, "warm_start": warm, "seconds": el, "steps_per_s": k / el,
                         "products_call1": mv[0], "products_call2": mv[1], "rel_err": err,
                         "m_last_final": integ.history[-1].m_last})
            print(f"[epirk] {k} steps warm={warm}: {el * 1e3:.1f} ms, products {mv}, err {err:.2e}",
                  file=sys.stderr, flush=True)
    best = max((r for r in rows if r["warm_start"]), key=lambda r: r["steps"])
    out = {"metric": "EPIRK4s3A time steps/s (2 phi-combination solves per step)", "value": best["steps_per_s"],
           "unit": "steps/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"nonlinear 2-D ADR {args.epirk_side}^2 periodic, eps 1e-2, alpha -10, "
                                  f"gamma 100, t in [0, 0.1], tol 1e-8, q 2"},
           "rows": rows}
    print(json.dumps(out), flush=True)
    prob.close()
    return 0


def bench_probe(args, K, torch):
    """Streaming ceiling: dst = src_0 + ... + src_{r-1} over arrays of
    --probe-mib MiB by the library's plain streaming kernel (16-byte loads),
    for r = 1 (a copy), 2, 4 and 6 reads per write (the 5-point pass streams
    about six arrays per one written) and three grid sizes; HIP events on the
    launch stream, best grid per r."""
    n = (args.probe_mib << 20) // 8
    srcs = [torch.full((n,), 1.0 + k, dtype=torch.float64, device="cuda") for k in range(6)]
    dst = torch.empty(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    rows = []
    for r in (1, 2, 4, 6):
        best = None
        for blocks in (512, 1024, 2048, 4096):
            for _ in range(2):
                K.stream_probe(srcs[:r], dst, blocks=blocks)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = max(1, args.steps) * 5
            e0.record(stream)
            for _ in range(reps):
                K.stream_probe(srcs[:r], dst, blocks=blocks)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = (r + 1) * n * 8 / (ms * 1e-3) / 1e9
            rows.append({"reads": r, "blocks": blocks, "us": ms * 1e3, "GB_s": gbs})
            if best is None or gbs > best["GB_s"]:
                best = rows[-1]
        print(f"[probe] {r} reads + 1 write: best {best['GB_s']:.0f} GB/s at {best['blocks']} workgroups",
              file=sys.stderr, flush=True)
    expect = sum(1.0 + k for k in range(6))
    ok = bool(torch.all(dst == expect).item())
    out = {"metric": "streaming ceiling (HBM GB/s of dst = sum of r arrays)", "unit": "GB/s",
           "peak": HBM_PEAK_GBS, "array_MiB": args.probe_mib, "result_checked": ok,
           "best": {str(r): max((x for x in rows if x["reads"] == r), key=lambda x: x["GB_s"]) for r in (1, 2, 4, 6)},
           "rows": rows}
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def _calibrate_copy(args, torch, out):
    """One plain streaming copy of a known size after the timed region, by the
    library's own probe kernel (dst = src, 16-byte loads), so that hardware byte
    counters can be scaled by what they read for it."""
    if args.calibrate_copy <= 0:
        return
    import paper_1804_05126_amd as K
    nbytes = args.calibrate_copy << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    K.stream_probe([src], dst, blocks=1024)      # reads and writes nbytes
    torch.cuda.synchronize()
    out["copy_calibration_bytes"] = nbytes
    del src, dst


def traffic_from_counters(fetch_csv, write_csv, key, out_path, kernel="kiops_solve_kernel"):
    """HBM bytes per launch of the solve kernel from two rocprofv3 counter runs.

    FETCH_SIZE and WRITE_SIZE (kilobytes per dispatch) of every dispatch whose
    name contains `kernel` are scaled by what the same counter reads for the
    calibration copy of the run (the library's streaming kernel, which reads
    and writes a known number of bytes: --calibrate-copy) and averaged over
    the launches.  Writes a record keyed by the workload and the current
    kernel sources, which the bench then reports as roofline.traffic."""
    import csv

    def per_dispatch(path, counter):
        rows = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            k = (r["Dispatch_Id"], r["Kernel_Name"])
            rows[k] = rows.get(k, 0.0) + float(r["Counter_Value"])
        return rows

    out = {"workload_key": key, "kernel_source_hash": _kernel_hash(), "counters": {}}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = per_dispatch(path, name)
        calib = [v for (d, n), v in rows.items() if "stream_probe_kernel" in n]
        launches = [v for (d, n), v in sorted(rows.items(), key=lambda x: int(x[0][0])) if kernel in n]
        if len(calib) != 1 or not launches:
            raise RuntimeError(f"{path}: need one calibration copy and the solve launches")
        # the copy moves copy_bytes in each direction; the counter reads kilobytes
        out["counters"][name] = {"calibration_kib": calib[0], "launch_kib": launches}
    return out


def _write_traffic(args):
    fetch_csv, write_csv = args.traffic_from.split(",")
    rec = traffic_from_counters(fetch_csv, write_csv, args.traffic_key, args.traffic_out)
    copy_bytes = float(args.calibrate_copy << 20)
    f = rec["counters"]["FETCH_SIZE"]
    w = rec["counters"]["WRITE_SIZE"]
    fetch_scale = copy_bytes / (f["calibration_kib"] * 1024.0)
    write_scale = copy_bytes / (w["calibration_kib"] * 1024.0)
    fb = [v * 1024.0 * fetch_scale for v in f["launch_kib"]]
    wb = [v * 1024.0 * write_scale for v in w["launch_kib"]]
    rec.update(fetch_scale=fetch_scale, write_scale=write_scale, launches=len(fb),
               fetch_bytes_per_launch=sum(fb) / len(fb), write_bytes_per_launch=sum(wb) / len(wb),
               hbm_bytes_per_launch=(sum(fb) + sum(wb)) / len(fb),
               per_launch_GB=[(a + b) / 1e9 for a, b in zip(fb, wb)])
    json.dump(rec, open(args.traffic_out, "w"), indent=1)
    print(json.dumps({k: rec[k] for k in ("workload_key", "hbm_bytes_per_launch", "fetch_scale", "write_scale")}))


def _traffic(path, key):
    """HBM bytes per launch from a counter summary under profiles/, if it was
    taken for this workload key and the current kernel sources."""
    if not os.path.exists(path):
        return None
    try:
        tj = json.load(open(path))
    except Exception:
        return None
    if tj.get("workload_key") != key or tj.get("kernel_source_hash") != _kernel_hash():
        return None
    return tj.get("hbm_bytes_per_launch")


def _lat(ms):
    lat = sorted(ms)
    return {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]}


def bench_diff3d(args, W, K, np, torch):
    """The 256^3 variable-coefficient diffusion-reaction solve (p = 2, tau = 1e-3,
    tol 1e-6); one step = one solve."""
    pr = W.cfg3(precision=args.precision)
    op = K.Operator.from_desc(pr.op, precision=args.precision)
    vecs = [torch.as_tensor(v, device="cuda") for v in pr.vectors]
    w = torch.empty(pr.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    recs = []

    def one():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, st, _ = K.phi_combination(op, pr.tau, vecs, tol=pr.tol, m_init=pr.m_init, q=args.q, out=w,
                                     estimate=args.estimate)
        e1.record(stream)
        return e0, e1, st
    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        recs.append(one())
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b, _ in recs]
    alg = sum(st["alg_bytes"] for *_, st in recs) / len(recs)
    achieved = alg / (sum(ms) / len(ms) * 1e-3) / 1e9
    st = recs[-1][2]
    out = {
        "metric": METRIC, "value": len(recs) / wall, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-basis/f64-accumulate", "data": "synthetic",
        "config": {"workload": (f"3D 7-point diffusion-reaction 256^3 periodic (N={pr.n}), kappa = box-averaged "
                                f"exp(N(0,0.5^2)), r~U[-5,0], p=2, tau=1e-3, tol {pr.tol:g}, IOP q={args.q}"),
                   "precision": args.precision, "estimate": args.estimate, "seed": pr.seed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _traffic(os.path.join(ROOT, "profiles", "traffic_diff3d.json"),
                                         f"diff3d-{args.precision}-q{args.q}"),
                     "kernel": (f"kiops_solve_kernel<{'Stencil3DNarrow' if args.q in (1, 2) else 'Stencil3D'}"
                                f"<{'double' if args.precision == 'fp64' else 'float'}>> (one persistent launch per solve)"),
                     "algorithmic_bytes_per_launch": alg,
                     "avg_launch_ms": sum(ms) / len(ms)},
        "latency_ms": _lat(ms),
        "solve": {k: st[k] for k in ("matvecs", "substeps", "rejections", "m_last", "grid_blocks")},
    }
    _calibrate_copy(args, torch, out)
    print(json.dumps(out), flush=True)


def bench_small(args, W, K, np, torch):
    """The 32^2 problem (N = 1024, p = 2, tau = 1e-2, tol 1e-8, q = 2): one solve
    at a time (latency), 1000 solves back to back on one stream, and the same
    1000 solves as one batched launch."""
    pr = W.cfg1()
    op = K.Operator.from_desc(pr.op)
    vecs = [torch.as_tensor(v, device="cuda") for v in pr.vectors]
    w = torch.empty(pr.n, dtype=torch.float64, device="cuda")
    count = 1000
    for _ in range(10):
        K.phi_combination(op, pr.tau, vecs, tol=pr.tol, out=w)
    torch.cuda.synchronize()
    lat = []
    for _ in range(50):
        s0 = time.perf_counter()
        _, st, _ = K.phi_combination(op, pr.tau, vecs, tol=pr.tol, out=w)
        lat.append((time.perf_counter() - s0) * 1e3)
    t0 = time.perf_counter()
    for _ in range(count):
        K.phi_combination(op, pr.tau, vecs, tol=pr.tol, out=w)
    torch.cuda.synchronize()
    loop_s = time.perf_counter() - t0
    outs = [torch.empty(pr.n, dtype=torch.float64, device="cuda") for _ in range(count)]
    probs = [dict(op=op, tau=pr.tau, vectors=vecs, tol=pr.tol, m_init=pr.m_init, q=pr.q, out=o) for o in outs]
    best, rows, _ = K.batch_tune_shape(probs, group_sizes=(8, 16, 32), tile_rows=(16, 8, 4))
    K.phi_batch(probs, group_size=best, tile_rows=rows)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, stats, status, plan = K.phi_batch(probs, group_size=best, tile_rows=rows)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t1
    ok = all(x["status"] == 0 for x in stats) and all(torch.equal(o, outs[0]) for o in outs[1:])
    out = {
        "metric": METRIC, "value": count / batch_s, "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": batch_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2-D ADR 32^2 (N=1024), p=2, tau=1e-2, tol 1e-8, q=2, m_init 10; 1000 solves",
                   "seed": pr.seed, "group_size": best, "tile_rows": rows},
        "roofline": {"bound": "latency", "achieved": None, "peak": None, "unit": None, "frac": None, "traffic": None,
                     "note": "the 48 KiB working set stays in L2; per-step barriers and epilogues dominate"},
        "single_solve_ms": _lat(lat), "matvecs_per_solve": st["matvecs"],
        "back_to_back_solves_per_s": count / loop_s, "batched_solves_per_s": count / batch_s,
        "batched_results_identical": ok,
    }
    print(json.dumps(out), flush=True)


def bench_batch(args, W, K, np, torch):
    """The batched workload: batch-count independent 2-D problems (side log-U[64,512],
    p in 1..4, tau log-U[1e-4,1e-1]) in one persistent launch, against the same
    problems solved one after another; the group size and the 2-D tile height
    are autotuned first."""
    prec = args.precision
    prs = W.cfg4(count=args.batch_count, precision=prec)
    probs = []
    for pr in prs:
        op = K.Operator.from_desc(pr.op, precision=prec)
        probs.append(dict(op=op, tau=pr.tau, vectors=[torch.as_tensor(v, device="cuda") for v in pr.vectors],
                          tol=pr.tol, m_init=pr.m_init, q=args.q))
    print("[bench] inputs ready", file=sys.stderr, flush=True)
    gcands, rcands = (8, 16, 32, 64), (16, 8, 4)
    best, rows, tune_ms = K.batch_tune_shape(probs, group_sizes=gcands, tile_rows=rcands)
    print(f"[bench] tuned group size {best}, tiles of 64 x {rows}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        K.phi_batch(probs, group_size=best, tile_rows=rows)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        outs, stats, status, plan = K.phi_batch(probs, group_size=best, tile_rows=rows)
        print(f"[bench] batch step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    batch_solves_s = len(probs) * args.steps / wall
    alg = sum(st["alg_bytes"] for st in stats)
    # the same problems one by one (the plain form), each on the whole GPU
    lat = []
    t1 = time.perf_counter()
    for pb in probs:
        s0 = time.perf_counter()
        K.phi_combination(pb["op"], pb["tau"], pb["vectors"], tol=pb["tol"], m_init=pb["m_init"], q=pb["q"])
        lat.append((time.perf_counter() - s0) * 1e3)
    loop_wall = time.perf_counter() - t1
    print("[bench] per-solve loop done", file=sys.stderr, flush=True)
    # completion times with every problem submitted at once: in the batch, the
    # device clock at each solve's end minus the batch's earliest start (last
    # timed batch); one by one, the running sum of the solve times in order
    t_first = min(st["clock_start_s"] for st in stats)
    batch_done = [(st["clock_end_s"] - t_first) * 1e3 for st in stats]
    loop_done = list(np.cumsum(lat))
    out = {
        "metric": METRIC, "value": batch_solves_s, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32-basis/f64-accumulate", "data": "synthetic",
        "config": {"workload": (f"batch of {len(probs)} 2-D ADR problems, side log-U[64,512], eps~U[1e-3,1e-1], "
                                f"alpha~U[-20,20], r~U[-1,0], p~U{{1..4}}, tau~log-U[1e-4,1e-1], tol {prs[0].tol:g}"),
                   "precision": prec, "seed": prs[0].seed, "group_size": best, "tile_rows": rows,
                   "groups": plan[0]},
        "roofline": {"bound": "hbm", "achieved": alg / (wall / args.steps) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg / (wall / args.steps) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"kiops_group_kernel<Stencil2D> (64 x {rows} tiles)"},
        "per_solve_loop": {"solves_per_s": len(probs) / loop_wall, **_lat(lat)},
        "batch_latency_ms": wall * 1e3 / args.steps,
        "completion_ms": {"batched": _lat(batch_done), "one_by_one": _lat(loop_done),
                          "note": "all problems submitted at t = 0; batched from the device clock, one by one "
                                  "as the running sum of per-solve times (host clock)"},
        "autotune": {"group_sizes": list(gcands), "tile_rows": list(rcands), "best_group_size": best,
                     "best_tile_rows": rows, "best_ms": tune_ms},
        "statuses_ok": all(st["status"] == 0 for st in stats),
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, W, K, np, torch):
    """The served workload: a Poisson stream of requests (half 2-D ADR with side
    log-U[64,2048], half 3-D diffusion-reaction with side log-U[32,192]; p in 1..4;
    tau log-U[1e-4,1e-1]; half mixed at tol 1e-6, half FP64 at tol 1e-8) replayed
    in real time at each arrival rate, against a server with an HBM budget.  The
    same requests are also solved by the plain form, one at a time in arrival
    order on the whole GPU (FIFO), replayed at the same arrival times.  Latency is
    completion (as seen by the host loop) minus scheduled arrival."""
    lams = [float(x) for x in args.serve_lams.split(",")]
    reqs = W.cfg5_requests(lam=lams[0], count=args.serve_count)
    gaps = np.diff([0.0] + [r.arrival_s for r in reqs]) * lams[0]   # unit-rate gaps; same draws at every rate
    inputs = []
    for r in reqs:
        pr = r.materialize()
        op = K.Operator.from_desc(pr.op, precision=pr.precision)
        vecs = [torch.as_tensor(v, device="cuda") for v in pr.vectors]
        w = torch.empty(pr.n, dtype=torch.float64, device="cuda")
        inputs.append((r, op, vecs, w))
        del pr
    torch.cuda.synchronize()
    print(f"[bench] {len(inputs)} requests ready", file=sys.stderr, flush=True)

    def solve_alone(r, op, vecs, w):
        _, st, status = K.phi_combination(op, r.tau, vecs, tol=r.tol, out=w)
        return st
    # warm-up: one small request of each family through the plain form
    for r, op, vecs, w in sorted(inputs, key=lambda x: x[0].n)[:4]:
        solve_alone(r, op, vecs, w)
    torch.cuda.synchronize()
    # service times of the plain form (each request alone on the whole GPU)
    service = []
    alg = 0.0
    for r, op, vecs, w in inputs:
        s0 = time.perf_counter()
        st = solve_alone(r, op, vecs, w)
        service.append(time.perf_counter() - s0)
        alg += st["alg_bytes"]
        print(f"[bench]   {r.kind} side {r.side} p {r.p} tau {r.tau:.2e} {r.precision}: "
              f"{service[-1] * 1e3:.1f} ms, {st['matvecs']} matvecs", file=sys.stderr, flush=True)
    print(f"[bench] plain-form service times measured: total {sum(service):.2f} s", file=sys.stderr, flush=True)

    def fifo(arrivals):
        """Plain form replayed live: each request starts when it has arrived and
        the previous one has finished."""
        lat = []
        t0 = time.perf_counter()
        for (r, op, vecs, w), a in zip(inputs, arrivals):
            now = time.perf_counter() - t0
            if now < a:
                time.sleep(a - now)
            solve_alone(r, op, vecs, w)
            lat.append(time.perf_counter() - t0 - a)
        return lat, time.perf_counter() - t0 - arrivals[0]

    def served(arrivals):
        srv = K.Server(pool_bytes=int(args.serve_pool_gb * (1 << 30)), group_size=args.serve_group)
        lat = [None] * len(inputs)
        tickets = {}
        nxt = 0
        stats = []
        t0 = time.perf_counter()
        try:
            while len(stats) < len(inputs):
                now = time.perf_counter() - t0
                while nxt < len(inputs) and arrivals[nxt] <= now:
                    r, op, vecs, w = inputs[nxt]
                    tickets[srv.submit(op, r.tau, vecs, tol=r.tol, out=w)] = nxt
                    nxt += 1
                srv.progress()
                finished = False
                for t in list(tickets):
                    done, st, _ = srv.result(t)
                    if done:
                        i = tickets.pop(t)
                        lat[i] = time.perf_counter() - t0 - arrivals[i]
                        stats.append(st)
                        finished = True
                        r = inputs[i][0]
                        mv = max(st["matvecs"], 1)
                        print(f"[bench]   served {r.kind} {r.side} {r.precision}: at {arrivals[i] * 1e3:.1f} ms, "
                              f"latency {lat[i] * 1e3:.1f} ms, {st['grid_blocks']} wg, {mv} matvecs, per matvec "
                              f"work {st['time_work_s'] / mv * 1e6:.1f} wait {st['time_wait_s'] / mv * 1e6:.1f} "
                              f"epi {st['time_epilogue_s'] / mv * 1e6:.1f} us", file=sys.stderr, flush=True)
                if not finished:
                    time.sleep(2e-4)
                if time.perf_counter() - t0 > 600:
                    raise RuntimeError("served requests did not finish within 600 s")
            span = time.perf_counter() - t0 - arrivals[0]
        finally:
            srv.close()
        return lat, span, stats

    rows = []
    for lam in lams:
        arrivals = list(np.cumsum(gaps) / lam)
        lat_s, span_s, stats = served(arrivals)
        ok = all(st["status"] == 0 for st in stats)
        lat_f, span_f = fifo(arrivals)
        row = {"lambda_req_s": lam,
               "served": {"solves_per_s": len(inputs) / span_s, **_lat([x * 1e3 for x in lat_s]),
                          "statuses_ok": ok},
               "plain_fifo": {"solves_per_s": len(inputs) / span_f, **_lat([x * 1e3 for x in lat_f])}}
        rows.append(row)
        print(f"[bench] lambda {lam:g}: {json.dumps(row)}", file=sys.stderr, flush=True)
    head = rows[min(1, len(rows) - 1)]
    span = len(inputs) / head["served"]["solves_per_s"]
    out = {
        "metric": METRIC, "value": head["served"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": len(inputs), "warmup": 4, "ms_per_step": span * 1e3 / len(inputs), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 and f32-basis/f64-accumulate", "data": "synthetic",
        "config": {"workload": (f"served: {len(inputs)} Poisson arrivals, 2-D ADR side log-U[64,2048] / "
                                f"3-D diffusion-reaction side log-U[32,192], p~U{{1..4}}, tau~log-U[1e-4,1e-1], "
                                f"tol 1e-6 mixed / 1e-8 FP64, HBM budget {args.serve_pool_gb:g} GB"),
                   "lambda_req_s": head["lambda_req_s"], "group_size": args.serve_group,
                   "requests_2d": sum(r.kind == "2d" for r, *_ in inputs),
                   "requests_mixed": sum(r.precision == "mixed" for r, *_ in inputs)},
        "roofline": {"bound": "hbm", "achieved": alg / span / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / span / 1e9 / HBM_PEAK_GBS, "traffic": None, "kernel": "kiops_serve_kernel"},
        "latency_ms": {k: head["served"][k] for k in ("p50", "p99")},
        "sweep": rows,
        "plain_service_s": {"total": sum(service), "max": max(service)},
    }
    print(json.dumps(out), flush=True)


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1804_05126_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    _rc = main()
    if _rc:   # a normal run ends by falling off the end (no SystemExit)
        sys.exit(_rc)
