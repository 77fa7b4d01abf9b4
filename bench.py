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
    ap.add_argument("--precision", type=str, default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-substeps", type=int, default=2)
    ap.add_argument("--traffic-json", type=str, default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, run one plain device copy of MIB MiB (a known-size "
                         "kernel that HBM traffic counters are scaled by)")
    return ap.parse_args()


def cpu_baseline(pr_sample, sweep_taus, substeps):
    """Time the oracle's exact-result route (full-Arnoldi Krylov, oracle/arnoldi.py)
    on the first `substeps` substeps of the smallest-tau solve of the same
    2048^2 problem, and extrapolate to the sweep: the substepped Krylov cost
    grows about linearly with tau, so a sweep costs sum(tau)/tau_sample times
    one solve, and one solve costs elapsed * tau_sample / t_reached."""
    import numpy as np  # noqa: F401
    from oracle import operators
    from oracle.arnoldi import phi_combination_arnoldi
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    ap = operators.make_apply(pr_sample.op)
    st = {}
    t0 = time.perf_counter()
    phi_combination_arnoldi(ap, pr_sample.tau, pr_sample.vectors, tol_o=1e-3 * pr_sample.tol, m=48,
                            stats=st, stop_after=substeps)
    el = time.perf_counter() - t0
    frac = st["t"] / pr_sample.tau
    t_solve = el / max(frac, 1e-300)
    t_sweep = t_solve * sum(sweep_taus) / pr_sample.tau
    return {
        "value": len(sweep_taus) / t_sweep,
        "unit": "solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"oracle full-Arnoldi route (m=48, CGS2, tol_o=1e-11) on the 2048^2 problem at "
                   f"tau={pr_sample.tau:g}: {st['substeps']} substeps, {st['matvecs']} products, "
                   f"{el:.1f} s covering t={st['t']:.3g} of {pr_sample.tau:g}; extrapolated "
                   f"linearly in tau to the 5-value sweep"),
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(instances shard by GPU with no exchange; see the design notes).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    import paper_1804_05126_amd as K

    taus = [float(t) for t in args.taus.split(",")] if args.taus else W.cfg2_tau_grid()
    side = args.side
    pr = W.cfg2(side, taus[0], q=args.q)       # operator and vectors shared by the sweep
    dev = torch.device("cuda:0")
    op = K.Operator.from_desc(pr.op, precision=args.precision)
    vecs = [torch.as_tensor(v, device=dev) for v in pr.vectors]
    w = torch.empty(pr.n, dtype=torch.float64, device=dev)
    tol = 1e-8 if args.precision == "fp64" else 1e-6
    stream = torch.cuda.current_stream()

    def one_solve(tau):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        _, st, _ = K.phi_combination(op, tau, vecs, tol=tol, m_init=10, q=args.q, out=w)
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
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            if tj.get("workload_side") == side and tj.get("kernel_source_hash") == _kernel_hash():
                traffic = tj.get("hbm_bytes_per_launch")
        except Exception:
            traffic = None
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
                         f"m_init=10, m_max=128"),
            "solves_per_step": len(taus),
            "precision": args.precision,
            "seed": pr.seed,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "kiops_solve_kernel<Stencil2D<double>, double> (one persistent launch per solve)",
            "algorithmic_bytes_per_launch": total_bytes / n_solves,
            "avg_launch_ms": total_ms / n_solves,
        },
        "latency_ms": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]},
        "matvecs_per_s": sum(st["matvecs"] for *_, st in records) / wall,
        "per_tau": per_tau,
    }
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)      # elementwise kernel: reads and writes nbytes
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
        del src, dst
    if not args.no_cpu_baseline:
        sample = W.cfg2(side, taus[0], q=args.q)
        out["cpu_baseline"] = cpu_baseline(sample, taus, args.cpu_sample_substeps)
    print(json.dumps(out), flush=True)


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1804_05126_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
