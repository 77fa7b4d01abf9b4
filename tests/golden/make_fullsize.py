"""Write the sampled oracle results of the full-size workloads (tests/golden/fullsize_*.npz).

The full-size GPU parity tests compare the device result with the exact
phi-combination on a fixed sample of entries.  The exact results at these
sizes take the oracle minutes to hours, so they are computed once, here, by
the oracle alone (``oracle/``; the inputs come from the seeded generators of
``workloads/``, which hold none of the method's arithmetic), and only a
sample of entries is stored:

  idx     sorted entry indices, drawn from PCG64(SAMPLE_SEED) without replacement
  val     the oracle result at idx
  norm2   the 2-norm of the whole oracle result
  route, params, stats   how it was computed (JSON text)

Cases (name -> workload, route):
  cfg3_256       3-D variable-coefficient diffusion-reaction, 256^3, kappa a
                 box-averaged exp(N(0, 0.5^2)) field, r ~ U[-5, 0], p = 2,
                 tau = 1e-3, seed 1003: per-term Lanczos (A is symmetric),
                 m grown until successive results agree to 1e-13.
  cfg2_2048_t3   2-D ADR 2048^2 with the per-cell reaction field of the
                 benchmark (seed 1002), p = 3, tau = 1e-3: full-Arnoldi
                 Krylov, m = 64, tol_o = 1e-11 (absolute, as in Eq. (36)).
  cfg2_2048_t25  the same at tau = 10^-2.5.

Usage: python tests/golden/make_fullsize.py [case ...]   (default: all)
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import operators  # noqa: E402
from oracle.arnoldi import phi_combination_arnoldi  # noqa: E402
from oracle.lanczos import phi_combination_lanczos  # noqa: E402

SAMPLE_SEED = 20180414
SAMPLES = 16384


def sample_indices(n: int) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return np.sort(g.choice(n, size=min(SAMPLES, n), replace=False)).astype(np.int64)


def log(msg):
    print(f"[golden] {msg}", flush=True)


def case_cfg3_256():
    pr = W.cfg3()
    M = operators.stencil_sparse(pr.op)       # the same operator as stencil_apply (pinned in the tests)
    st = {}
    w = phi_combination_lanczos(lambda v: M @ v, pr.tau, pr.vectors, rtol=1e-13, stats=st, log=log)
    return pr, w, "lanczos", {"rtol": 1e-13}, st


def _cfg2_arnoldi(tau):
    pr = W.cfg2(2048, tau)
    st = {}
    w = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-11, m=64,
                                stats=st)
    return pr, w, "arnoldi", {"tol_o": 1e-11, "m": 64}, st


CASES = {
    "cfg3_256": case_cfg3_256,
    "cfg2_2048_t3": lambda: _cfg2_arnoldi(1e-3),
    "cfg2_2048_t25": lambda: _cfg2_arnoldi(10.0 ** -2.5),
}


def main(names):
    for name in names or list(CASES):
        t0 = time.time()
        log(f"{name}: start")
        pr, w, route, params, st = CASES[name]()
        idx = sample_indices(pr.n)
        meta = {"case": name, "route": route, "params": params, "stats": st, "n": pr.n, "p": pr.p,
                "tau": pr.tau, "seed": pr.seed, "seconds": time.time() - t0}
        out = os.path.join(HERE, f"fullsize_{name}.npz")
        np.savez(out, idx=idx, val=w[idx], norm2=np.float64(np.linalg.norm(w)),
                 meta=np.array(json.dumps(meta, default=str)))
        log(f"{name}: wrote {out} in {meta['seconds']:.0f} s ({json.dumps(st, default=str)[:200]})")


if __name__ == "__main__":
    main(sys.argv[1:])
