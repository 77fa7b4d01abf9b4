"""Seeded input generators for the φ-combination workloads.

Everything here is data: operator descriptions (grid sizes, spacing, constant
coefficients, per-cell coefficient fields) and the vectors b_0..b_p, all drawn
from ``numpy.random.Generator(PCG64(seed))``.  The draw order is fixed: the
scalar parameters of an instance, then its coefficient fields, then
v_0..v_p, then tau (when tau is drawn at all).

Operator family (the linear part of the paper's 2-D advection-diffusion-
reaction test problem, Section 4, made periodic and with a per-cell reaction
field in place of the reaction Jacobian):

    (A u)_i = sum_d [ (kf_{i,d+} (u_{i+e_d} - u_i) - kf_{i,d-} (u_i - u_{i-e_d})) / h^2
                      - a_d (u_{i+e_d} - u_{i-e_d}) / (2 h) ] + r_i u_i

on a periodic nx*ny*nz box with x the fastest index.  The face diffusivity
kf is the constant ``diff`` when ``kappa`` is None, otherwise the arithmetic
mean of the two cells' ``kappa`` values.  A 2-D problem is the case nz = 1.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class StencilDesc:
    """Periodic 5-point (nz == 1) or 7-point stencil operator, as data."""

    nx: int
    ny: int
    nz: int = 1
    h: float = 1.0
    diff: float = 0.0
    kappa: Optional[np.ndarray] = None      # per-cell diffusivity, float64[N]
    adv: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    reaction: Optional[np.ndarray] = None   # per-cell reaction r, float64[N]
    # general form: per-cell weights [5|7][N] of the points (centre, +x, -x,
    # +y, -y[, +z, -z]); the coefficient fields above are then unused
    weights: Optional[np.ndarray] = None

    @property
    def kind(self) -> str:
        return "stencil2d" if self.nz == 1 else "stencil3d"

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class CsrDesc:
    """General sparse matrix in CSR form (0-based, int32 indices)."""

    n: int
    rowptr: np.ndarray   # int32[n + 1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]

    kind = "csr"

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


@dataclasses.dataclass
class Problem:
    """One φ-combination request: w = sum_k tau^k phi_k(tau A) b_k."""

    name: str
    op: object                   # StencilDesc or CsrDesc
    tau: float
    vectors: List[np.ndarray]    # [b_0, ..., b_p], float64[N] each
    tol: float = 1e-8
    q: int = 2
    m_init: int = 10
    seed: int = 0
    precision: str = "fp64"      # "fp64" or "mixed"

    @property
    def p(self) -> int:
        return len(self.vectors) - 1

    @property
    def n(self) -> int:
        return self.op.n


def adr2d_problem(side: int, p: int, tau: float, seed: int, *, diff: float = 1e-2,
                  adv: float = 10.0, r_range: Tuple[float, float] = (-1.0, 0.0),
                  tol: float = 1e-8, q: int = 2, m_init: int = 10,
                  constant_reaction: Optional[float] = None,
                  name: Optional[str] = None, precision: str = "fp64") -> Problem:
    """2-D ADR operator diff*L5 - adv*(Dx + Dy) + diag(r) on a side x side
    periodic grid with h = 1/side, r ~ U[r_range] per cell (or a constant
    when ``constant_reaction`` is given), vectors ~ N(0, 1)."""
    g = _rng(seed)
    n = side * side
    if constant_reaction is None:
        r = g.uniform(r_range[0], r_range[1], size=n)
    else:
        r = np.full(n, float(constant_reaction))
    vecs = [g.standard_normal(n) for _ in range(p + 1)]
    op = StencilDesc(nx=side, ny=side, nz=1, h=1.0 / side, diff=diff,
                     adv=(adv, adv, 0.0), reaction=r)
    return Problem(name=name or f"adr2d_{side}_p{p}", op=op, tau=tau, vectors=vecs,
                   tol=tol, q=q, m_init=m_init, seed=seed, precision=precision)


def cfg1(seed: int = 1001) -> Problem:
    """32x32 periodic ADR, h = 1/32, A = 1e-2 L5 - 10 (Dx+Dy) + diag(r),
    r ~ U[-1,0], p = 2, tau = 1e-2, tol 1e-8, q = 2, m_init = 10."""
    return adr2d_problem(32, 2, 1e-2, seed, name="cfg1_adr2d_32")


def cfg2_tau_grid() -> List[float]:
    """Five log-uniformly spaced step sizes over [1e-3, 1e-1]."""
    return [10.0 ** e for e in (-3.0, -2.5, -2.0, -1.5, -1.0)]


def cfg2(side: int, tau: float, seed: int = 1002, q: int = 2, **kw) -> Problem:
    """Same ADR operator at side^2 (512^2 or 2048^2), p = 3, FP64, tol 1e-8."""
    return adr2d_problem(side, 3, tau, seed, q=q, name=f"cfg2_adr2d_{side}_tau{tau:.3g}", **kw)


def _box_average7(f: np.ndarray) -> np.ndarray:
    """Mean of a cell and its six face neighbours on a periodic 3-D box
    (array indexed [z, y, x])."""
    s = f.copy()
    for ax in range(3):
        s += np.roll(f, 1, axis=ax) + np.roll(f, -1, axis=ax)
    return s / 7.0


def diffusion3d_problem(side: int, p: int, tau: float, seed: int, *,
                        log_sigma: float = 0.5, r_range=(-5.0, 0.0), tol: float = 1e-6,
                        q: int = 2, m_init: int = 10, constant: Optional[Tuple[float, float]] = None,
                        name: Optional[str] = None, precision: str = "fp64") -> Problem:
    """3-D variable-coefficient diffusion-reaction on a side^3 periodic box,
    h = 1/side: kappa = 7-point periodic box average of exp(g), g ~ N(0, sigma^2)
    per cell; r ~ U[r_range]; vectors ~ N(0,1).  ``constant=(kappa0, r0)``
    replaces both fields by constants (used for closed-form checks)."""
    g = _rng(seed)
    shape = (side, side, side)
    if constant is None:
        kap = _box_average7(np.exp(g.normal(0.0, log_sigma, size=shape))).reshape(-1)
        r = g.uniform(r_range[0], r_range[1], size=side ** 3)
    else:
        kap = np.full(side ** 3, float(constant[0]))
        r = np.full(side ** 3, float(constant[1]))
    vecs = [g.standard_normal(side ** 3) for _ in range(p + 1)]
    op = StencilDesc(nx=side, ny=side, nz=side, h=1.0 / side, diff=0.0, kappa=kap,
                     adv=(0.0, 0.0, 0.0), reaction=r)
    return Problem(name=name or f"diff3d_{side}_p{p}", op=op, tau=tau, vectors=vecs,
                   tol=tol, q=q, m_init=m_init, seed=seed, precision=precision)


def cfg3(side: int = 256, seed: int = 1003, precision: str = "fp64") -> Problem:
    """256^3 variable-coefficient diffusion-reaction, p = 2, tau = 1e-3, tol 1e-6."""
    return diffusion3d_problem(side, 2, 1e-3, seed, name=f"cfg3_diff3d_{side}",
                               precision=precision)


def _log_uniform(g: np.random.Generator, lo: float, hi: float) -> float:
    return float(math.exp(g.uniform(math.log(lo), math.log(hi))))


def cfg4(count: int = 256, seed: int = 1004, precision: str = "fp64",
         side_range=(64, 512)) -> List[Problem]:
    """Batch of independent 2-D ADR instances: side log-uniform in side_range,
    eps ~ U[1e-3, 1e-1], alpha ~ U[-20, 20] (applied as -alpha (Dx + Dy)),
    r ~ U[-1, 0], p ~ U{1..4}, tau ~ log-U[1e-4, 1e-1].  tol is 1e-8 for FP64
    and 1e-6 for the mixed form."""
    g = _rng(seed)
    tol = 1e-8 if precision == "fp64" else 1e-6
    out = []
    for i in range(count):
        side = int(round(_log_uniform(g, side_range[0], side_range[1])))
        eps = float(g.uniform(1e-3, 1e-1))
        alpha = float(g.uniform(-20.0, 20.0))
        p = int(g.integers(1, 5))
        n = side * side
        r = g.uniform(-1.0, 0.0, size=n)
        vecs = [g.standard_normal(n) for _ in range(p + 1)]
        tau = _log_uniform(g, 1e-4, 1e-1)
        op = StencilDesc(nx=side, ny=side, nz=1, h=1.0 / side, diff=eps,
                         adv=(alpha, alpha, 0.0), reaction=r)
        out.append(Problem(name=f"cfg4_{i}_adr2d_{side}_p{p}", op=op, tau=tau, vectors=vecs,
                           tol=tol, seed=seed, precision=precision))
    return out


@dataclasses.dataclass
class Request:
    """One arrival of the served workload.  Arrays are drawn lazily from
    ``seed`` so that a long arrival stream does not sit in host memory."""

    index: int
    arrival_s: float
    kind: str          # "2d" or "3d"
    side: int
    p: int
    tau: float
    precision: str     # "fp64" (tol 1e-8) or "mixed" (tol 1e-6)
    seed: int

    @property
    def tol(self) -> float:
        return 1e-8 if self.precision == "fp64" else 1e-6

    @property
    def n(self) -> int:
        return self.side ** (2 if self.kind == "2d" else 3)

    def materialize(self) -> Problem:
        if self.kind == "2d":
            g = _rng(self.seed)
            eps = float(g.uniform(1e-3, 1e-1))
            alpha = float(g.uniform(-20.0, 20.0))
            n = self.side * self.side
            r = g.uniform(-1.0, 0.0, size=n)
            vecs = [g.standard_normal(n) for _ in range(self.p + 1)]
            op = StencilDesc(nx=self.side, ny=self.side, nz=1, h=1.0 / self.side, diff=eps,
                             adv=(alpha, alpha, 0.0), reaction=r)
            return Problem(name=f"req{self.index}_2d_{self.side}", op=op, tau=self.tau,
                           vectors=vecs, tol=self.tol, seed=self.seed, precision=self.precision)
        return diffusion3d_problem(self.side, self.p, self.tau, self.seed, tol=self.tol,
                                   name=f"req{self.index}_3d_{self.side}",
                                   precision=self.precision)


def cfg5_requests(lam: float, count: int, seed: int = 1005,
                  side2d=(64, 2048), side3d=(32, 192)) -> List[Request]:
    """Poisson arrival stream with rate ``lam`` per second: half 2-D 5-point
    ADR (side log-uniform in side2d), half 3-D 7-point diffusion-reaction
    (side log-uniform in side3d); p ~ U{1..4}; tau ~ log-U[1e-4, 1e-1];
    precision class 50/50 between mixed (tol 1e-6) and FP64 (tol 1e-8)."""
    g = _rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(g.exponential(1.0 / lam))
        kind = "2d" if g.uniform() < 0.5 else "3d"
        lo, hi = side2d if kind == "2d" else side3d
        side = int(round(_log_uniform(g, lo, hi)))
        p = int(g.integers(1, 5))
        tau = _log_uniform(g, 1e-4, 1e-1)
        precision = "mixed" if g.uniform() < 0.5 else "fp64"
        sub_seed = int(g.integers(0, 2 ** 31 - 1))
        out.append(Request(index=i, arrival_s=t, kind=kind, side=side, p=p, tau=tau,
                           precision=precision, seed=sub_seed))
    return out


def csr_from_random_pattern(n: int, per_row: int, band: int, seed: int,
                            diag_shift: float = -4.0) -> CsrDesc:
    """Random sparse matrix: each row holds its diagonal plus ``per_row``
    distinct off-diagonal columns drawn within +-band (periodic), values
    N(0,1), diagonal N(0,1) + diag_shift."""
    g = _rng(seed)
    rows_cols = []
    rows_vals = []
    for i in range(n):
        offs = g.choice(np.arange(1, 2 * band + 1), size=min(per_row, 2 * band), replace=False)
        cols = np.unique(np.concatenate(([i], (i + offs - band) % n)))
        vals = g.standard_normal(cols.size)
        vals[cols == i] += diag_shift
        rows_cols.append(cols.astype(np.int32))
        rows_vals.append(vals)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum([c.size for c in rows_cols])
    return CsrDesc(n=n, rowptr=rowptr, col=np.concatenate(rows_cols),
                   val=np.concatenate(rows_vals))


def random_vectors(n: int, p: int, seed: int) -> List[np.ndarray]:
    g = _rng(seed)
    return [g.standard_normal(n) for _ in range(p + 1)]


def pick(seq: Sequence, idx: Sequence[int]) -> list:
    return [seq[i] for i in idx]
