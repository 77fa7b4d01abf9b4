"""Algorithm 1 (Task II) of Section 3.2, assembled from the oracle's parts.

    tau = T_end; m = max(m_min, min(m_init, m_max)); T_now = 0; w = b_0
    while T_now < T_end:
        start vector [w; mu y(T_now)], y(t) = [t^{p-1}/(p-1)!, ..., t, 1]   Alg. 1, Eq. (47)
        extend the IOP basis to m (Algorithm 2)
        F = exp(tau H~), H~ = [[H_j, e_1], [0, 0]]                        Eqs. (37)-(38)
        eps = beta |h_{j+1,j}| |F(j, j+1)|                                Eq. (36)
              (or a variant of Section 3.4, below)
        decision (Algorithm 4)
        accepted: w = beta V(1:N, 1:j) F(1:j, 1); T_now += tau             Alg. 3, Eq. (33)
        rejected: extend the basis (j < m_max) or shrink tau (j = m_max)

B is scaled by nu and the trailing entries by mu (Eqs. (48)-(49)).  This is
the paper's method, not the exact result: it serves to compare the device
controller's decisions (substeps, rejections, Krylov sizes) with the same
algorithm run on the CPU.  The exact result comes from ``augmented``,
``spectral`` or ``arnoldi``.

Error-estimate variants (Section 3.4; the error of Eq. (33) is the series
Eq. (35), whose first term is Eq. (36)):
  "one"        Eq. (36): beta |h| |a|,  a = tau e_j^T phi_1(tau H_j) e_1
  "two"        the first two terms of Eq. (35): beta |h| ||a v_{j+1} + b A~ v_{j+1}||,
               b = tau^2 e_j^T phi_2(tau H_j) e_1
  "corrected"  the corrected scheme named after Eq. (30): the result takes the
               first term, w += beta h a v_{j+1}(1:N), and eps is the second
               term alone, beta |h| |b| ||A~ v_{j+1}||
a and b are entries of exp(tau [[H_j, e_1, 0], [0, 0, 1], [0, 0, 0]]) (Theorem 1
applied to H_j); A~ v_{j+1} is one more product with the augmented matrix.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, List, Sequence

import numpy as np

from .augmented import b_norm_scaling, trailing_entries
from .controller import ControllerState, decide, record
from .expm import expm
from .iop import IOPBasis


@dataclasses.dataclass
class KiopsStats:
    substeps: int = 0
    rejections: int = 0
    matvecs: int = 0
    expms: int = 0
    breakdowns: int = 0
    m_last: int = 0
    last_omega: float = 0.0
    trace: List[tuple] = dataclasses.field(default_factory=list)


def kiops(apply_A: Callable[[np.ndarray], np.ndarray], T_end: float,
          vectors: Sequence[np.ndarray], tol: float = 1e-7, m_init: int = 10,
          m_min: int = 10, m_max: int = 128, q: int = 2,
          max_substeps: int = 100000, normalize_B: bool = True, estimate: str = "one"):
    vectors = [np.asarray(v, dtype=np.float64) for v in vectors]
    p = len(vectors) - 1
    st = KiopsStats()
    w = vectors[0].copy()
    if T_end == 0.0:
        return w, st
    nu, mu = b_norm_scaling(vectors) if normalize_B else (1.0, 1.0)
    Bcols = [vectors[p - c] for c in range(p)]
    cs = ControllerState(T_end=T_end, tol=tol, m_min=m_min, m_max=m_max)
    cs.tau = T_end
    cs.m = max(m_min, min(m_init, m_max))
    while cs.T_now < T_end:
        if st.substeps >= max_substeps:
            raise RuntimeError("substep limit reached")
        y0 = mu * trailing_entries(p, cs.T_now)
        basis = IOPBasis(apply_A, Bcols, nu, w, y0, q, m_max)
        if basis.beta == 0.0:
            w = np.zeros_like(w)
            break
        while True:
            before = basis.j
            basis.extend(cs.m)
            st.matvecs += basis.j - before
            j = basis.j
            extra = 0 if estimate == "one" else 1
            Ht = np.zeros((j + 1 + extra, j + 1 + extra))
            Ht[:j, :j] = basis.H[:j, :j]
            Ht[0, j] = 1.0
            if extra:
                Ht[j, j + 1] = 1.0
            F = expm(cs.tau * Ht)
            st.expms += 1
            h = basis.H[j, j - 1]
            a = F[j - 1, j]
            if basis.breakdown:
                eps = 0.0
            elif estimate == "one":
                eps = basis.beta * abs(h) * abs(a)
            else:
                b = F[j - 1, j + 1]
                Av = basis.apply_aug(basis.V[j])
                if estimate == "two":
                    eps = basis.beta * abs(h) * np.linalg.norm(a * basis.V[j] + b * Av)
                else:
                    eps = basis.beta * abs(h) * abs(b) * np.linalg.norm(Av)
            d = decide(cs, j, eps, basis.breakdown)
            record(cs, d, j, eps)
            st.last_omega = d.omega
            st.trace.append((st.substeps, j, cs.tau, d.omega, d.accept, d.branch))
            if d.accept:
                if basis.breakdown:
                    st.breakdowns += 1
                w = basis.beta * (basis.V[:j, :basis.N].T @ F[:j, 0])
                if estimate == "corrected" and not basis.breakdown:
                    w = w + basis.beta * h * a * basis.V[j, :basis.N]
                cs.T_now = cs.T_now + cs.tau
                if T_end - cs.T_now <= 8.0 * np.finfo(float).eps * T_end:
                    cs.T_now = T_end
                cs.tau = min(d.tau_new, T_end - cs.T_now)
                cs.m = d.m_new
                st.substeps += 1
                break
            st.rejections += 1
            if j == m_max:
                cs.tau = d.tau_new
            else:
                cs.m = d.m_new
    st.m_last = cs.m
    return w, st
