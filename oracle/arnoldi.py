"""Exact-to-tolerance result for large N: full-Arnoldi Krylov on A~.

The result is e^{T A~} [b_0; e_p] restricted to its first N entries
(Theorem 1), advanced in substeps (Eqs. (23)-(28)) with a fixed Krylov
dimension m and a fully orthonormal basis (classical Gram-Schmidt applied
twice).  Per substep of length dt:

    start vector [w; y(t)], y(t) = [t^{p-1}/(p-1)!, ..., t, 1]     (Eq. (47): the
                                                                  trailing entries are exact)
    A~ V_m = V_m H_m + h_{m+1,m} v_{m+1} e_m^T                    (Eq. (30), full Arnoldi)
    F = exp(dt H~), H~ = [[H_m, e_1], [0, 0]]                     (Eqs. (37)-(38))
    err = beta |h_{m+1,m}| |F(m, m+1)|                            (Eq. (36))
    accept when err <= tol_o dt / T, else halve dt (same basis)
    w = beta V_m(1:N, :) F(1:m, 1)                                (Eq. (33))

Deliberately simpler than KIOPS: no IOP, no normalisation of B, no
adaptivity of m, conservative step control (halve on failure, grow by 1.5
after success).  It is checked against the dense and DFT results.
"""

from __future__ import annotations

from typing import Callable, Sequence

import numpy as np

from .augmented import trailing_entries
from .expm import expm


def arnoldi_basis(apply_aug: Callable[[np.ndarray], np.ndarray], v1: np.ndarray, m: int):
    """m steps of the Arnoldi process from the unit vector v1, each new vector
    orthogonalised against all earlier ones by classical Gram-Schmidt applied
    twice.  Returns (V (m+1, n), H (m+1, m), k, happy): k steps were made; happy
    when the process broke down (the new vector vanished)."""
    n = v1.size
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    V[0] = v1
    for j in range(m):
        z = apply_aug(V[j])
        pre = float(np.linalg.norm(z))
        h = V[: j + 1] @ z
        z = z - V[: j + 1].T @ h
        h2 = V[: j + 1] @ z           # second pass of classical Gram-Schmidt
        z = z - V[: j + 1].T @ h2
        H[: j + 1, j] = h + h2
        s = float(np.linalg.norm(z))
        if s <= 1e-13 * pre:
            return V, H, j + 1, True
        H[j + 1, j] = s
        V[j + 1] = z / s
    return V, H, m, False


def phi_combination_arnoldi(apply_A: Callable[[np.ndarray], np.ndarray], T: float,
                            vectors: Sequence[np.ndarray], tol_o: float = 1e-12,
                            m: int = 48, max_substeps: int = 100000, stats: dict = None,
                            stop_after: int = 0) -> np.ndarray:
    """``stop_after`` > 0 ends the run after that many substeps (a partial
    result for timing samples); ``stats`` receives substeps, matvecs and the
    time t reached."""
    vectors = [np.asarray(v, dtype=np.float64) for v in vectors]
    p = len(vectors) - 1
    N = vectors[0].size
    Bcols = [vectors[p - c] for c in range(p)]     # B = [b_p, ..., b_1]
    w = vectors[0].copy()
    if T == 0.0:
        return w
    t = 0.0
    dt = T
    substeps = 0
    matvecs = 0

    def apply_aug(v):
        x, y = v[:N], v[N:]
        out = np.empty(N + p)
        ax = apply_A(x)
        for c in range(p):
            ax = ax + y[c] * Bcols[c]
        out[:N] = ax
        if p > 0:
            out[N:N + p - 1] = y[1:]
            out[N + p - 1] = 0.0
        return out

    while t < T:
        substeps += 1
        if substeps > max_substeps:
            raise RuntimeError("oracle Arnoldi: substep limit")
        v0 = np.concatenate([w, trailing_entries(p, t)])
        beta = float(np.linalg.norm(v0))
        if beta == 0.0:
            return np.zeros(N)
        V, H, k, happy = arnoldi_basis(apply_aug, v0 / beta, m)
        matvecs += k
        Ht = np.zeros((k + 1, k + 1))
        Ht[:k, :k] = H[:k, :k]
        Ht[0, k] = 1.0
        dt = min(dt, T - t)
        while True:
            F = expm(dt * Ht)
            err = 0.0 if happy else beta * abs(H[k, k - 1]) * abs(F[k - 1, k])
            if err <= tol_o * dt / T:
                break
            dt *= 0.5
            if dt < 1e-300:
                raise RuntimeError("oracle Arnoldi: step underflow")
        w = beta * (V[:k, :N].T @ F[:k, 0])
        t = t + dt
        if T - t <= 8.0 * np.finfo(float).eps * T:
            t = T
        dt = 1.5 * dt
        if stop_after and substeps >= stop_after:
            break
    if stats is not None:
        stats.update(substeps=substeps, matvecs=matvecs, t=t)
    return w
