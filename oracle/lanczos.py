"""Exact-to-tolerance result for symmetric A: one Lanczos process per term.

Test infrastructure only (see the package docstring).

By the definition of the phi-combination (Eq. (4)),

    w = sum_k tau^k phi_k(tau A) b_k,

and for a symmetric A every term can be computed on its own, with no use of
the augmented matrix of Theorem 1: so this route also checks Theorem 1 (the
KIOPS path, the dense route and the Arnoldi route all go through Eq. (14)).

For one term, the Arnoldi process of Section 3.2 applied to a symmetric A
gives a symmetric tridiagonal H (the Lanczos recurrence): with
q_1 = b / ||b||,

    beta_j q_{j+1} = A q_j - alpha_j q_j - beta_{j-1} q_{j-1},
    alpha_j = <q_j, A q_j>,  beta_j = ||A q_j - alpha_j q_j - beta_{j-1} q_{j-1}||,

and phi_k(tau A) b ~= ||b|| Q_m phi_k(tau T_m) e_1 (the projection of Eq. (33)
for a single vector), where T_m is tridiagonal with diagonal alpha and
off-diagonal beta.  phi_k(tau T_m) e_1 = S phi_k(tau Lambda) S^T e_1 from the
symmetric eigendecomposition T_m = S Lambda S^T and the scalar phi_k of
``oracle.phi``.

m grows until two successive coefficient vectors (checked every
``check_every`` steps) agree to ``rtol`` relative; the basis is not stored:
a first run of the recurrence finds alpha, beta and m, a second run rebuilds
q_1..q_m from the recorded alpha, beta and accumulates Q_m y.  No
reorthogonalisation (plain Lanczos): the convergence test is on the
projected result, and the route is pinned against the dense, DFT and Arnoldi
results in the tests.
"""

from __future__ import annotations

from typing import Callable, Sequence

import numpy as np

from .phi import phi


def _coefficients(alpha, beta, k: int, tau: float, bnorm: float) -> np.ndarray:
    """y = ||b|| tau^k phi_k(tau T) e_1 for the tridiagonal T(alpha, beta)."""
    m = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=np.float64))
    if m > 1:
        off = np.asarray(beta[: m - 1], dtype=np.float64)
        T += np.diag(off, 1) + np.diag(off, -1)
    lam, S = np.linalg.eigh(T)
    f = np.real(phi(k, tau * lam))
    return bnorm * (tau ** k) * (S @ (f * S[0, :]))


def phi_term_lanczos(apply_A: Callable[[np.ndarray], np.ndarray], tau: float, k: int,
                     b: np.ndarray, rtol: float = 1e-13, m_max: int = 2000,
                     check_every: int = 10, stats: dict = None) -> np.ndarray:
    """tau^k phi_k(tau A) b for symmetric A (``apply_A``: x -> A x)."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if tau == 0.0:                     # phi_0(0) = 1; tau^k = 0 for k >= 1
        return b.copy() if k == 0 else np.zeros_like(b)
    if bnorm == 0.0:
        return np.zeros_like(b)
    # ---- first run: alpha, beta and the dimension m
    alpha, beta = [], []
    q_prev = np.zeros_like(b)
    q = b / bnorm
    y_old = None
    agreed = 0
    m = 0
    matvecs = 0
    invariant = False
    while True:
        z = apply_A(q)
        matvecs += 1
        znorm = float(np.linalg.norm(z))
        a = float(np.dot(q, z))
        z -= a * q
        if beta:
            z -= beta[-1] * q_prev
        bt = float(np.linalg.norm(z))
        alpha.append(a)
        m += 1
        if bt <= 1e-13 * znorm:
            invariant = True          # the Krylov space is invariant: T_m is exact
            break
        beta.append(bt)
        if m % check_every == 0:
            y = _coefficients(alpha, beta, k, tau, bnorm)
            if y_old is not None:
                ypad = np.zeros(m)
                ypad[: y_old.size] = y_old
                if np.linalg.norm(y - ypad) <= rtol * np.linalg.norm(y):
                    agreed += 1
                else:
                    agreed = 0
                if agreed >= 2:
                    break
            y_old = y
        if m >= m_max:
            raise RuntimeError("oracle Lanczos: no convergence within m_max steps")
        q_prev, q = q, z / bt
    y = _coefficients(alpha, beta, k, tau, bnorm)
    # ---- second run: rebuild q_1..q_m from the recorded recurrence, accumulate Q y
    out = y[0] * (b / bnorm)
    q_prev = np.zeros_like(b)
    q = b / bnorm
    for j in range(m - 1):
        z = apply_A(q)
        matvecs += 1
        z -= alpha[j] * q
        if j > 0:
            z -= beta[j - 1] * q_prev
        q_prev, q = q, z / beta[j]
        out += y[j + 1] * q
    if stats is not None:
        stats.update(m=m, matvecs=matvecs, invariant=invariant)
    return out


def phi_combination_lanczos(apply_A: Callable[[np.ndarray], np.ndarray], tau: float,
                            vectors: Sequence[np.ndarray], rtol: float = 1e-13,
                            stats: dict = None, log=None) -> np.ndarray:
    """sum_k tau^k phi_k(tau A) b_k (Eq. (4)) for symmetric A, term by term."""
    vectors = [np.asarray(v, dtype=np.float64) for v in vectors]
    w = np.zeros_like(vectors[0])
    per_term = []
    for k, b in enumerate(vectors):
        st = {}
        w += phi_term_lanczos(apply_A, tau, k, b, rtol=rtol, stats=st)
        per_term.append(st)
        if log is not None:
            log(f"lanczos term k={k}: m={st.get('m')} matvecs={st.get('matvecs')}")
    if stats is not None:
        stats["terms"] = per_term
    return w
