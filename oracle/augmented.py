"""Theorem 1 (Section 3.1, Eqs. (13)-(15), with the corrigendum's column order).

For A (N x N), vectors b_0..b_p and tau:
    B = [b_p, ..., b_2, b_1]  (N x p),
    K = p x p upper shift (ones on the first superdiagonal),
    A~ = [[A, B], [0, K]],   v = [b_0; e_p],
    w = e^{tau A~} v,   w(1:N) = sum_j tau^j phi_j(tau A) b_j,
    w(N+1:N+p) = [tau^{p-1}/(p-1)!, ..., tau, 1].

``phi_combination_dense`` is the exact result written out: the augmented
matrix assembled densely and exponentiated by ``oracle.expm`` (small N only).
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .expm import expm
from . import operators


def augmented_matrix(A: np.ndarray, vectors: Sequence[np.ndarray]):
    """Return (A~, v) of Eq. (13) for vectors = [b_0, ..., b_p]."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    p = len(vectors) - 1
    At = np.zeros((n + p, n + p))
    At[:n, :n] = A
    for c in range(p):
        At[:n, n + c] = vectors[p - c]          # column c of B is b_{p-c}
    for i in range(p - 1):
        At[n + i, n + i + 1] = 1.0              # K: upper shift
    v = np.zeros(n + p)
    v[:n] = vectors[0]
    if p > 0:
        v[n + p - 1] = 1.0                      # e_p
    return At, v


def phi_combination_dense(A: np.ndarray, tau: float, vectors: Sequence[np.ndarray],
                          full: bool = False) -> np.ndarray:
    """sum_j tau^j phi_j(tau A) b_j via Eq. (14); ``full`` returns all N+p entries."""
    At, v = augmented_matrix(A, vectors)
    w = expm(tau * At) @ v
    return w if full else w[: A.shape[0]]


def phi_combination_times(A: np.ndarray, times: Sequence[float], vectors: Sequence[np.ndarray],
                          task: int = 2) -> List[np.ndarray]:
    """Algorithm 1 with an array of output times T_1 < ... < T_n: the result at
    T_k is the first N entries of exp(T_k A~) v (Theorem 1, Eq. (14)); for
    Task I it is further multiplied by (1 / T_k)^p (Algorithm 1, the scaling
    after the time loop), which leaves phi_p(T_k A) b_p when only b_p is
    nonzero.  Dense, for small N."""
    p = len(vectors) - 1
    out = []
    for t in times:
        w = phi_combination_dense(A, t, vectors)
        out.append(w * (1.0 / t) ** p if task == 1 else w)
    return out


def phi_combination_dense_desc(desc, tau: float, vectors: Sequence[np.ndarray]) -> np.ndarray:
    return phi_combination_dense(operators.dense(desc), tau, vectors)


def trailing_entries(p: int, t: float) -> np.ndarray:
    """Eq. (15) / Eq. (47): [t^{p-1}/(p-1)!, ..., t, 1]."""
    out = np.empty(p)
    fact = 1.0
    for i in range(p):          # entry p-1-i holds t^i / i!
        if i > 0:
            fact *= i
        out[p - 1 - i] = t ** i / fact
    return out


def b_norm_scaling(vectors: Sequence[np.ndarray]):
    """Eqs. (48)-(49): nu = 2^{-ceil(log2 ||B||_1)}, mu = 1/nu, with ||B||_1 the
    largest absolute column sum of B = [b_p..b_1]; nu = mu = 1 when B is empty
    or zero."""
    p = len(vectors) - 1
    if p == 0:
        return 1.0, 1.0
    nb = max(float(np.sum(np.abs(vectors[k]))) for k in range(1, p + 1))
    if nb == 0.0:
        return 1.0, 1.0
    e = int(np.ceil(np.log2(nb)))
    return 2.0 ** (-e), 2.0 ** e


def exact_dense_list(A, tau, vectors) -> List[np.ndarray]:
    return [phi_combination_dense(A, tau, vectors)]
