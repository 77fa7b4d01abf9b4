"""Dense matrix exponential for the oracle.

The definition is the power series e^M = sum_k M^k / k!  (Eq. (32) in
Section 3.3.1 uses the same series).  Together with the semigroup property
e^M = (e^{M / 2^s})^{2^s} it gives a plainly correct algorithm:

  1. pick the smallest s >= 0 with ||M||_1 / 2^s <= 1/2;
  2. sum the series of X = M / 2^s until a term is below 2^-60 of the sum
     (at most 40 terms; the tail after a term t is below 2 ||t||_1 because
     ||X||_1 <= 1/2);
  3. square the result s times.

This is the scaling-and-squaring idea the paper uses for its small exponential
(Section 3.3.1) with the series itself in place of the diagonal Pade
approximant.  It is written independently of the device routine (which
evaluates a fixed-degree Taylor polynomial by Paterson-Stockmeyer with its own
scaling thresholds) and is pinned against closed forms and SciPy's Pade-based
expm in the tests.
"""

from __future__ import annotations

import math

import numpy as np


def expm(M: np.ndarray) -> np.ndarray:
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    if M.shape != (n, n):
        raise ValueError("square matrix expected")
    if n == 0:
        return M.copy()
    norm1 = float(np.max(np.sum(np.abs(M), axis=0)))
    if not math.isfinite(norm1):
        raise FloatingPointError("non-finite matrix")
    s = 0
    if norm1 > 0.5:
        s = int(math.ceil(math.log2(norm1 / 0.5)))
    X = M / (2.0 ** s)
    S = np.eye(n)
    T = np.eye(n)
    for k in range(1, 41):
        T = T @ X / k
        S = S + T
        if np.max(np.sum(np.abs(T), axis=0)) <= 2.0 ** -60 * max(1.0, np.max(np.sum(np.abs(S), axis=0))):
            break
    for _ in range(s):
        S = S @ S
    return S


def expm_apply(M: np.ndarray, v: np.ndarray) -> np.ndarray:
    """e^M v through the same series applied to the vector, with
    e^M v = (e^{M/s})^s v and ||M||_1 / s <= 1/2 (no squaring of matrices)."""
    M = np.asarray(M, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    norm1 = float(np.max(np.sum(np.abs(M), axis=0))) if M.size else 0.0
    steps = max(1, int(math.ceil(norm1 / 0.5)))
    X = M / steps
    out = v.copy()
    for _ in range(steps):
        term = out.copy()
        acc = out.copy()
        for k in range(1, 41):
            term = X @ term / k
            acc = acc + term
            if np.linalg.norm(term, 1) <= 2.0 ** -60 * max(1e-300, np.linalg.norm(acc, 1)):
                break
        out = acc
    return out
