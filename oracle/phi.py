"""Scalar phi-functions, Eq. (3) of Section 2:

    phi_0(z) = e^z,   phi_k(z) = int_0^1 e^{z(1-theta)} theta^{k-1}/(k-1)! dtheta  (k >= 1).

Two standard consequences of the definition are used, each valid for every
complex z:
  * the power series  phi_k(z) = sum_{i>=0} z^i / (i+k)!,
  * the recurrence    phi_{k+1}(z) = (phi_k(z) - 1/k!) / z   (z != 0).
The series is summed for |z| < max(1, k) (60 terms; for negative z its
cancellation costs at most a factor of about 2k); the recurrence, started
from e^z, is used for |z| >= max(1, k), where the step from order j to j+1
amplifies the relative error by at most (j+1)/|z| <= 1.
"""

from __future__ import annotations

import math

import numpy as np


def phi(k: int, z):
    """phi_k evaluated elementwise on a real or complex array (or scalar)."""
    if k < 0:
        raise ValueError("k must be >= 0")
    z = np.asarray(z)
    cplx = np.iscomplexobj(z)
    dt = np.complex128 if cplx else np.float64
    z = z.astype(dt)
    out = np.empty_like(z)
    small = np.abs(z) < max(1.0, float(k))
    if np.any(small):
        zs = z[small]
        # sum_{i>=0} z^i/(i+k)!; with |z| < max(1, k) the term ratio is below
        # |z|/(i+k) and 60 terms leave a tail under 1e-17 of the leading term
        term = np.full_like(zs, 1.0 / math.factorial(k))
        acc = term.copy()
        for i in range(1, 60):
            term = term * zs / (i + k)
            acc = acc + term
        out[small] = acc
    big = ~small
    if np.any(big):
        zb = z[big]
        val = np.exp(zb)
        for j in range(k):
            val = (val - 1.0 / math.factorial(j)) / zb
        out[big] = val
    return out


def phi_all(p: int, z):
    """[phi_0(z), ..., phi_p(z)] as a list of arrays."""
    return [phi(k, z) for k in range(p + 1)]
