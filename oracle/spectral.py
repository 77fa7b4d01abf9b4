"""Exact result for constant-coefficient periodic stencils.

With constant diffusivity (``diff``, or a constant ``kappa`` field), constant
advection and a constant reaction r0, the operator is diagonalised by the
discrete Fourier transform.  In numpy's convention a shift u_{i+1} multiplies
mode k by e^{+i theta}, theta = 2 pi k / n, so along each axis

    (u_{i+1} - 2 u_i + u_{i-1}) / h^2   ->  -4 sin^2(theta/2) / h^2
    (u_{i+1} - u_{i-1}) / (2 h)         ->   i sin(theta) / h

and the definition (Eq. (4)) is applied mode by mode:
    w^ = sum_j tau^j phi_j(tau lambda) b_j^.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np

from .phi import phi


def _constant_fields(desc):
    if desc.kappa is None:
        kap = float(desc.diff)
    else:
        k = np.asarray(desc.kappa)
        kap = float(k.flat[0])
        if not np.all(k == kap):
            raise ValueError("kappa must be constant for the spectral oracle")
    if desc.reaction is None:
        r0 = 0.0
    else:
        r = np.asarray(desc.reaction)
        r0 = float(r.flat[0])
        if not np.all(r == r0):
            raise ValueError("reaction must be constant for the spectral oracle")
    return kap, r0


def eigenvalues(desc) -> np.ndarray:
    """lambda on the [z, y, x] DFT grid."""
    kap, r0 = _constant_fields(desc)
    lam = np.full((desc.nz, desc.ny, desc.nx), complex(r0))
    for axis, size, a in ((2, desc.nx, desc.adv[0]), (1, desc.ny, desc.adv[1]),
                          (0, desc.nz, desc.adv[2])):
        if size == 1:
            continue
        theta = 2.0 * np.pi * np.arange(size) / size
        contrib = -4.0 * kap * np.sin(theta / 2.0) ** 2 / desc.h ** 2 - 1j * a * np.sin(theta) / desc.h
        sh = [1, 1, 1]
        sh[axis] = size
        lam = lam + contrib.reshape(sh)
    return lam


def phi_combination_fft(desc, tau: float, vectors: Sequence[np.ndarray]) -> np.ndarray:
    shape = (desc.nz, desc.ny, desc.nx)
    z = tau * eigenvalues(desc)
    acc = np.zeros(shape, dtype=np.complex128)
    for j, b in enumerate(vectors):
        bh = np.fft.fftn(np.asarray(b, dtype=np.float64).reshape(shape))
        acc += (tau ** j) * phi(j, z) * bh
        del bh
    return np.real(np.fft.ifftn(acc)).reshape(-1)
