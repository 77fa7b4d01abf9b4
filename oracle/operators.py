"""Operators of the workloads, applied and assembled from their data.

The paper treats A as an external matrix-vector routine (Section 3.3, after
Algorithm 2).  The workloads use the linear part of the 2-D
advection-diffusion-reaction problem of Section 4 (standard second-order
differences, made periodic) and a 3-D variable-coefficient analogue:

    (A u)_i = sum_d [ (kf_{i,d+} (u_{i+e_d} - u_i) - kf_{i,d-} (u_i - u_{i-e_d})) / h^2
                      - a_d (u_{i+e_d} - u_{i-e_d}) / (2 h) ] + r_i u_i,

kf = the constant ``diff``, or the mean of the two cells' kappa.  Arrays are
flattened with x fastest (index = x + nx (y + ny z)).

General form (per-cell weights, the operator given by its stencil rows):
    (A u)_i = W_0[i] u_i + W_1[i] u_{i+e_x} + W_2[i] u_{i-e_x} + W_3[i] u_{i+e_y}
              + W_4[i] u_{i-e_y} [+ W_5[i] u_{i+e_z} + W_6[i] u_{i-e_z}]  (periodic)
with 5 weights per cell in 2-D (nz = 1) and 7 in 3-D.

``stencil_apply`` uses whole-array shifts; ``stencil_sparse`` builds the same
matrix entry by entry.  The two are written separately so each checks the other.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _axes(desc):
    # (array axis of the [z, y, x] view, size along it, advection coefficient)
    return ((2, desc.nx, desc.adv[0]), (1, desc.ny, desc.adv[1]), (0, desc.nz, desc.adv[2]))


def _weights(desc):
    w = getattr(desc, "weights", None)
    if w is None:
        return None
    return np.asarray(w, dtype=np.float64).reshape(-1, desc.nx * desc.ny * desc.nz)


def stencil_apply(desc, u: np.ndarray) -> np.ndarray:
    shape = (desc.nz, desc.ny, desc.nx)
    U = np.asarray(u, dtype=np.float64).reshape(shape)
    Wt = _weights(desc)
    if Wt is not None:
        out = Wt[0].reshape(shape) * U
        for s, (axis, _, _) in enumerate(_axes(desc)[: (Wt.shape[0] - 1) // 2]):
            out = out + Wt[1 + 2 * s].reshape(shape) * np.roll(U, -1, axis=axis)   # u_{i+e_d}
            out = out + Wt[2 + 2 * s].reshape(shape) * np.roll(U, 1, axis=axis)    # u_{i-e_d}
        return out.reshape(-1)
    if desc.reaction is not None:
        out = np.asarray(desc.reaction, dtype=np.float64).reshape(shape) * U
    else:
        out = np.zeros(shape)
    K = None if desc.kappa is None else np.asarray(desc.kappa, dtype=np.float64).reshape(shape)
    h2 = desc.h * desc.h
    for axis, size, a in _axes(desc):
        if size == 1:
            continue  # the neighbour is the cell itself: both differences vanish
        up = np.roll(U, -1, axis=axis)   # u_{i+e_d}
        dn = np.roll(U, 1, axis=axis)    # u_{i-e_d}
        if K is None:
            kp = km = desc.diff
        else:
            kp = 0.5 * (K + np.roll(K, -1, axis=axis))
            km = 0.5 * (K + np.roll(K, 1, axis=axis))
        out = out + (kp * (up - U) - km * (U - dn)) / h2
        if a != 0.0:
            out = out - a * (up - dn) / (2.0 * desc.h)
    return out.reshape(-1)


def stencil_sparse(desc) -> sp.csr_matrix:
    """The same operator as a sparse matrix, assembled entry by entry."""
    nx, ny, nz = desc.nx, desc.ny, desc.nz
    n = nx * ny * nz
    idx = np.arange(n)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    rows, cols, vals = [], [], []
    Wt = _weights(desc)
    if Wt is not None:
        rows.append(idx)
        cols.append(idx)
        vals.append(Wt[0])
        for d, size in enumerate((nx, ny, nz)[: (Wt.shape[0] - 1) // 2]):
            coords = [x, y, z]
            plus = [c.copy() for c in coords]
            minus = [c.copy() for c in coords]
            plus[d] = (coords[d] + 1) % size
            minus[d] = (coords[d] - 1) % size
            rows += [idx, idx]
            cols += [plus[0] + nx * (plus[1] + ny * plus[2]), minus[0] + nx * (minus[1] + ny * minus[2])]
            vals += [Wt[1 + 2 * d], Wt[2 + 2 * d]]
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
        return A.tocsr()
    diag = np.zeros(n) if desc.reaction is None else np.asarray(desc.reaction, dtype=np.float64).copy()
    kap = None if desc.kappa is None else np.asarray(desc.kappa, dtype=np.float64)
    h = desc.h
    for d, (size, a) in enumerate(((nx, desc.adv[0]), (ny, desc.adv[1]), (nz, desc.adv[2]))):
        if size == 1:
            continue
        coords = [x, y, z]
        plus = [c.copy() for c in coords]
        minus = [c.copy() for c in coords]
        plus[d] = (coords[d] + 1) % size
        minus[d] = (coords[d] - 1) % size
        jp = plus[0] + nx * (plus[1] + ny * plus[2])
        jm = minus[0] + nx * (minus[1] + ny * minus[2])
        if kap is None:
            kp = np.full(n, desc.diff)
            km = np.full(n, desc.diff)
        else:
            kp = 0.5 * (kap + kap[jp])
            km = 0.5 * (kap + kap[jm])
        # diffusion: kp (u+ - u)/h^2 - km (u - u-)/h^2
        rows += [idx, idx]
        cols += [jp, jm]
        vals += [kp / h ** 2 - a / (2 * h), km / h ** 2 + a / (2 * h)]
        diag = diag - (kp + km) / h ** 2
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A.tocsr()  # duplicate (row, col) pairs are summed (size-2 periodic axes)


def stencil_dense(desc) -> np.ndarray:
    """Dense matrix with column j equal to A e_j (small N only)."""
    n = desc.n
    if n > 8192:
        raise ValueError("dense assembly is for small problems")
    A = np.empty((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = stencil_apply(desc, e)
        e[j] = 0.0
    return A


def csr_matrix(desc) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(desc.val, dtype=np.float64),
                          np.asarray(desc.col), np.asarray(desc.rowptr)),
                         shape=(desc.n, desc.n))


def make_apply(desc):
    """Return x -> A x for a StencilDesc or CsrDesc."""
    if getattr(desc, "kind", None) == "csr":
        M = csr_matrix(desc)
        return lambda v: M @ v
    return lambda v: stencil_apply(desc, v)


def dense(desc) -> np.ndarray:
    if getattr(desc, "kind", None) == "csr":
        return csr_matrix(desc).toarray()
    return stencil_dense(desc)


def norm1_bound(desc) -> float:
    """||A||_1 (maximum absolute column sum), exact, from the sparse form."""
    if getattr(desc, "kind", None) == "csr":
        M = csr_matrix(desc)
    else:
        M = stencil_sparse(desc)
    return float(np.max(np.asarray(abs(M).sum(axis=0)).ravel()))
