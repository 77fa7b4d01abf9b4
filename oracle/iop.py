"""Algorithm 2 of Section 3.3: the incomplete orthogonalization procedure.

Works on augmented vectors [x; y] of length N + p without forming A~; the
product A~ [x; y] = [A x + nu B y; K y] is the block form of the augmented
product of Theorem 1 (B already scaled by nu of Eq. (48)).  Each new vector is
orthogonalised, by modified Gram-Schmidt, against the last q basis vectors
(the paper's procedure is q = 2); q = 0 means all of them (full Arnoldi).

Readings (listed with the other readings of the paper in the design notes):
  * "s ~ 0" (happy breakdown) is taken as s <= 1e-12 ||A~ v_j||.
  * "H(i+1, j) = s" stores h_{j+1,j}.
"""

from __future__ import annotations

from typing import Callable, Sequence

import numpy as np

BREAKDOWN_REL = 1e-12


class IOPBasis:
    """Incrementally extendable basis V (rows are basis vectors) and H."""

    def __init__(self, apply_A: Callable[[np.ndarray], np.ndarray], Bcols: Sequence[np.ndarray],
                 nu: float, x0: np.ndarray, y0: np.ndarray, q: int, m_max: int,
                 breakdown_rel: float = BREAKDOWN_REL):
        self.apply_A = apply_A
        self.Bcols = [np.asarray(b, dtype=np.float64) for b in Bcols]
        self.nu = float(nu)
        self.N = int(np.asarray(x0).size)
        self.p = len(self.Bcols)
        self.q = int(q)
        self.m_max = int(m_max)
        self.breakdown_rel = breakdown_rel
        v = np.concatenate([np.asarray(x0, dtype=np.float64), np.asarray(y0, dtype=np.float64)])
        self.beta = float(np.linalg.norm(v))
        self.V = np.zeros((m_max + 1, self.N + self.p))
        self.H = np.zeros((m_max + 1, m_max + 1))
        self.j = 0
        self.breakdown = False
        self.matvecs = 0
        if self.beta > 0.0:
            self.V[0] = v / self.beta
        else:
            self.breakdown = True

    def apply_aug(self, v: np.ndarray) -> np.ndarray:
        """A~ v for v = [x; y] (Algorithm 2, Theorem 1)."""
        N, p = self.N, self.p
        x, y = v[:N], v[N:]
        out = np.empty(N + p)
        ax = self.apply_A(x)
        for c in range(p):
            ax = ax + self.nu * y[c] * self.Bcols[c]
        out[:N] = ax
        if p > 0:
            out[N:N + p - 1] = y[1:]
            out[N + p - 1] = 0.0
        return out

    def extend(self, m: int) -> None:
        """Run Algorithm 2 until j == m (or breakdown)."""
        m = min(int(m), self.m_max)
        while self.j < m and not self.breakdown:
            c = self.j                          # extend from v_{c+1} (1-based)
            w = self.apply_aug(self.V[c])
            self.matvecs += 1
            pre = float(np.linalg.norm(w))
            lo = 0 if self.q == 0 else max(0, c - self.q + 1)
            for i in range(lo, c + 1):
                hij = float(self.V[i] @ w)
                self.H[i, c] = hij
                w = w - hij * self.V[i]
            s = float(np.linalg.norm(w))
            self.j = c + 1
            if s <= self.breakdown_rel * pre:
                self.breakdown = True
                self.H[c + 1, c] = 0.0
                break
            self.H[c + 1, c] = s
            self.V[c + 1] = w / s


def iop_basis(apply_A, Bcols, nu, x0, y0, m, q, m_max=None):
    """Convenience: build m steps and return (V (j+1 rows), H (j+1 x j), j, breakdown)."""
    b = IOPBasis(apply_A, Bcols, nu, x0, y0, q, m_max or m)
    b.extend(m)
    j = b.j
    return b.V[: j + 1].copy(), b.H[: j + 1, :j].copy(), j, b.breakdown, b.beta
