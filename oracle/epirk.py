"""EPIRK4s3A (Section 4, Eq. (51)) on the paper's 2-D advection-diffusion-
reaction test problem (Section 4, "ADR 2D"), plain FP64 on the CPU.

Test infrastructure only: it is the reference for the library's integrator
driver and is never imported by it.

Problem: u_t = eps Lap(u) - alpha (u_x + u_y) + gamma u (u - 1/2)(1 - u) on the
unit square, here with periodic boundaries on an n x n grid of spacing 1/n
(the paper uses homogeneous Neumann boundaries; the initial condition
256 (x y (1 - x)(1 - y))^2 + 0.3 has zero normal derivative there, so its
periodic extension is smooth), eps = 1/100, alpha = -10, gamma = 100.

    f(u)  = A_lin u + gamma g(u),      g(u) = u (u - 1/2)(1 - u)
    J_n   = A_lin + diag(gamma g'(u_n))                          (the Jacobian at u_n)
    r(U)  = f(U) - f(u_n) - J_n (U - u_n)                         (Section 2, after Eq. (2))

One step of size h (Eq. (51)):

    U_2     = u_n + 1/2 phi_1(h J_n / 2) h f(u_n)
    U_3     = u_n + 2/3 phi_1(2 h J_n / 3) h f(u_n)
    u_{n+1} = u_n + phi_1(h J_n) h f(u_n)
                  + (32 phi_3(h J_n) - 144 phi_4(h J_n)) h r(U_2)
                  + (-27/2 phi_3(h J_n) + 81 phi_4(h J_n)) h r(U_3)

The stage terms are single phi_1 products; the last line is one
phi-combination of Eq. (4) with tau = 1 and the matrix h J_n (the grouping of
Eqs. (10)-(11), written for the coefficients of Eq. (51)):
b_0 = 0, b_1 = h f(u_n), b_2 = 0, b_3 = h (32 r(U_2) - 27/2 r(U_3)),
b_4 = h (-144 r(U_2) + 81 r(U_3)).  Every phi-combination is the dense exact
result of Theorem 1 (small N) or the full-Arnoldi oracle (larger N).
"""

from __future__ import annotations

import numpy as np

from . import operators
from .arnoldi import phi_combination_arnoldi
from .augmented import phi_combination_dense

EPS, ALPHA, GAMMA = 1.0e-2, -10.0, 100.0


class _Desc:
    """Periodic 5-point operator data in the shape oracle.operators reads."""

    def __init__(self, n, eps, alpha, reaction=None):
        self.nx, self.ny, self.nz = n, n, 1
        self.h = 1.0 / n
        self.diff = eps
        self.kappa = None
        self.adv = (alpha, alpha, 0.0)
        self.reaction = reaction
        self.kind = "stencil2d"

    @property
    def n(self):
        return self.nx * self.ny


def initial_condition(n: int) -> np.ndarray:
    """u = 256 (x y (1 - x)(1 - y))^2 + 0.3 at the cell points x_i = i / n."""
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x, indexing="xy")      # index x + n y
    return (256.0 * (X * Y * (1 - X) * (1 - Y)) ** 2 + 0.3).reshape(-1)


def g(u):
    return u * (u - 0.5) * (1.0 - u)


def dg(u):
    """g'(u) = -3 u^2 + 3 u - 1/2."""
    return -3.0 * u * u + 3.0 * u - 0.5


class ADR2D:
    def __init__(self, n: int, eps: float = EPS, alpha: float = ALPHA, gamma: float = GAMMA):
        self.n_side = n
        self.gamma = gamma
        self.lin = _Desc(n, eps, alpha)
        self.apply_lin = operators.make_apply(self.lin)

    def f(self, u):
        return self.apply_lin(u) + self.gamma * g(u)

    def jacobian_desc(self, u):
        return _Desc(self.n_side, self.lin.diff, self.lin.adv[0], reaction=self.gamma * dg(u))


class _Scaled:
    """h A for an operator description A (for the tau = 1 form of Eq. (10))."""

    def __init__(self, desc, h):
        self.desc, self.h = desc, h
        self.nx, self.ny, self.nz, self.kind = desc.nx, desc.ny, desc.nz, desc.kind


def _dense(desc):
    if isinstance(desc, _Scaled):
        return desc.h * operators.dense(desc.desc)
    return operators.dense(desc)


def _apply(desc):
    if isinstance(desc, _Scaled):
        inner = operators.make_apply(desc.desc)
        return lambda v: desc.h * inner(v)
    return operators.make_apply(desc)


def _phi_comb(desc, tau, vectors, route, tol_o):
    if route == "dense":
        return phi_combination_dense(_dense(desc), tau, vectors)
    return phi_combination_arnoldi(_apply(desc), tau, vectors, tol_o=tol_o)


def epirk4s3a_step(prob: ADR2D, u: np.ndarray, h: float, route: str = "dense", tol_o: float = 1e-12):
    """One step of Eq. (51) from u_n = u."""
    fu = prob.f(u)
    J = prob.jacobian_desc(u)
    zero = np.zeros_like(u)

    def remainder(U):
        # f(U) - f(u_n) - J_n (U - u_n); the linear part of f cancels
        return prob.f(U) - fu - operators.make_apply(J)(U - u)

    # stages: c phi_1(c h J) h f = (c h) phi_1((c h) J) f, the Eq. (4) result at tau = c h
    U2 = u + _phi_comb(J, 0.5 * h, [zero, fu], route, tol_o)
    U3 = u + _phi_comb(J, 2.0 * h / 3.0, [zero, fu], route, tol_o)
    r2, r3 = remainder(U2), remainder(U3)
    # Eq. (4) with tau = 1 and the matrix h J_n
    hJ = _Scaled(J, h)
    b = [zero, h * fu, zero, h * (32.0 * r2 - 13.5 * r3), h * (-144.0 * r2 + 81.0 * r3)]
    return u + _phi_comb(hJ, 1.0, b, route, tol_o)


def integrate(prob: ADR2D, u0: np.ndarray, h: float, nsteps: int, route: str = "dense",
              tol_o: float = 1e-12) -> np.ndarray:
    u = np.array(u0, dtype=np.float64)
    for _ in range(nsteps):
        u = epirk4s3a_step(prob, u, h, route, tol_o)
    return u
