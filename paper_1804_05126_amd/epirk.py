"""EPIRK4s3A exponential integrator (Section 4, Eq. (51)) driving the
phi-combination solver, with the two-call grouping of Section 2 and the
warm start of Section 3.6.

A step of size h from u_n, with J_n the Jacobian of f at u_n and
r(U) = f(U) - f(u_n) - J_n (U - u_n) the nonlinear remainder:

    U_2     = u_n + 1/2 phi_1(h J_n / 2) h f(u_n)
    U_3     = u_n + 2/3 phi_1(2 h J_n / 3) h f(u_n)
    u_{n+1} = u_n + phi_1(h J_n) h f(u_n)
                  + (32 phi_3(h J_n) - 144 phi_4(h J_n)) h r(U_2)
                  + (-27/2 phi_3(h J_n) + 81 phi_4(h J_n)) h r(U_3)

takes two solver calls (Section 2, tasks I and II):

  * call 1, one integration with two output times T = [h/2, 2h/3] of the
    single term phi_1(T J_n) f(u_n) (Task I: the result scaled by 1/T), so
    U_2 = u_n + (h/2) out_1 and U_3 = u_n + (2h/3) out_2;
  * call 2, the combination of Eq. (4) at tau = h with b_0 = 0, b_1 = f(u_n),
    b_2 = 0, b_3 = (32 r(U_2) - 27/2 r(U_3)) / h^2,
    b_4 = (-144 r(U_2) + 81 r(U_3)) / h^3, which is Eqs. (10)-(11) written for
    the operator J_n and the coefficients of Eq. (51).

Each call starts from the Krylov dimension the same call ended with at the
previous step (Algorithm 1 returns m_l; Section 3.6), unless warm_start is off.

The problem supplies f(u) and the Jacobian as a library operator whose
reaction field it rewrites in place at every step (the operator reads its
arrays at every call).
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

from . import Operator, apply, phi_combination, phi_combination_times, _torch


class ADR2D:
    """The 2-D advection-diffusion-reaction test problem of Section 4,

        u_t = eps Lap(u) - alpha (u_x + u_y) + gamma u (u - 1/2)(1 - u),

    eps = 1/100, alpha = -10, gamma = 100, on an n x n periodic grid of spacing
    1/n (the paper's boundaries are homogeneous Neumann; its initial condition
    has zero normal derivative there, so the periodic extension is smooth).
    The linear part is the library's 5-point operator; the Jacobian is the same
    operator with the reaction field gamma g'(u_n), g(u) = u (u - 1/2)(1 - u)."""

    def __init__(self, n: int, eps: float = 1e-2, alpha: float = -10.0, gamma: float = 100.0,
                 precision: str = "fp64"):
        torch = _torch()
        self.n_side = n
        self.N = n * n
        self.gamma = gamma
        h = 1.0 / n
        self.lin = Operator("stencil2d", nx=n, ny=n, nz=1, h=h, diff=eps, adv=(alpha, alpha, 0.0))
        self.reaction = torch.zeros(self.N, dtype=torch.float64, device="cuda")
        self.jac = Operator("stencil2d", nx=n, ny=n, nz=1, h=h, diff=eps, adv=(alpha, alpha, 0.0),
                            reaction=self.reaction, precision=precision)

    def initial_condition(self):
        """u = 256 (x y (1 - x)(1 - y))^2 + 0.3 at the points x_i = i / n (index x + n y)."""
        torch = _torch()
        x = torch.arange(self.n_side, dtype=torch.float64, device="cuda") / self.n_side
        Y, X = torch.meshgrid(x, x, indexing="ij")
        return (256.0 * (X * Y * (1 - X) * (1 - Y)) ** 2 + 0.3).reshape(-1).contiguous()

    def g(self, u):
        return u * (u - 0.5) * (1.0 - u)

    def f(self, u):
        return apply(self.lin, u) + self.gamma * self.g(u)

    def set_jacobian(self, u):
        """Rewrite the Jacobian operator's reaction field: gamma g'(u) = gamma (-3u^2 + 3u - 1/2)."""
        self.reaction.copy_(self.gamma * (-3.0 * u * u + 3.0 * u - 0.5))

    def remainder(self, U, u, fu):
        """r(U) = f(U) - f(u) - J (U - u); the linear part cancels, leaving
        gamma (g(U) - g(u) - g'(u) (U - u))."""
        return self.gamma * (self.g(U) - self.g(u)) - self.reaction * (U - u)

    def close(self):
        self.lin.close()
        self.jac.close()


@dataclasses.dataclass
class StepInfo:
    m_init: List[int]          # Krylov dimension each call started from
    m_last: List[int]          # dimension each call ended with
    matvecs: List[int]
    substeps: List[int]
    rejections: List[int]


class EPIRK4s3A:
    """Constant-step EPIRK4s3A on a problem with f, set_jacobian, remainder
    and a Jacobian operator `jac` (see ADR2D)."""

    def __init__(self, problem, tol: float = 1e-8, q: int = 2, m_init: int = 10, warm_start: bool = True):
        self.prob = problem
        self.tol = tol
        self.q = q
        self.m0 = m_init
        self.warm_start = warm_start
        self.m = [m_init, m_init]        # per call kind
        self.history: List[StepInfo] = []

    def step(self, u, h: float):
        torch = _torch()
        P = self.prob
        fu = P.f(u)
        P.set_jacobian(u)
        zero = torch.zeros_like(u)
        m_used = list(self.m)
        # call 1 (Task I): phi_1(T J) f(u_n) at T = h/2 and 2h/3
        t2, t3 = 0.5 * h, 2.0 * h / 3.0
        (o2, o3), s1, _ = phi_combination_times(P.jac, [t2, t3], [zero, fu], task=1, tol=self.tol,
                                                m_init=m_used[0], q=self.q)
        U2 = u + t2 * o2
        U3 = u + t3 * o3
        r2 = P.remainder(U2, u, fu)
        r3 = P.remainder(U3, u, fu)
        # call 2 (Task II): Eq. (4) at tau = h
        b3 = (32.0 * r2 - 13.5 * r3) / (h * h)
        b4 = (-144.0 * r2 + 81.0 * r3) / (h * h * h)
        w, s2, _ = phi_combination(P.jac, h, [zero, fu, zero, b3, b4], tol=self.tol, m_init=m_used[1], q=self.q)
        if self.warm_start:
            self.m = [s1["m_last"], s2["m_last"]]
        self.history.append(StepInfo(m_init=m_used, m_last=[s1["m_last"], s2["m_last"]],
                                     matvecs=[s1["matvecs"], s2["matvecs"]],
                                     substeps=[s1["substeps"], s2["substeps"]],
                                     rejections=[s1["rejections"], s2["rejections"]]))
        return u + w

    def integrate(self, u0, h: float, nsteps: int):
        u = u0.clone()
        for _ in range(nsteps):
            u = self.step(u, h)
        return u
