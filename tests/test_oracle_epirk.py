"""Pins of the oracle's EPIRK4s3A integrator (Section 4, Eq. (51)) on the
paper's 2-D advection-diffusion-reaction problem (periodic stand-in).

Each check is against something other than the oracle itself:
  * linear problem (gamma = 0): one step is the matrix exponential
    exp(h A) u exactly (phi_1(hA) h A u = (e^{hA} - I) u and r = 0), checked
    against scipy's expm;
  * a single cell (the stencil terms vanish, u' = gamma g(u)): fourth-order
    convergence against scipy's DOP853 at tight tolerance;
  * the 8 x 8 grid: fourth-order convergence against scipy's Radau with the
    exact Jacobian at tight tolerance;
  * the full-Arnoldi route agrees with the dense route.
A wrong coefficient or term of Eq. (51) lowers the observed order below 3.5.
"""

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from oracle import epirk as E
from oracle import operators


def test_linear_step_is_matrix_exponential():
    prob = E.ADR2D(8, gamma=0.0)
    u0 = E.initial_condition(8)
    A = operators.dense(prob.lin)
    for h in (1e-3, 1e-2, 5e-2):
        got = E.epirk4s3a_step(prob, u0, h)
        ref = expm(h * A) @ u0
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def _orders(errs):
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_single_cell_fourth_order():
    prob = E.ADR2D(1)
    u0 = np.array([0.3])
    T = 0.05
    ref = solve_ivp(lambda t, y: prob.f(y), (0.0, T), u0, method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    errs = [abs(E.integrate(prob, u0, T / k, k) - ref)[0] for k in (2, 4, 8, 16)]
    orders = _orders(errs)
    assert min(orders) >= 3.8, (errs, orders)
    assert errs[-1] <= 1e-6


def test_grid_8x8_fourth_order_against_radau():
    n = 8
    prob = E.ADR2D(n)
    u0 = E.initial_condition(n)
    T = 0.004
    ref = solve_ivp(lambda t, y: prob.f(y), (0.0, T), u0, method="Radau", rtol=1e-13, atol=1e-14,
                    jac=lambda t, y: operators.dense(prob.jacobian_desc(y))).y[:, -1]
    errs = [np.linalg.norm(E.integrate(prob, u0, T / k, k) - ref) / np.linalg.norm(ref) for k in (2, 4, 8)]
    orders = _orders(errs)
    assert min(orders) >= 3.8, (errs, orders)


def test_arnoldi_route_matches_dense_route():
    prob = E.ADR2D(8)
    u0 = E.initial_condition(8)
    a = E.integrate(prob, u0, 1e-3, 2, route="dense")
    b = E.integrate(prob, u0, 1e-3, 2, route="arnoldi", tol_o=1e-13)
    assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(a)


def test_initial_condition_and_jacobian():
    # u0 = 256 (x y (1-x)(1-y))^2 + 0.3: 0.3 on the x = 0 and y = 0 lines, 1.3 at the centre
    u0 = E.initial_condition(8).reshape(8, 8)
    assert np.allclose(u0[0, :], 0.3) and np.allclose(u0[:, 0], 0.3)
    assert u0[4, 4] == pytest.approx(1.3)
    # the Jacobian's reaction is gamma g'(u): a finite-difference check of f
    prob = E.ADR2D(6)
    u = 0.2 + 0.6 * np.random.default_rng(3).random(36)
    v = np.random.default_rng(4).standard_normal(36)
    eps = 1e-6
    fd = (prob.f(u + eps * v) - prob.f(u - eps * v)) / (2 * eps)
    Jv = operators.make_apply(prob.jacobian_desc(u))(v)
    assert np.linalg.norm(fd - Jv) <= 1e-6 * np.linalg.norm(Jv)
