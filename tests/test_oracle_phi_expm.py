"""Pins of the oracle's scalar phi_k (Eq. (3)) and dense exponential.

Everything here is checked against something other than the oracle itself:
closed forms, Gauss-Legendre quadrature of the integral in Eq. (3),
scipy.linalg.expm, and the matrix identities Eq. (17) and Eq. (38).
"""

import math

import numpy as np
import pytest
import scipy.linalg as sl

from oracle.expm import expm, expm_apply
from oracle.phi import phi


def _quad_phi(k, z, n=200):
    """Gauss-Legendre quadrature of int_0^1 e^{z(1-t)} t^{k-1}/(k-1)! dt."""
    x, wq = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (x + 1.0)
    wq = 0.5 * wq
    return np.sum(wq * np.exp(z * (1.0 - t)) * t ** (k - 1)) / math.factorial(k - 1)


def test_phi0_is_exp():
    z = np.array([-30.0, -1.0, -0.3, 0.0, 0.7, 2.5])
    assert np.allclose(phi(0, z), np.exp(z), rtol=1e-15, atol=0)
    zc = np.array([0.3 + 0.4j, -5 + 20j, 1j])
    assert np.allclose(phi(0, zc), np.exp(zc), rtol=1e-15, atol=0)


@pytest.mark.parametrize("z", [0.5, -0.8, 0.9j, -0.6 + 0.6j, 1.5, -3.0, -40.0, 7.0 - 3.0j, -1000.0 + 50j])
def test_phi1_phi2_closed_forms(z):
    e = np.exp(z)
    assert abs(phi(1, z) - (e - 1) / z) <= 1e-14 * abs((e - 1) / z)
    ref2 = (e - 1 - z) / z ** 2
    assert abs(phi(2, z) - ref2) <= 1e-12 * abs(ref2)


def test_phi_at_zero():
    for k in range(9):
        assert phi(k, 0.0) == pytest.approx(1.0 / math.factorial(k), rel=1e-16)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_phi_against_quadrature_of_eq3(k):
    zs = [0.2, -0.9, 0.99, 1.01, -2.0, 3.5, -7.5, 0.5 + 0.5j, -4 + 6j, 2j, -9.0 - 1.0j]
    for z in zs:
        ref = _quad_phi(k, z)
        got = phi(k, z)
        assert abs(got - ref) <= 5e-14 * abs(ref), (k, z)


def test_phi_recurrence_consistency_large_z():
    # phi_{k+1}(z) z = phi_k(z) - 1/k!  holds on both evaluation branches
    z = np.array([-0.99, 0.999, -1.0001, 12.0, -250.0, 30j, -3 + 3j])
    for k in range(5):
        lhs = phi(k + 1, z) * z
        rhs = phi(k, z) - 1.0 / math.factorial(k)
        assert np.allclose(lhs, rhs, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("scale", [1e-3, 0.3, 1.0, 7.0, 60.0, 400.0])
def test_expm_vs_scipy(scale):
    g = np.random.Generator(np.random.PCG64(11))
    for n in (1, 3, 17, 40):
        M = g.standard_normal((n, n))
        M = scale * M / max(1e-300, np.linalg.norm(M, 1))
        # make it mildly non-normal and dissipative like a Krylov Hessenberg matrix
        M = M - 0.5 * scale * np.eye(n)
        ref = sl.expm(M)
        got = expm(M)
        assert np.linalg.norm(got - ref, 1) <= 1e-12 * max(1.0, np.linalg.norm(ref, 1)) * max(1.0, scale / 10)


def test_expm_shift_matrix_eq17():
    p, tau = 6, 0.37
    K = np.diag(np.ones(p - 1), 1)
    E = expm(tau * K)
    for i in range(p):
        for j in range(p):
            ref = tau ** (j - i) / math.factorial(j - i) if j >= i else 0.0
            assert E[i, j] == pytest.approx(ref, rel=1e-15, abs=1e-300)


def test_expm_closed_forms():
    d = np.array([-3.0, -0.5, 0.0, 1.25])
    assert np.allclose(expm(np.diag(d)), np.diag(np.exp(d)), rtol=2e-14, atol=0)
    lam = -2.0
    J = np.array([[lam, 1.0], [0.0, lam]])
    assert np.allclose(expm(J), np.exp(lam) * np.array([[1.0, 1.0], [0.0, 1.0]]), rtol=1e-14, atol=0)
    th = 9.0
    R = np.array([[0.0, th], [-th, 0.0]])
    ref = np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]])
    assert np.allclose(expm(R), ref, rtol=0, atol=1e-13)


def test_expm_block_identity_eq38():
    # exp([[tau M, tau e1], [0, 0]]) = [[e^{tau M}, tau phi_1(tau M) e1], [0, 1]]
    g = np.random.Generator(np.random.PCG64(5))
    m, tau = 12, 0.8
    M = g.standard_normal((m, m)) - 3 * np.eye(m)
    Ht = np.zeros((m + 1, m + 1))
    Ht[:m, :m] = M
    Ht[0, m] = 1.0
    F = expm(tau * Ht)
    eM = sl.expm(tau * M)
    # tau phi_1(tau M) e1 = M^{-1} (e^{tau M} - I) e1
    ref_col = np.linalg.solve(M, (eM - np.eye(m))[:, 0])
    assert np.allclose(F[:m, :m], eM, rtol=1e-12, atol=1e-14)
    assert np.allclose(F[:m, m], ref_col, rtol=1e-11, atol=1e-14)
    assert F[m, m] == pytest.approx(1.0, abs=1e-15)
    assert np.all(F[m, :m] == 0.0)


def test_expm_apply_matches_matrix():
    g = np.random.Generator(np.random.PCG64(3))
    M = 5.0 * g.standard_normal((30, 30)) / 30 ** 0.5 - 4 * np.eye(30)
    v = g.standard_normal(30)
    ref = sl.expm(M) @ v
    assert np.linalg.norm(expm_apply(M, v) - ref) <= 1e-12 * np.linalg.norm(ref)
