"""Pins of the error-estimate variants of Section 3.4 (one-term Eq. (36),
two terms of Eq. (35), corrected scheme) in the oracle.

Checked against independent computations on a small ADR problem (dense
augmented matrix of Theorem 1 exponentiated by scipy):
  * Eq. (35) itself: beta tau h sum_k e_m^T phi_k(tau H_m) e_1 (tau A~)^{k-1}
    v_{m+1}, with phi_k(tau H_m) from its power series, equals the true error
    of Eq. (33) for the IOP basis (q = 2) and the full-Arnoldi one (q = 0);
  * a = F(m, m+1) and b = F(m, m+2) of exp(tau [[H, e_1, 0], [0, 0, 1], [0, 0, 0]])
    are tau e_m^T phi_1 e_1 and tau^2 e_m^T phi_2 e_1 (power series);
  * the corrected result equals beta V_{m+1} exp(tau Hbar) e_1 with
    Hbar = [[H_m, 0], [h_{m+1,m} e_m^T, 0]] (the form of the corrected scheme
    in the literature the paper cites), and its true error is its estimate
    (the second term) to within 5% once the series converges;
  * Algorithm 1 with every variant meets the tolerance against the exact
    result.
"""

from math import factorial

import numpy as np
import pytest
from scipy.linalg import expm as scipy_expm

import workloads as W
from oracle import augmented, operators
from oracle.iop import IOPBasis
from oracle.kiops import kiops


def _setup(q, m):
    pr = W.adr2d_problem(6, 2, 2e-2, seed=7)
    desc, vecs, p = pr.op, pr.vectors, 2
    nu, mu = augmented.b_norm_scaling(vecs)
    Bcols = [vecs[p - c] for c in range(p)]
    basis = IOPBasis(operators.make_apply(desc), Bcols, nu, vecs[0], mu * augmented.trailing_entries(p, 0.0), q, 20)
    basis.extend(m)
    N = desc.n
    At = np.zeros((N + p, N + p))
    At[:N, :N] = operators.dense(desc)
    for c in range(p):
        At[:N, N + c] = nu * Bcols[c]
    for i in range(p - 1):
        At[N + i, N + i + 1] = 1.0
    return basis, At, pr.tau


def _phi_series(Z, k, terms=80):
    out = np.zeros_like(Z)
    P = np.eye(Z.shape[0])
    for i in range(terms):
        out += P / factorial(i + k)
        P = P @ Z
    return out


@pytest.mark.parametrize("q", [2, 0])
@pytest.mark.parametrize("m", [4, 6, 8])
def test_eq35_series_is_the_true_error(q, m):
    basis, At, tau = _setup(q, m)
    j = basis.j
    H, h, beta = basis.H[:j, :j], basis.H[j, j - 1], basis.beta
    true = scipy_expm(tau * At) @ (beta * basis.V[0]) - beta * basis.V[:j].T @ scipy_expm(tau * H)[:, 0]
    series = np.zeros_like(true)
    w = basis.V[j].copy()
    for k in range(1, 40):
        series += beta * tau * h * _phi_series(tau * H, k)[j - 1, 0] * w
        w = tau * (At @ w)
    assert np.linalg.norm(series - true) <= 1e-9 * np.linalg.norm(true)


@pytest.mark.parametrize("m", [4, 8, 12])
def test_phi1_phi2_entries_of_the_extended_exponential(m):
    basis, At, tau = _setup(2, m)
    j = basis.j
    H = basis.H[:j, :j]
    Ht = np.zeros((j + 2, j + 2))
    Ht[:j, :j] = H
    Ht[0, j] = 1.0
    Ht[j, j + 1] = 1.0
    F = scipy_expm(tau * Ht)
    assert F[j - 1, j] == pytest.approx(tau * _phi_series(tau * H, 1)[j - 1, 0], rel=1e-9)
    assert F[j - 1, j + 1] == pytest.approx(tau * tau * _phi_series(tau * H, 2)[j - 1, 0], rel=1e-9)


@pytest.mark.parametrize("m", [6, 8, 10])
def test_corrected_scheme_form_and_its_estimate(m):
    basis, At, tau = _setup(2, m)
    j = basis.j
    H, h, beta = basis.H[:j, :j], basis.H[j, j - 1], basis.beta
    Ht = np.zeros((j + 2, j + 2))
    Ht[:j, :j] = H
    Ht[0, j] = 1.0
    Ht[j, j + 1] = 1.0
    F = scipy_expm(tau * Ht)
    a, b = F[j - 1, j], F[j - 1, j + 1]
    corrected = beta * basis.V[:j].T @ F[:j, 0] + beta * h * a * basis.V[j]
    Hbar = np.zeros((j + 1, j + 1))
    Hbar[:j, :j] = H
    Hbar[j, j - 1] = h
    saad = beta * basis.V[:j + 1].T @ scipy_expm(tau * Hbar)[:, 0]
    assert np.linalg.norm(corrected - saad) <= 1e-12 * np.linalg.norm(saad)
    true = scipy_expm(tau * At) @ (beta * basis.V[0])
    est = beta * abs(h) * abs(b) * np.linalg.norm(At @ basis.V[j])
    assert np.linalg.norm(true - corrected) == pytest.approx(est, rel=0.05)


@pytest.mark.parametrize("estimate", ["one", "two", "corrected"])
def test_algorithm1_meets_tolerance_with_each_estimate(estimate):
    pr = W.adr2d_problem(16, 2, 2e-2, seed=11)
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    w, st = kiops(operators.make_apply(pr.op), pr.tau, pr.vectors, tol=1e-8, estimate=estimate)
    assert np.linalg.norm(w - ref) <= 1e-7 * np.linalg.norm(ref)
    assert st.substeps >= 1
