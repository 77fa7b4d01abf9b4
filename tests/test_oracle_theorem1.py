"""Pins of Theorem 1 (Section 3.1) as the oracle writes it out.

The dense route (augmented matrix of Eq. (13), exponentiated) is checked
against results fixed by other means: elementwise closed forms for diagonal
A, eigendecomposition for symmetric A, A = 0, p = 0 (plain exponential),
Eq. (15), scipy's expm_multiply on the sparse augmented matrix, and the ODE
(5) the combination solves.  A test also fixes the corrigendum's column
order of B.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import augmented, operators
from oracle.augmented import augmented_matrix, phi_combination_dense, trailing_entries
from oracle.phi import phi


def _vecs(n, p, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    return [g.standard_normal(n) for _ in range(p + 1)]


@pytest.mark.parametrize("p", [0, 1, 2, 4])
def test_diagonal_A_closed_form(p):
    g = np.random.Generator(np.random.PCG64(20 + p))
    a = g.uniform(-60.0, 2.0, size=25)
    tau = 0.3
    vecs = _vecs(25, p, 30 + p)
    got = phi_combination_dense(np.diag(a), tau, vecs)
    ref = sum(tau ** k * phi(k, tau * a) * vecs[k] for k in range(p + 1))
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_symmetric_A_eigendecomposition():
    pr = W.diffusion3d_problem(4, 3, 2e-3, seed=9)
    A = operators.dense(pr.op)
    assert np.allclose(A, A.T)
    lam, Q = np.linalg.eigh(A)
    ref = sum(pr.tau ** k * (Q @ (phi(k, pr.tau * lam) * (Q.T @ b))) for k, b in enumerate(pr.vectors))
    got = phi_combination_dense(A, pr.tau, pr.vectors)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_A_zero_gives_taylor_polynomial():
    vecs = _vecs(10, 4, 1)
    tau = 0.7
    got = phi_combination_dense(np.zeros((10, 10)), tau, vecs)
    ref = sum(tau ** j / math.factorial(j) * vecs[j] for j in range(5))
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_p0_is_plain_exponential():
    pr = W.cfg1()
    A = operators.dense(pr.op)
    got = phi_combination_dense(A, pr.tau, pr.vectors[:1])
    ref = sl.expm(pr.tau * A) @ pr.vectors[0]
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_trailing_entries_eq15(p):
    pr = W.adr2d_problem(8, p, 0.05, seed=4)
    A = operators.dense(pr.op)
    w = phi_combination_dense(A, 0.05, pr.vectors, full=True)
    ref = np.array([0.05 ** (p - 1 - i) / math.factorial(p - 1 - i) for i in range(p)])
    assert np.allclose(w[-p:], ref, rtol=1e-13, atol=1e-15)
    assert np.allclose(trailing_entries(p, 0.05), ref, rtol=1e-15)


def test_corrigendum_column_order_of_B():
    """B = [b_p, ..., b_1] (corrigendum to Eqs. (18)-(19)); the reverse
    order gives a different, wrong combination."""
    pr = W.adr2d_problem(6, 3, 0.02, seed=8)
    A = operators.dense(pr.op)
    tau = pr.tau
    lam, X = np.linalg.eig(A)
    Xi = np.linalg.inv(X)
    ref = np.real(sum(tau ** k * (X @ (phi(k, tau * lam) * (Xi @ b))) for k, b in enumerate(pr.vectors)))
    got = phi_combination_dense(A, tau, pr.vectors)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    wrong_order = [pr.vectors[0]] + list(reversed(pr.vectors[1:]))
    bad = phi_combination_dense(A, tau, wrong_order)
    assert np.linalg.norm(bad - ref) > 1e-3 * np.linalg.norm(ref)


def test_against_scipy_expm_multiply_sparse_augmented():
    pr = W.adr2d_problem(48, 3, 3e-3, seed=12)
    S = operators.stencil_sparse(pr.op)
    n, p = pr.n, pr.p
    nu, mu = augmented.b_norm_scaling(pr.vectors)
    # sparse augmented matrix with nu-scaled B and mu-scaled e_p (Eqs. (48)-(49))
    Bm = sp.csr_matrix(np.stack([nu * pr.vectors[p - c] for c in range(p)], axis=1))
    K = sp.diags([np.ones(p - 1)], [1], shape=(p, p))
    At = sp.bmat([[S, Bm], [None, K]]).tocsc()
    v = np.concatenate([pr.vectors[0], np.zeros(p - 1), [mu]])
    ref = spla.expm_multiply(pr.tau * At, v)[:n]
    A = S.toarray()
    got = phi_combination_dense(A, pr.tau, pr.vectors)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_solves_ode_5():
    """w(t) = sum t^k phi_k(tA) b_k satisfies w' = A w + sum_k t^{k-1}/(k-1)! b_k."""
    pr = W.adr2d_problem(5, 3, 0.0, seed=2)
    A = operators.dense(pr.op)
    t, dt = 0.01, 1e-5
    wp = phi_combination_dense(A, t + dt, pr.vectors)
    wm = phi_combination_dense(A, t - dt, pr.vectors)
    w0 = phi_combination_dense(A, t, pr.vectors)
    deriv = (wp - wm) / (2 * dt)
    rhs = A @ w0 + sum(t ** (k - 1) / math.factorial(k - 1) * pr.vectors[k] for k in range(1, 4))
    assert np.linalg.norm(deriv - rhs) <= 1e-6 * np.linalg.norm(rhs)


def test_b_norm_scaling_powers_of_two():
    vecs = [np.ones(3), np.array([1.0, -2.0, 0.5]), np.array([3.0, 3.0, 3.0])]
    nu, mu = augmented.b_norm_scaling(vecs)   # ||B||_1 = 9 -> 2^4
    assert (nu, mu) == (1.0 / 16.0, 16.0)
    assert augmented.b_norm_scaling([np.ones(3)]) == (1.0, 1.0)
    assert augmented.b_norm_scaling([np.ones(3), np.zeros(3)]) == (1.0, 1.0)
    assert augmented.b_norm_scaling([np.ones(2), np.array([0.25, 0.25])]) == (2.0, 0.5)
