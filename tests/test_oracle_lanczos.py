"""Pins of the per-term Lanczos route (oracle/lanczos.py) for symmetric A.

The route computes each tau^k phi_k(tau A) b_k on its own (Eq. (4)), with no
augmented matrix, so agreement with the augmented routes also checks
Theorem 1.  It is pinned against:
  * the eigendecomposition of A (Q phi_k(tau Lambda) Q^T b_k, numpy.linalg.eigh);
  * the dense augmented exponential (Eq. (14)) on variable-coefficient boxes;
  * the DFT closed form on a constant-coefficient 48^3 box;
  * the full-Arnoldi route on a variable-coefficient 32^3 box;
  * the special cases tau = 0 (w = b_0) and A = 0 (w = sum_k tau^k / k! b_k).
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators, spectral
from oracle.arnoldi import phi_combination_arnoldi
from oracle.lanczos import phi_combination_lanczos, phi_term_lanczos
from oracle.phi import phi


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("side,scale", [(8, 0.3), (12, 0.3), (10, 0.01)])
def test_lanczos_vs_dense_augmented(side, scale):
    # tau chosen so that tau ||A||_1 is about 400 (scale 0.3) or about 10 (0.01)
    pr = W.diffusion3d_problem(side, 2, 1e-3 * (256 / side) ** 2 * scale, seed=77 + side)
    A = operators.dense(pr.op)
    assert np.array_equal(A, A.T)
    ref = augmented.phi_combination_dense(A, pr.tau, pr.vectors)
    got = phi_combination_lanczos(operators.make_apply(pr.op), pr.tau, pr.vectors)
    assert rel(got, ref) <= 1e-12


def test_lanczos_terms_vs_eigendecomposition():
    pr = W.diffusion3d_problem(8, 3, 2e-2, seed=11)
    A = operators.dense(pr.op)
    lam, Q = np.linalg.eigh(A)
    for k, b in enumerate(pr.vectors):
        ref = (pr.tau ** k) * (Q @ (np.real(phi(k, pr.tau * lam)) * (Q.T @ b)))
        got = phi_term_lanczos(operators.make_apply(pr.op), pr.tau, k, b)
        assert rel(got, ref) <= 1e-12, k


def test_lanczos_vs_dft_constant_box():
    pr = W.diffusion3d_problem(48, 2, 8e-3, seed=5, constant=(1.3, -2.0))
    ref = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    got = phi_combination_lanczos(operators.make_apply(pr.op), pr.tau, pr.vectors)
    assert rel(got, ref) <= 1e-12


def test_lanczos_vs_arnoldi_variable_box():
    pr = W.diffusion3d_problem(32, 2, 8e-3, seed=6)
    ref = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-12)
    got = phi_combination_lanczos(operators.make_apply(pr.op), pr.tau, pr.vectors)
    assert rel(got, ref) <= 1e-11


def test_lanczos_special_cases():
    g = np.random.Generator(np.random.PCG64(3))
    vecs = [g.standard_normal(200) for _ in range(4)]
    zero = lambda v: np.zeros_like(v)   # noqa: E731
    # tau = 0: only b_0 survives
    w0 = phi_combination_lanczos(zero, 0.0, vecs)
    assert np.array_equal(w0, vecs[0])
    # A = 0: phi_k(0) = 1/k!  (the Krylov space of every term is invariant at once)
    tau = 0.7
    got = phi_combination_lanczos(zero, tau, vecs)
    ref = sum(tau ** k / math.factorial(k) * b for k, b in enumerate(vecs))
    assert rel(got, ref) <= 1e-15
    # A = lambda I: phi_k(tau lambda) b_k exactly, from one Lanczos step
    lam = -3.0
    got = phi_combination_lanczos(lambda v: lam * v, tau, vecs)
    ref = sum(tau ** k * float(np.real(phi(k, tau * lam))) * b for k, b in enumerate(vecs))
    assert rel(got, ref) <= 1e-14
