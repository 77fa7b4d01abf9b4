"""Pins of the oracle's Algorithm 2 (IOP) and of its full-Arnoldi route.

IOP: the factorisation Eq. (30), orthonormality inside the window, the band
of H, Theorem 2 (Eq. (31)), full orthogonality when the window covers the
whole basis, the Lanczos special case, and breakdown where it must occur.
Arnoldi route: against the dense Theorem 1 result and the DFT result, and
against itself at a 100x tighter tolerance.
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators, spectral
from oracle.arnoldi import phi_combination_arnoldi
from oracle.iop import IOPBasis, iop_basis


def _setup(pr):
    p = pr.p
    nu, mu = augmented.b_norm_scaling(pr.vectors)
    Bcols = [pr.vectors[p - c] for c in range(p)]
    y0 = mu * augmented.trailing_entries(p, 0.0)
    A = operators.dense(pr.op)
    At, _ = augmented.augmented_matrix(A, [pr.vectors[0]] + [nu * b for b in pr.vectors[1:]])
    return Bcols, nu, y0, At, operators.make_apply(pr.op)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_iop_factorisation_eq30_and_window(q):
    pr = W.cfg1()
    Bcols, nu, y0, At, ap = _setup(pr)
    m = 30
    V, H, j, bd, beta = iop_basis(ap, Bcols, nu, pr.vectors[0], y0, m, q)
    assert j == m and not bd
    Vm = V[:m].T                    # (N+p) x m, columns v_1..v_m
    Vm1 = V[: m + 1].T
    R = At @ Vm - Vm1 @ H           # Eq. (30): A~ V_m = V_{m+1} H_{m+1,m}
    assert np.linalg.norm(R) <= 1e-14 * np.linalg.norm(At, 2) * math.sqrt(m)
    G = V @ V.T
    assert np.allclose(np.diag(G), 1.0, atol=1e-14)
    for i in range(m + 1):
        for k in range(m + 1):
            if i != k and abs(i - k) < q:
                assert abs(G[i, k]) <= 1e-13
    # banded upper Hessenberg: h_{ik} = 0 unless k-q+1 <= i <= k+1
    for i in range(m + 1):
        for k in range(m):
            if i > k + 1 or i < k - q + 1:
                assert H[i, k] == 0.0


def test_iop_basis_is_not_orthogonal_beyond_window():
    pr = W.cfg1()
    Bcols, nu, y0, At, ap = _setup(pr)
    V, H, j, bd, beta = iop_basis(ap, Bcols, nu, pr.vectors[0], y0, 40, 2)
    G = V @ V.T
    off = max(abs(G[i, k]) for i in range(41) for k in range(41) if abs(i - k) >= 3)
    assert off > 1e-6      # Section 3.3: the columns are not orthonormal in general


def test_theorem2_polynomials():
    pr = W.adr2d_problem(10, 2, 0.0, seed=6, diff=1e-3, adv=0.5)
    Bcols, nu, y0, At, ap = _setup(pr)
    m = 12
    v = np.concatenate([pr.vectors[0], y0])
    V, H, j, bd, beta = iop_basis(ap, Bcols, nu, pr.vectors[0], y0, m, 2)
    Hm = H[:m, :m]
    Vm = V[:m].T
    y = np.zeros(m)
    y[0] = 1.0
    x = v.copy()
    for k in range(m - 1):              # degrees 0..m-2 (Eq. (31))
        rhs = np.linalg.norm(v) * (Vm @ y)
        assert np.linalg.norm(x - rhs) <= 1e-11 * np.linalg.norm(x), k
        x = At @ x
        y = Hm @ y
    # degree m-1 and beyond is not reproduced in general
    rhs = np.linalg.norm(v) * (Vm @ (Hm @ y))
    assert np.linalg.norm(At @ x - rhs) > 1e-8 * np.linalg.norm(At @ x)


def test_full_window_is_full_arnoldi():
    pr = W.cfg1()
    Bcols, nu, y0, At, ap = _setup(pr)
    V, H, j, bd, beta = iop_basis(ap, Bcols, nu, pr.vectors[0], y0, 25, 0)
    G = V @ V.T
    assert np.allclose(G, np.eye(26), atol=1e-12)
    V2, H2, *_ = iop_basis(ap, Bcols, nu, pr.vectors[0], y0, 25, 30)   # window >= m
    assert np.allclose(H2, H, rtol=1e-12, atol=1e-9)


def test_lanczos_case_symmetric_p0():
    pr = W.diffusion3d_problem(5, 0, 1e-3, seed=1)
    ap = operators.make_apply(pr.op)
    V, H, j, bd, beta = iop_basis(ap, [], 1.0, pr.vectors[0], np.zeros(0), 15, 2)
    T = H[:15, :15]
    assert np.allclose(T, T.T, rtol=1e-11, atol=1e-9 * np.abs(T).max())
    assert np.count_nonzero(np.triu(T, 2)) == 0
    Vf, Hf, *_ = iop_basis(ap, [], 1.0, pr.vectors[0], np.zeros(0), 6, 0)
    assert np.allclose(Hf[:6, :6], H[:6, :6], rtol=1e-9, atol=1e-9 * np.abs(T).max())


@pytest.mark.parametrize("p,q", [(0, 2), (1, 2), (3, 0), (3, 4), (4, 0)])
def test_breakdown_zero_operator(p, q):
    """A = 0: the Krylov space of A~ and [b_0; e_p] has dimension p+1, so the
    procedure breaks down at j = p+1 whenever its window spans that space
    (q = 0, or q >= p+1)."""
    n = 20
    g = np.random.Generator(np.random.PCG64(p))
    vecs = [g.standard_normal(n) for _ in range(p + 1)]
    nu, mu = augmented.b_norm_scaling(vecs)
    Bcols = [vecs[p - c] for c in range(p)]
    y0 = mu * augmented.trailing_entries(p, 0.0)
    b = IOPBasis(lambda x: 0.0 * x, Bcols, nu, vecs[0], y0, q, 50)
    b.extend(50)
    assert b.breakdown and b.j == p + 1


def test_no_breakdown_when_window_is_shorter_than_invariant_space():
    """With the paper's window of 2 and p = 3 the new vector keeps components
    along older basis vectors, so no breakdown occurs (Section 3.3: the IOP
    basis spans K_m but is not orthonormal)."""
    p, n = 3, 20
    g = np.random.Generator(np.random.PCG64(p))
    vecs = [g.standard_normal(n) for _ in range(p + 1)]
    nu, mu = augmented.b_norm_scaling(vecs)
    b = IOPBasis(lambda x: 0.0 * x, [vecs[p - c] for c in range(p)], nu, vecs[0],
                 mu * augmented.trailing_entries(p, 0.0), 2, 12)
    b.extend(12)
    assert not b.breakdown and b.j == 12


def test_breakdown_scalar_operator():
    n = 16
    v = np.random.Generator(np.random.PCG64(0)).standard_normal(n)
    b = IOPBasis(lambda x: -3.0 * x, [], 1.0, v, np.zeros(0), 2, 20)
    b.extend(20)
    assert b.breakdown and b.j == 1 and b.H[0, 0] == pytest.approx(-3.0)


# ---------------------------------------------------------------- Arnoldi route

def test_arnoldi_vs_dense_cfg1():
    pr = W.cfg1()
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-12)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_arnoldi_vs_dense_3d_variable_kappa():
    pr = W.diffusion3d_problem(8, 2, 1e-3, seed=4)
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-12)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_arnoldi_vs_dft_stiff_2d():
    pr = W.adr2d_problem(96, 3, 1e-2, seed=10, constant_reaction=-0.5)
    ref = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    got = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-12)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_arnoldi_self_convergence():
    pr = W.adr2d_problem(40, 2, 3e-2, seed=13)
    ap = operators.make_apply(pr.op)
    a = phi_combination_arnoldi(ap, pr.tau, pr.vectors, tol_o=1e-10)
    b = phi_combination_arnoldi(ap, pr.tau, pr.vectors, tol_o=1e-12)
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b) * 10
