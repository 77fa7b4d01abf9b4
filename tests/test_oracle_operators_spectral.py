"""Pins of the oracle's operators and its DFT route.

The shifted-array form and the entry-by-entry sparse form of each operator
are written separately and must agree; the DFT eigenvalues must equal the
eigenvalues of the assembled matrix; the DFT result must equal the dense
Theorem 1 result; pure diffusion must be symmetric and annihilate constants.
"""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators, spectral


@pytest.mark.parametrize("shape", [(7, 5, 1), (2, 6, 1), (4, 3, 5), (6, 6, 6), (3, 2, 2)])
def test_apply_matches_sparse_assembly(shape):
    nx, ny, nz = shape
    g = np.random.Generator(np.random.PCG64(nx * 100 + ny * 10 + nz))
    n = nx * ny * nz
    for kappa in (None, np.exp(g.standard_normal(n))):
        desc = W.StencilDesc(nx=nx, ny=ny, nz=nz, h=0.1, diff=0.3, kappa=kappa,
                             adv=(1.5, -2.0, 0.7), reaction=g.uniform(-1, 0, n))
        S = operators.stencil_sparse(desc)
        u = g.standard_normal(n)
        assert np.allclose(operators.stencil_apply(desc, u), S @ u, rtol=1e-14, atol=1e-11)


def test_pure_diffusion_symmetric_and_kills_constants():
    pr = W.diffusion3d_problem(5, 1, 1e-3, seed=3)
    desc = pr.op
    A = operators.dense(desc)
    assert np.allclose(A, A.T, rtol=0, atol=1e-9)
    ones = np.ones(desc.n)
    assert np.allclose(operators.stencil_apply(desc, ones), desc.reaction, rtol=1e-12, atol=1e-9)


def test_csr_apply():
    c = W.csr_from_random_pattern(50, 4, 6, seed=3)
    M = np.zeros((50, 50))
    for i in range(50):
        for k in range(c.rowptr[i], c.rowptr[i + 1]):
            M[i, c.col[k]] += c.val[k]
    u = np.random.Generator(np.random.PCG64(1)).standard_normal(50)
    assert np.allclose(operators.make_apply(c)(u), M @ u, rtol=1e-14, atol=1e-14)


def _const2d(side, r0, diff=1e-2, adv=10.0):
    return W.StencilDesc(nx=side, ny=side, nz=1, h=1.0 / side, diff=diff, adv=(adv, adv, 0.0),
                         reaction=np.full(side * side, r0))


def test_dft_eigenvalues_equal_matrix_eigenvalues_2d():
    desc = _const2d(8, -0.4)
    lam = np.sort_complex(spectral.eigenvalues(desc).ravel())
    ev = np.sort_complex(np.linalg.eigvals(operators.dense(desc)))
    # match as multisets: greedy nearest matching
    ev = list(ev)
    for l in lam:
        k = int(np.argmin([abs(l - e) for e in ev]))
        assert abs(l - ev[k]) <= 1e-9 * max(1.0, abs(l))
        ev.pop(k)


def test_dft_eigenvalues_equal_matrix_eigenvalues_3d():
    n = 4
    desc = W.StencilDesc(nx=n, ny=n, nz=n, h=1.0 / n, kappa=np.full(n ** 3, 1.7),
                         reaction=np.full(n ** 3, -2.0))
    lam = np.sort(spectral.eigenvalues(desc).real.ravel())
    ev = np.sort(np.linalg.eigvalsh(operators.dense(desc)))
    assert np.allclose(lam, ev, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("p", [0, 1, 3])
def test_dft_equals_dense_theorem1(p):
    desc = _const2d(12, -0.3)
    g = np.random.Generator(np.random.PCG64(p))
    vecs = [g.standard_normal(desc.n) for _ in range(p + 1)]
    tau = 0.02
    ref = augmented.phi_combination_dense(operators.dense(desc), tau, vecs)
    got = spectral.phi_combination_fft(desc, tau, vecs)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_dft_equals_dense_3d():
    pr = W.diffusion3d_problem(6, 2, 2e-3, seed=5, constant=(1.3, -2.5))
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
