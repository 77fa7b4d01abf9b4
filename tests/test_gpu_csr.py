"""GPU parity of the general sparse (CSR) operator path against the oracle.

The CSR path takes two phases per Krylov step (elementwise formation, then
the sparse product with the inner products).  Checked: the first-substep IOP
basis and H against the oracle's Algorithm 2; solves against the dense
Theorem-1 result (the 2-D stencil assembled as CSR, random banded matrices,
FP64 and mixed, IOP and full window); the 512^2 stencil as CSR against the
full-Arnoldi oracle; and an out-of-range column index, which the product's
bounds checks read as zero (the same as dropping that entry).
"""

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import augmented, operators
from oracle.arnoldi import phi_combination_arnoldi
from oracle.iop import iop_basis as oracle_iop

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _csr_desc(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return W.CsrDesc(n=M.shape[0], rowptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32),
                     val=M.data.astype(np.float64))


def _solve(desc, tau, vecs, precision="fp64", tol=1e-8, q=2, **kw):
    import paper_1804_05126_amd as K
    op = K.Operator.from_desc(desc, precision=precision)
    w, st, status = K.phi_combination(op, tau, to_dev(vecs), tol=tol, q=q, **kw)
    return w.cpu().numpy(), st


def _random_banded(n, seed, scale):
    d = W.csr_from_random_pattern(n, per_row=6, band=40, seed=seed)
    return W.CsrDesc(n=d.n, rowptr=d.rowptr, col=d.col, val=d.val * scale)


def test_iop_basis_csr_matches_oracle():
    import paper_1804_05126_amd as K
    desc = _random_banded(2000, 5, 10.0)
    vecs = W.random_vectors(2000, 3, seed=6)
    p, m, q = 3, 20, 2
    announce("iop csr n=2000 p=3 q=2 m=20")
    op = K.Operator.from_desc(desc)
    basis, H, j, beta, nu = K.iop_basis(op, to_dev(vecs), m, q)
    nu_o, mu_o = augmented.b_norm_scaling(vecs)
    Vo, Ho, jo, bdo, beta_o = oracle_iop(operators.make_apply(desc), [vecs[p - c] for c in range(p)], nu_o,
                                         vecs[0], mu_o * augmented.trailing_entries(p, 0.0), m, q)
    assert nu == nu_o and j == jo and not bdo
    assert beta == pytest.approx(beta_o, rel=1e-13)
    assert np.max(np.abs(H.cpu().numpy() - Ho)) <= 1e-9 * np.max(np.abs(Ho))
    assert np.max(np.abs(basis.cpu().numpy() - Vo)) <= 1e-8


@pytest.mark.parametrize("q", [2, 0])
def test_csr_stencil_48_vs_dense(q):
    pr = W.adr2d_problem(48, 2, 1e-2, seed=48)
    desc = _csr_desc(operators.stencil_sparse(pr.op))
    announce(f"csr (2-D stencil 48^2) q={q} vs dense")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(desc, pr.tau, pr.vectors, q=q)
    assert rel(got, ref) <= 1e-8


@pytest.mark.parametrize("n,p,tau,seed", [(1500, 2, 0.2, 1), (1200, 4, 0.5, 2), (777, 0, 1.0, 3)])
def test_csr_random_vs_dense(n, p, tau, seed):
    desc = _random_banded(n, seed, 2.0)
    vecs = W.random_vectors(n, p, seed=seed + 100)
    announce(f"csr random n={n} p={p} tau={tau} vs dense")
    ref = augmented.phi_combination_dense(operators.dense(desc), tau, vecs)
    got, st = _solve(desc, tau, vecs)
    assert rel(got, ref) <= 1e-8


def test_csr_mixed_vs_dense():
    desc = _random_banded(1500, 9, 2.0)
    vecs = W.random_vectors(1500, 2, seed=10)
    announce("csr mixed n=1500")
    ref = augmented.phi_combination_dense(operators.dense(desc), 0.2, vecs)
    got, st = _solve(desc, 0.2, vecs, precision="mixed", tol=1e-6)
    assert rel(got, ref) <= 1e-5


def test_csr_out_of_range_column_reads_zero():
    desc = _random_banded(900, 12, 2.0)
    col = desc.col.copy()
    k = int(desc.rowptr[450]) + 1             # an off-diagonal entry of row 450
    col[k] = 10 ** 6                           # outside [0, n)
    bad = W.CsrDesc(n=desc.n, rowptr=desc.rowptr, col=col, val=desc.val)
    val = desc.val.copy()
    val[k] = 0.0
    dropped = W.CsrDesc(n=desc.n, rowptr=desc.rowptr, col=desc.col, val=val)
    vecs = W.random_vectors(900, 2, seed=13)
    announce("csr with one column index out of range")
    ref = augmented.phi_combination_dense(operators.dense(dropped), 0.3, vecs)
    got, st = _solve(bad, 0.3, vecs)
    assert rel(got, ref) <= 1e-8


def test_csr_stencil_512_vs_arnoldi():
    pr = W.cfg2(512, 1e-3)
    desc = _csr_desc(operators.stencil_sparse(pr.op))
    announce("csr (2-D stencil 512^2) p=3 tau=1e-3 vs Arnoldi oracle")
    got, st = _solve(desc, pr.tau, pr.vectors)
    ref = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-11, m=64)
    announce(f"  stats {st}")
    assert rel(got, ref) <= 1e-8
