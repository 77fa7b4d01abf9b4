"""GPU parity of the two device building blocks against the oracle:

* the small exponential (Section 3.3.1) on projected matrices H~ taken from
  the oracle's own IOP of the 32x32 ADR problem, over a range of tau that
  exercises every Pade degree and the squaring;
* Algorithm 2 (basis V and Hessenberg H) on several grids, windows and p,
  compared element by element with the oracle's IOP.
"""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators
from oracle.expm import expm
from oracle.iop import iop_basis as oracle_iop

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _oracle_H(m=128):
    pr = W.cfg1()
    p = pr.p
    nu, mu = augmented.b_norm_scaling(pr.vectors)
    V, H, j, bd, beta = oracle_iop(operators.make_apply(pr.op), [pr.vectors[p - c] for c in range(p)], nu,
                                   pr.vectors[0], mu * augmented.trailing_entries(p, 0.0), m, 2)
    return H


@pytest.mark.parametrize("j", [1, 4, 15, 16, 47, 100, 128])
@pytest.mark.parametrize("tau", [1e-5, 1e-3, 1e-2, 6e-2])
def test_small_expm_matches_oracle(j, tau):
    import torch
    import paper_1804_05126_amd as K
    H = _oracle_H()
    n = j + 1
    Ht = np.zeros((n, n))
    Ht[:j, :j] = H[:j, :j]
    Ht[0, j] = 1.0
    announce(f"small_expm j={j} tau={tau} norm={np.linalg.norm(tau * Ht, 1):.3g}")
    F = K.small_expm(torch.as_tensor(Ht, device="cuda"), tau).cpu().numpy()
    ref = expm(tau * Ht)
    scale = max(1.0, np.linalg.norm(ref, 1))
    assert np.linalg.norm(F - ref, 1) <= 1e-11 * scale
    # the two entries the solver consumes: first column and F(j, j+1)
    assert np.linalg.norm(F[:j, 0] - ref[:j, 0]) <= 1e-11 * max(1.0, np.linalg.norm(ref[:j, 0]))


def test_small_expm_random_dense():
    import torch
    import paper_1804_05126_amd as K
    g = np.random.Generator(np.random.PCG64(8))
    for n, sc in ((1, 0.3), (2, 3.0), (33, 0.5), (64, 20.0), (129, 4.0)):
        M = sc * g.standard_normal((n, n)) / np.sqrt(n) - sc * np.eye(n)
        F = K.small_expm(torch.as_tensor(M, device="cuda"), 1.0).cpu().numpy()
        ref = expm(M)
        assert np.linalg.norm(F - ref, 1) <= 1e-11 * max(1.0, np.linalg.norm(ref, 1)), (n, sc)


CASES = [
    # (nx, ny, p, q, m, seed)
    (32, 32, 2, 2, 30, 1001),
    (70, 37, 3, 2, 25, 11),
    (64, 16, 0, 2, 20, 12),
    (130, 50, 4, 3, 24, 13),
    (20, 24, 1, 1, 12, 14),
    (96, 80, 2, 4, 28, 15),
    (5, 3, 2, 2, 10, 16),
    (40, 30, 2, 0, 24, 17),     # q = 0: full window
    (70, 37, 3, 0, 30, 18),
]


@pytest.mark.parametrize("nx,ny,p,q,m,seed", CASES)
def test_iop_basis_matches_oracle(nx, ny, p, q, m, seed):
    import paper_1804_05126_amd as K
    g = np.random.Generator(np.random.PCG64(seed))
    n = nx * ny
    desc = W.StencilDesc(nx=nx, ny=ny, nz=1, h=1.0 / max(nx, ny), diff=1e-2, adv=(10.0, -7.0, 0.0),
                         reaction=g.uniform(-1, 0, n))
    vecs = [g.standard_normal(n) for _ in range(p + 1)]
    announce(f"iop {nx}x{ny} p={p} q={q} m={m}")
    op = K.Operator.from_desc(desc)
    basis, H, j, beta, nu = K.iop_basis(op, to_dev(vecs), m, q)
    nu_o, mu_o = augmented.b_norm_scaling(vecs)
    Vo, Ho, jo, bdo, beta_o = oracle_iop(operators.make_apply(desc), [vecs[p - c] for c in range(p)], nu_o,
                                         vecs[0], mu_o * augmented.trailing_entries(p, 0.0), m, q)
    assert nu == nu_o
    assert j == jo and not bdo
    assert beta == pytest.approx(beta_o, rel=1e-13)
    Hd = H.cpu().numpy()
    assert np.max(np.abs(Hd - Ho)) <= 1e-9 * np.max(np.abs(Ho))
    Vd = basis.cpu().numpy()
    assert np.max(np.abs(Vd - Vo)) <= 1e-8, np.max(np.abs(Vd - Vo))
    assert np.max(np.abs(Vd[:4] - Vo[:4])) <= 1e-12


def test_iop_breakdown_zero_operator():
    import paper_1804_05126_amd as K
    g = np.random.Generator(np.random.PCG64(3))
    desc = W.StencilDesc(nx=40, ny=30, nz=1, h=0.1, diff=0.0, adv=(0.0, 0.0, 0.0), reaction=None)
    vecs = [g.standard_normal(1200) for _ in range(2)]
    op = K.Operator.from_desc(desc)
    basis, H, j, beta, nu = K.iop_basis(op, to_dev(vecs), 10, 2)
    assert j == 2      # Krylov space of dimension p + 1 = 2, inside the window
