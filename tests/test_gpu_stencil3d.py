"""GPU parity of the 7-point (3-D) operator path against the oracle.

The 3-D variable-coefficient operator (and the 2-D 5-point operator with a
diffusivity field, which runs on the same marching pass with nz = 1) is
checked: the first-substep IOP basis and H against the oracle's Algorithm 2;
whole solves against the dense Theorem-1 result for N <= 4096, against the
full-Arnoldi oracle for ragged mid-size boxes (several z chunks, partial x and
y tiles), and at the full 256^3 size against the DFT closed form
(constant coefficients) and, with the seeded variable field, through
linearity and the FP64 / mixed agreement.  FP64 at tol 1e-8 must be within
1e-8; mixed at tol 1e-6 within 1e-5 (relative 2-norm error).
"""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators, spectral
from oracle.arnoldi import phi_combination_arnoldi
from oracle.iop import iop_basis as oracle_iop

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _field3d(g, nx, ny, nz, sigma=0.5):
    """kappa = 7-point box average of exp(N(0, sigma^2)) on a periodic box."""
    f = np.exp(g.normal(0.0, sigma, size=(nz, ny, nx)))
    s = f.copy()
    for ax in range(3):
        s += np.roll(f, 1, axis=ax) + np.roll(f, -1, axis=ax)
    return (s / 7.0).reshape(-1)


def _problem(nx, ny, nz, p, tau, seed, *, kappa=True, adv=(0.0, 0.0, 0.0), diff=0.0, tol=1e-8):
    g = np.random.Generator(np.random.PCG64(seed))
    n = nx * ny * nz
    kap = _field3d(g, nx, ny, nz) if kappa else None
    r = g.uniform(-5.0, 0.0, n)
    desc = W.StencilDesc(nx=nx, ny=ny, nz=nz, h=1.0 / max(nx, ny, nz), diff=diff, kappa=kap,
                         adv=adv, reaction=r)
    vecs = [g.standard_normal(n) for _ in range(p + 1)]
    return W.Problem(name=f"s3d_{nx}x{ny}x{nz}", op=desc, tau=tau, vectors=vecs, tol=tol)


def _solve(pr, precision="fp64", **kw):
    import paper_1804_05126_amd as K
    op = K.Operator.from_desc(pr.op, precision=precision)
    args = dict(tol=pr.tol, m_init=pr.m_init, q=pr.q)
    args.update(kw)
    w, st, status = K.phi_combination(op, pr.tau, to_dev(pr.vectors), **args)
    return w.cpu().numpy(), st


@pytest.mark.parametrize("nx,ny,nz,p,q,m", [(12, 10, 9, 2, 2, 20), (70, 6, 5, 3, 3, 16),
                                            (16, 16, 16, 1, 2, 24), (33, 9, 1, 2, 2, 18)])
def test_iop_basis_3d_matches_oracle(nx, ny, nz, p, q, m):
    import paper_1804_05126_amd as K
    pr = _problem(nx, ny, nz, p, 1.0, seed=nx * 100 + ny + nz)
    vecs = pr.vectors
    announce(f"iop 3d {nx}x{ny}x{nz} p={p} q={q} m={m}")
    op = K.Operator.from_desc(pr.op)
    basis, H, j, beta, nu = K.iop_basis(op, to_dev(vecs), m, q)
    nu_o, mu_o = augmented.b_norm_scaling(vecs)
    Vo, Ho, jo, bdo, beta_o = oracle_iop(operators.make_apply(pr.op), [vecs[p - c] for c in range(p)], nu_o,
                                         vecs[0], mu_o * augmented.trailing_entries(p, 0.0), m, q)
    assert nu == nu_o
    assert j == jo and not bdo
    assert beta == pytest.approx(beta_o, rel=1e-13)
    Hd = H.cpu().numpy()
    assert np.max(np.abs(Hd - Ho)) <= 1e-9 * np.max(np.abs(Ho))
    Vd = basis.cpu().numpy()
    assert np.max(np.abs(Vd - Vo)) <= 1e-8, np.max(np.abs(Vd - Vo))


@pytest.mark.parametrize("nx,ny,nz,p,tau,kappa,adv", [
    (12, 10, 9, 2, 2e-3, True, (0.0, 0.0, 0.0)),
    (16, 16, 16, 1, 1e-3, True, (0.0, 0.0, 0.0)),
    (7, 5, 3, 3, 5e-3, False, (3.0, -2.0, 1.0)),
    (9, 11, 13, 4, 2e-3, True, (1.0, 0.5, -2.0)),
    (40, 33, 1, 2, 1e-3, True, (0.0, 0.0, 0.0)),     # 5-point with a diffusivity field
    (3, 2, 2, 0, 1e-2, True, (0.0, 0.0, 0.0)),       # tiny box, axes of length 2
])
def test_3d_vs_dense(nx, ny, nz, p, tau, kappa, adv):
    pr = _problem(nx, ny, nz, p, tau, seed=7 * nx + ny + nz, kappa=kappa, adv=adv,
                  diff=0.0 if kappa else 0.7)
    announce(f"3d dense {nx}x{ny}x{nz} p={p} tau={tau} kappa={kappa} adv={adv}")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(pr)
    assert rel(got, ref) <= 1e-8, (rel(got, ref), st)


def test_3d_full_window_q0_vs_dense():
    pr = _problem(12, 10, 9, 2, 2e-3, seed=91)
    pr.q = 0
    announce("3d 12x10x9 q=0 vs dense")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(pr)
    assert rel(got, ref) <= 1e-8


def test_3d_mixed_vs_dense():
    pr = _problem(16, 16, 16, 2, 1e-3, seed=77, tol=1e-6)
    announce("3d mixed 16^3")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(pr, precision="mixed")
    assert rel(got, ref) <= 1e-5


@pytest.mark.parametrize("nx,ny,nz,p,tau", [(70, 6, 37, 2, 1e-3), (64, 12, 33, 3, 3e-3)])
def test_3d_ragged_chunks_vs_arnoldi(nx, ny, nz, p, tau):
    pr = _problem(nx, ny, nz, p, tau, seed=nx + ny + nz)
    announce(f"3d ragged {nx}x{ny}x{nz} p={p} tau={tau} vs Arnoldi")
    ref = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-12)
    got, st = _solve(pr)
    assert rel(got, ref) <= 1e-8


def test_cfg3_shape_64_vs_arnoldi():
    pr = W.diffusion3d_problem(64, 2, 1e-3, seed=1003, tol=1e-8)
    announce("64^3 variable kappa p=2 tau=1e-3 vs Arnoldi oracle")
    got, st = _solve(pr)
    ref = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-11, m=64)
    assert rel(got, ref) <= 1e-8
    got_m, _ = _solve(W.diffusion3d_problem(64, 2, 1e-3, seed=1003, tol=1e-6), precision="mixed")
    assert rel(got_m, ref) <= 1e-5


# ----------------------------------------------------------- full size 256^3

@pytest.mark.parametrize("precision,tol,bound", [("fp64", 1e-8, 1e-8), ("mixed", 1e-6, 1e-5)])
def test_256_constant_coefficients_vs_dft(precision, tol, bound):
    pr = W.diffusion3d_problem(256, 2, 1e-3, seed=1003, tol=tol, constant=(1.0, -2.5))
    announce(f"256^3 constant kappa/r {precision} vs DFT")
    got, st = _solve(pr, precision=precision)
    announce(f"  stats {st}")
    ref = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    assert rel(got, ref) <= bound


def test_256_cfg3_linearity_and_mixed_agreement():
    import torch
    import paper_1804_05126_amd as K
    pr = W.cfg3()
    announce("256^3 cfg3 (variable kappa) linearity, FP64 vs mixed")
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    a, st, _ = K.phi_combination(op, pr.tau, vecs, tol=1e-8)
    announce(f"  fp64 stats {st}")
    b, _, _ = K.phi_combination(op, pr.tau, [-3.0 * v for v in vecs], tol=1e-8)
    assert float(torch.linalg.norm(b + 3.0 * a) / torch.linalg.norm(a)) <= 1e-8
    opm = K.Operator.from_desc(pr.op, precision="mixed")
    c, stm, _ = K.phi_combination(opm, pr.tau, vecs, tol=1e-6)
    announce(f"  mixed stats {stm}")
    assert float(torch.linalg.norm(c - a) / torch.linalg.norm(a)) <= 1e-5
