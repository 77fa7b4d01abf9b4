"""End-to-end GPU parity of kiops_phi_combination against the oracle.

FP64 results at tol 1e-8 must be within 1e-8 relative 2-norm error of the
exact result (dense Theorem 1 for small N, full-Arnoldi Krylov for larger N,
the DFT closed form for constant-coefficient grids up to the full 2048^2
size); mixed precision at tol 1e-6 within 1e-5.  Edge cases: tau = 0, p = 0,
in-place output, ragged tiles, tiny grids, forced substepping (small m_max),
non-finite input, substep limit.
"""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators, spectral
from oracle.arnoldi import phi_combination_arnoldi
from oracle.kiops import kiops as oracle_kiops

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _solve(pr, precision="fp64", **kw):
    import paper_1804_05126_amd as K
    op = K.Operator.from_desc(pr.op, precision=precision)
    vecs = to_dev(pr.vectors)
    args = dict(tol=pr.tol, m_init=pr.m_init, q=pr.q)
    args.update(kw)
    w, st, status = K.phi_combination(op, pr.tau, vecs, **args)
    return w.cpu().numpy(), st


def test_cfg1_matches_dense_and_oracle_trace():
    pr = W.cfg1()
    announce("cfg1 32x32 p=2 tau=1e-2")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(pr)
    assert rel(got, ref) <= 1e-8
    wk, sk = oracle_kiops(operators.make_apply(pr.op), pr.tau, pr.vectors, tol=pr.tol, m_init=pr.m_init)
    # same algorithm on both sides: the same decisions on this problem
    assert st["substeps"] == sk.substeps
    assert st["matvecs"] >= sk.matvecs
    assert st["m_last"] == sk.m_last
    assert st["rejections"] == sk.rejections


@pytest.mark.parametrize("p", [0, 1, 3, 4, 8])
def test_dense_parity_various_p(p):
    pr = W.adr2d_problem(24, p, 2e-2, seed=100 + p)
    announce(f"24x24 p={p}")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(pr)
    assert rel(got, ref) <= 1e-8


@pytest.mark.parametrize("nx,ny,p,tau", [(100, 37, 3, 5e-3), (7, 5, 2, 0.3), (65, 17, 1, 1e-2),
                                         (130, 48, 2, 2e-3)])
def test_ragged_grids_vs_dense_or_arnoldi(nx, ny, p, tau):
    g = np.random.Generator(np.random.PCG64(nx * 1000 + ny))
    n = nx * ny
    desc = W.StencilDesc(nx=nx, ny=ny, nz=1, h=1.0 / max(nx, ny), diff=1e-2, adv=(10.0, 3.0, 0.0),
                         reaction=g.uniform(-1, 0, n))
    vecs = [g.standard_normal(n) for _ in range(p + 1)]
    pr = W.Problem(name="ragged", op=desc, tau=tau, vectors=vecs)
    announce(f"ragged {nx}x{ny} p={p} tau={tau}")
    if n <= 4096:
        ref = augmented.phi_combination_dense(operators.dense(desc), tau, vecs)
    else:
        ref = phi_combination_arnoldi(operators.make_apply(desc), tau, vecs, tol_o=1e-12)
    got, st = _solve(pr)
    assert rel(got, ref) <= 1e-8


@pytest.mark.parametrize("side,p,tau", [(24, 3, 2e-2), (40, 2, 5e-3)])
def test_full_window_q0_vs_dense(side, p, tau):
    pr = W.adr2d_problem(side, p, tau, seed=500 + side, q=0)
    announce(f"{side}x{side} p={p} q=0 (full Arnoldi) vs dense")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(pr)
    assert rel(got, ref) <= 1e-8


def test_full_window_q0_512_vs_arnoldi_and_q2():
    pr = W.cfg2(512, 1e-3, q=0)
    announce("512^2 p=3 tau=1e-3 q=0 vs Arnoldi oracle and the q=2 solve")
    got, st = _solve(pr)
    ref = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-11, m=64)
    assert rel(got, ref) <= 1e-8
    got2, st2 = _solve(W.cfg2(512, 1e-3, q=2))
    announce(f"  q=0 stats {st}; q=2 stats {st2}")
    assert rel(got2, ref) <= 1e-8


def test_small_mmax_forces_step_size_control():
    pr = W.adr2d_problem(48, 2, 5e-2, seed=31)
    announce("48x48 m_max=24 (tau control)")
    ref = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-12)
    got, st = _solve(pr, m_max=24)
    assert st["substeps"] > 1
    assert rel(got, ref) <= 1e-8
    wk, sk = oracle_kiops(operators.make_apply(pr.op), pr.tau, pr.vectors, tol=1e-8, m_max=24)
    assert abs(st["substeps"] - sk.substeps) <= max(1, sk.substeps // 10)


def test_tau_zero_and_in_place():
    import torch
    import paper_1804_05126_amd as K
    pr = W.cfg1()
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    w, st, _ = K.phi_combination(op, 0.0, vecs)
    assert torch.equal(w, vecs[0]) and st["matvecs"] == 0
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    b0 = vecs[0].clone()
    inplace = [b0] + vecs[1:]
    w2, st2, _ = K.phi_combination(op, pr.tau, inplace, tol=1e-8, out=b0)
    assert rel(b0.cpu().numpy(), ref) <= 1e-8


def test_deterministic_bitwise():
    import torch
    import paper_1804_05126_amd as K
    pr = W.adr2d_problem(200, 3, 1e-2, seed=41)
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    a, _, _ = K.phi_combination(op, pr.tau, vecs)
    b, _, _ = K.phi_combination(op, pr.tau, vecs)
    assert torch.equal(a, b)


def test_mixed_precision_cfg1():
    pr = W.cfg1()
    pr.tol = 1e-6
    announce("cfg1 mixed")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(pr, precision="mixed", tol=1e-6)
    assert rel(got, ref) <= 1e-5


def test_nonfinite_input_reports_status():
    import paper_1804_05126_amd as K
    pr = W.cfg1()
    vecs = [v.copy() for v in pr.vectors]
    vecs[0][17] = np.nan
    op = K.Operator.from_desc(pr.op)
    _, st, status = K.phi_combination(op, pr.tau, to_dev(vecs), check=False)
    assert status == 4     # KIOPS_ERR_NONFINITE


def test_substep_limit_reports_not_converged():
    import paper_1804_05126_amd as K
    pr = W.adr2d_problem(64, 2, 0.1, seed=5)
    op = K.Operator.from_desc(pr.op)
    _, st, status = K.phi_combination(op, pr.tau, to_dev(pr.vectors), m_min=10, m_max=10,
                                      max_substeps=2, check=False)
    assert status == 5     # KIOPS_ERR_NOT_CONVERGED
    assert st["substeps"] == 2 and 0.0 < st["t_reached"] < pr.tau


# ----------------------------------------------------------- full sizes

def test_512_vs_arnoldi():
    pr = W.cfg2(512, 1e-3)
    announce("512^2 p=3 tau=1e-3 vs Arnoldi oracle")
    got, st = _solve(pr)
    ref = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-11, m=64)
    assert rel(got, ref) <= 1e-8


@pytest.mark.parametrize("tau", W.cfg2_tau_grid())
def test_2048_constant_reaction_vs_dft(tau):
    # every step size of the benchmark sweep, including the two heaviest
    # (tau = 10^-1.5 and 0.1: many substeps and rejections at m_max)
    pr = W.cfg2(2048, tau, constant_reaction=-0.5)
    announce(f"2048^2 p=3 tau={tau:.4g} constant r vs DFT")
    got, st = _solve(pr)
    ref = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    err = rel(got, ref)
    announce(f"  rel err {err:.3e}; stats matvecs {st['matvecs']} substeps {st['substeps']} "
             f"rejections {st['rejections']}")
    assert err <= 1e-8


@pytest.mark.parametrize("tau", [1e-3, 1e-1])
def test_2048_constant_reaction_mixed_vs_dft(tau):
    pr = W.cfg2(2048, tau, constant_reaction=-0.5)
    announce(f"2048^2 p=3 tau={tau:.4g} constant r, mixed precision, vs DFT")
    got, st = _solve(pr, precision="mixed", tol=1e-6)
    ref = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    err = rel(got, ref)
    announce(f"  rel err {err:.3e}; stats matvecs {st['matvecs']} substeps {st['substeps']}")
    assert err <= 1e-5


def test_2048_linearity_variable_reaction():
    import torch
    import paper_1804_05126_amd as K
    pr = W.cfg2(2048, 1e-3)
    announce("2048^2 linearity")
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    a, _, _ = K.phi_combination(op, pr.tau, vecs)
    b, _, _ = K.phi_combination(op, pr.tau, [2.0 * v for v in vecs])
    assert float(torch.linalg.norm(b - 2.0 * a) / torch.linalg.norm(a)) <= 1e-8
