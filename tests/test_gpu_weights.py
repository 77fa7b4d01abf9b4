"""GPU parity of the general stencil form (per-cell weights [5|7][N]) against
the oracle: whole solves against the dense exact result (Theorem 1) in 2-D
and 3-D, FP64 and mixed, IOP window and full window; weights written from the
coefficient form against the coefficient-form operator's own pass; y = A x by
kiops_apply; a batch of weights operators against single solves; argument
checks."""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _weights_problem(nx, ny, nz, p, tau, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    n = nx * ny * nz
    nw = 5 if nz == 1 else 7
    Wt = g.standard_normal((nw, n))
    Wt[0] -= 4.0                       # a decaying diagonal
    desc = W.StencilDesc(nx=nx, ny=ny, nz=nz, h=1.0, weights=Wt)
    vecs = [g.standard_normal(n) for _ in range(p + 1)]
    return W.Problem(name="weights", op=desc, tau=tau, vectors=vecs)


def _solve(pr, precision="fp64", **kw):
    import paper_1804_05126_amd as K
    op = K.Operator.from_desc(pr.op, precision=precision)
    args = dict(tol=pr.tol if precision == "fp64" else 1e-6, m_init=pr.m_init, q=pr.q)
    args.update(kw)
    w, st, status = K.phi_combination(op, pr.tau, to_dev(pr.vectors), **args)
    return w.cpu().numpy(), st


@pytest.mark.parametrize("nx,ny,nz,p,tau,q", [(24, 20, 1, 2, 0.1, 2), (37, 11, 1, 3, 0.05, 0),
                                              (10, 9, 8, 2, 0.1, 2), (12, 7, 5, 4, 0.05, 3)])
def test_weights_vs_dense(nx, ny, nz, p, tau, q):
    pr = _weights_problem(nx, ny, nz, p, tau, seed=nx * 1000 + ny * 10 + nz)
    announce(f"weights {nx}x{ny}x{nz} p={p} tau={tau} q={q}")
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    got, st = _solve(pr, q=q)
    assert st["pass_kind"] == 5
    assert rel(got, ref) <= 1e-8
    gm, _ = _solve(pr, precision="mixed", q=q)
    assert rel(gm, ref) <= 1e-5


def test_weights_from_coefficients_match_the_7pt_pass():
    g = np.random.Generator(np.random.PCG64(77))
    nx, ny, nz, h = 20, 16, 12, 1.0 / 20
    n = nx * ny * nz
    kap = g.uniform(0.5, 2.0, n)
    adv = (1.0, -2.0, 0.5)
    r = g.uniform(-3, 0, n)
    coef = W.StencilDesc(nx=nx, ny=ny, nz=nz, h=h, kappa=kap, adv=adv, reaction=r)
    K3 = kap.reshape(nz, ny, nx)
    Wt = np.zeros((7, n))
    Wt[0] = r
    for d, axis in enumerate((2, 1, 0)):
        kp = (0.5 * (K3 + np.roll(K3, -1, axis=axis))).reshape(-1)
        km = (0.5 * (K3 + np.roll(K3, 1, axis=axis))).reshape(-1)
        Wt[0] -= (kp + km) / h ** 2
        Wt[1 + 2 * d] = kp / h ** 2 - adv[d] / (2 * h)
        Wt[2 + 2 * d] = km / h ** 2 + adv[d] / (2 * h)
    gen = W.StencilDesc(nx=nx, ny=ny, nz=nz, h=h, weights=Wt)
    vecs = [g.standard_normal(n) for _ in range(3)]
    announce("weights written from a kappa field vs the 7-point pass")
    a, _ = _solve(W.Problem(name="coef", op=coef, tau=1e-3, vectors=vecs))
    b, st = _solve(W.Problem(name="gen", op=gen, tau=1e-3, vectors=vecs))
    assert st["pass_kind"] == 5
    assert rel(b, a) <= 1e-8


def test_weights_apply_and_batch():
    import torch
    import paper_1804_05126_amd as K
    pr = _weights_problem(30, 17, 1, 2, 0.05, seed=5)
    op = K.Operator.from_desc(pr.op)
    x = np.random.default_rng(6).standard_normal(op.n)
    y = K.apply(op, to_dev([x])[0])
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), operators.make_apply(pr.op)(x)) <= 1e-13
    announce("batch of 6 weights operators vs single solves")
    prs = [_weights_problem(16 + 4 * i, 12, 1, 1 + i % 3, 0.02 * (i + 1), seed=50 + i) for i in range(6)]
    probs = []
    for q in prs:
        o = K.Operator.from_desc(q.op)
        probs.append(dict(op=o, tau=q.tau, vectors=to_dev(q.vectors), tol=1e-8, m_init=10, q=2))
    ws, stats, status, plan = K.phi_batch(probs, group_size=8)
    assert status == 0
    for q, pb, w in zip(prs, probs, ws):
        ref = augmented.phi_combination_dense(operators.dense(q.op), q.tau, q.vectors)
        assert rel(w.cpu().numpy(), ref) <= 1e-8


def test_weights_argument_checks():
    import torch
    import paper_1804_05126_amd as K
    n = 8 * 8
    wts = torch.zeros(5 * n, dtype=torch.float64, device="cuda")
    kap = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        K.Operator("stencil2d", nx=8, ny=8, h=1.0, weights=wts, kappa=kap)
    with pytest.raises(Exception):
        K.Operator("stencil2d", nx=8, ny=8, h=1.0, weights=wts, diff=1.0)
    with pytest.raises(Exception):
        K.Operator("stencil2d", nx=8, ny=8, h=1.0, weights=torch.zeros(4 * n, dtype=torch.float64, device="cuda"))
