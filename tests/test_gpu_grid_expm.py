"""GPU checks of the attempt's small exponential spread over the grid.

exp(tau H~) (Section 3.3.1, Eq. (37)) normally runs on workgroup 0 for small
bases and as stages of products on several workgroups from a padded size of
96 on; KIOPS_GRID_EXPM moves that threshold (0 = never, 16 = always).  The
staged products are the one-workgroup products tile by tile, so the solution
and every controller decision must be bitwise the same in both modes; with
the grid mode forced the solve must still match the oracle's dense route of
Theorem 1.
"""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu

KEYS = ("matvecs", "expms", "rejections", "substeps", "status")


def _solve(monkeypatch, mode, op, tau, vecs, tol):
    import paper_1804_05126_amd as K
    monkeypatch.setenv("KIOPS_GRID_EXPM", str(mode))
    w, st, status = K.phi_combination(op, tau, vecs, tol=tol)
    assert status == 0
    return w.cpu().numpy(), st


@pytest.mark.parametrize("side,tau,precision", [(128, 1e-2, "fp64"), (96, 3e-2, "mixed")])
def test_grid_expm_bitwise_2d(monkeypatch, side, tau, precision):
    import paper_1804_05126_amd as K
    tol = 1e-8 if precision == "fp64" else 1e-6
    pr = W.adr2d_problem(side, 3, tau, seed=7001, tol=tol)
    op = K.Operator.from_desc(pr.op, precision=precision)
    vecs = to_dev(pr.vectors)
    announce(f"grid expm 2d {side}^2 tau {tau} {precision}")
    w0, s0 = _solve(monkeypatch, 0, op, pr.tau, vecs, tol)
    for mode in (16, 96):
        w, s = _solve(monkeypatch, mode, op, pr.tau, vecs, tol)
        assert np.array_equal(w, w0), mode
        assert all(s[k] == s0[k] for k in KEYS), (mode, {k: (s[k], s0[k]) for k in KEYS})
    announce(f"  products {s0['matvecs']} exponentials {s0['expms']} rejections {s0['rejections']}")


def test_grid_expm_bitwise_3d(monkeypatch):
    import paper_1804_05126_amd as K
    pr = W.diffusion3d_problem(24, 2, 2e-3, seed=7002, tol=1e-8)
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    announce("grid expm 3d 24^3")
    w0, s0 = _solve(monkeypatch, 0, op, pr.tau, vecs, pr.tol)
    w1, s1 = _solve(monkeypatch, 16, op, pr.tau, vecs, pr.tol)
    assert np.array_equal(w1, w0)
    assert all(s1[k] == s0[k] for k in KEYS)


@pytest.mark.parametrize("side,p,tau", [(48, 2, 2e-2), (64, 4, 5e-3)])
def test_grid_expm_forced_vs_dense(monkeypatch, side, p, tau):
    import paper_1804_05126_amd as K
    pr = W.adr2d_problem(side, p, tau, seed=7003 + side)
    op = K.Operator.from_desc(pr.op)
    announce(f"grid expm forced, {side}^2 p {p} vs dense")
    w, st = _solve(monkeypatch, 16, op, pr.tau, to_dev(pr.vectors), pr.tol)
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    assert rel(w, ref) <= 1e-8, (rel(w, ref), st["expms"])


def test_grid_expm_forced_in_batch(monkeypatch):
    import paper_1804_05126_amd as K
    prs = W.cfg4(count=6, seed=7004, precision="fp64", side_range=(16, 64))
    probs = [dict(op=K.Operator.from_desc(pr.op), tau=pr.tau, vectors=to_dev(pr.vectors), tol=pr.tol,
                  m_init=pr.m_init, q=pr.q) for pr in prs]
    announce("grid expm forced in a batch of 6 (groups of 8 workgroups)")
    monkeypatch.setenv("KIOPS_GRID_EXPM", "16")
    ws, stats, status, _ = K.phi_batch(probs, group_size=8)
    assert status == 0
    monkeypatch.setenv("KIOPS_GRID_EXPM", "0")
    ws0, stats0, status0, _ = K.phi_batch(probs, group_size=8)
    assert status0 == 0
    for pr, w, w0, st in zip(prs, ws, ws0, stats):
        assert st["status"] == 0
        assert np.array_equal(w.cpu().numpy(), w0.cpu().numpy()), pr.name
        ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
        assert rel(w.cpu().numpy(), ref) <= 1e-8, pr.name
