"""GPU parity of several output times in one integration (Algorithm 1 with an
array of times; Algorithm 3 writes each intermediate output from the basis of
the substep that contains it), Task II and Task I, against the oracle's dense
route at every time."""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _solve_times(pr, times, task, precision="fp64", tol=None, **kw):
    import paper_1804_05126_amd as K
    op = K.Operator.from_desc(pr.op, precision=precision)
    outs, st, status = K.phi_combination_times(op, times, to_dev(pr.vectors), task=task,
                                               tol=tol if tol is not None else pr.tol, **kw)
    assert status == 0
    return [o.cpu().numpy() for o in outs], st


@pytest.mark.parametrize("task", [2, 1])
def test_times_2d_vs_dense(task):
    pr = W.adr2d_problem(40, 2, 2e-2, seed=6001)
    times = [2e-3, 7e-3, 1.1e-2, 2e-2]
    announce(f"times 2d 40^2 task {task}")
    got, st = _solve_times(pr, times, task)
    ref = augmented.phi_combination_times(operators.dense(pr.op), times, pr.vectors, task=task)
    for t, g, r in zip(times, got, ref):
        assert rel(g, r) <= 1e-8, (t, rel(g, r))
    announce(f"  stats: substeps {st['substeps']} expms {st['expms']}")


def test_many_times_in_one_substep_3d():
    pr = W.diffusion3d_problem(12, 3, 2e-3, seed=6002, tol=1e-8)
    times = list(np.geomspace(1e-5, 2e-3, 12))
    announce("times 3d 12^3, 12 times")
    got, st = _solve_times(pr, times, 2)
    ref = augmented.phi_combination_times(operators.dense(pr.op), times, pr.vectors, task=2)
    for t, g, r in zip(times, got, ref):
        assert rel(g, r) <= 1e-8, (t, rel(g, r))
    assert st["expms"] >= 12 - 1           # one small exponential per intermediate output at least


def test_single_time_equals_plain_call():
    import paper_1804_05126_amd as K
    pr = W.adr2d_problem(64, 3, 1e-2, seed=6003)
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    a, _, _ = K.phi_combination(op, pr.tau, vecs)
    (b,), _, _ = K.phi_combination_times(op, [pr.tau], vecs, task=2)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_times_mixed_vs_dense():
    pr = W.adr2d_problem(48, 2, 1e-2, seed=6004, tol=1e-6)
    times = [1e-3, 4e-3, 1e-2]
    got, st = _solve_times(pr, times, 2, precision="mixed")
    ref = augmented.phi_combination_times(operators.dense(pr.op), times, pr.vectors, task=2)
    for t, g, r in zip(times, got, ref):
        assert rel(g, r) <= 1e-5, (t, rel(g, r))


def test_times_rejects_bad_arguments():
    import paper_1804_05126_amd as K
    pr = W.adr2d_problem(32, 1, 1e-2, seed=6005)
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    for times, task in (([2e-3, 1e-3], 2), ([0.0, 1e-3], 2), ([1e-3], 3)):
        with pytest.raises(K.KiopsError) as e:
            K.phi_combination_times(op, times, vecs, task=task)
        assert e.value.status == 1                 # KIOPS_ERR_INVALID_ARG
