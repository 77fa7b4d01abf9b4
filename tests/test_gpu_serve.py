"""GPU parity of the served form (continuous batching in one long-lived launch).

Requests of the served workload's recipe (2-D 5-point and 3-D 7-point
operators, FP64 at tol 1e-8 and mixed at tol 1e-6, p in 1..4) are submitted
while earlier ones are running; each result must match the same request solved
alone (before the server was opened) within its tolerance class, and small
ones the dense Theorem-1 result.  A pool smaller than one request's workspace
is refused with KIOPS_ERR_BUDGET; a request larger than what is free waits
until memory frees up.
"""

import time

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _requests(count, seed):
    reqs = W.cfg5_requests(lam=1000.0, count=count, seed=seed, side2d=(16, 96), side3d=(8, 20))
    return [r.materialize() for r in reqs]


def _inputs(prs):
    import paper_1804_05126_amd as K
    return [(K.Operator.from_desc(pr.op, precision=pr.precision), to_dev(pr.vectors)) for pr in prs]


def _drain(srv, tickets, timeout_s=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        srv.progress()
        for t in tickets:
            if t in out:
                continue
            done, st, w = srv.result(t)
            if done:
                out[t] = (st, w.cpu().numpy())
        assert time.time() - t0 < timeout_s, "served requests did not finish"
    return out


def test_served_mix_matches_alone_and_dense():
    import paper_1804_05126_amd as K
    prs = _requests(24, seed=5001)
    ins = _inputs(prs)
    announce(f"served: {len(prs)} requests ({sum(p.op.nz > 1 for p in prs)} 3-D)")
    alone = []
    for pr, (op, vecs) in zip(prs, ins):
        w, st, status = K.phi_combination(op, pr.tau, vecs, tol=pr.tol)
        assert status == 0
        alone.append(w.cpu().numpy())
    srv = K.Server(pool_bytes=4 << 30, group_size=16)
    try:
        tickets = []
        for i, (pr, (op, vecs)) in enumerate(zip(prs, ins)):
            tickets.append(srv.submit(op, pr.tau, vecs, tol=pr.tol))
            if i % 3 == 2:
                srv.progress()
        res = _drain(srv, tickets)
    finally:
        srv.close()
    for pr, a, t in zip(prs, alone, tickets):
        st, w = res[t]
        assert st["status"] == 0
        bound = 1e-8 if pr.precision == "fp64" else 1e-5
        assert rel(w, a) <= 2 * bound, (pr.name, rel(w, a))
        if pr.n <= 4096:
            ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
            assert rel(w, ref) <= bound, (pr.name, rel(w, ref))


def test_served_budget_admission():
    import paper_1804_05126_amd as K
    pr_big = W.adr2d_problem(256, 2, 1e-3, seed=5002)
    pr_small = W.adr2d_problem(32, 2, 1e-2, seed=5003)
    op_big, v_big = K.Operator.from_desc(pr_big.op), to_dev(pr_big.vectors)
    op_small, v_small = K.Operator.from_desc(pr_small.op), to_dev(pr_small.vectors)
    ref_big, _, _ = K.phi_combination(op_big, pr_big.tau, v_big)
    ref_small = augmented.phi_combination_dense(operators.dense(pr_small.op), pr_small.tau, pr_small.vectors)
    need = op_big.workspace_bytes(2)
    announce(f"served budget: request needs about {need >> 20} MiB")
    srv = K.Server(pool_bytes=64 << 20, group_size=16)     # smaller than the large request
    try:
        with pytest.raises(K.KiopsError) as e:
            srv.submit(op_big, pr_big.tau, v_big)
        assert e.value.status == 6                          # KIOPS_ERR_BUDGET
        t = srv.submit(op_small, pr_small.tau, v_small)
        res = _drain(srv, [t])
    finally:
        srv.close()
    assert rel(res[t][1], ref_small) <= 1e-8
    # a pool for one large request at a time: the second waits for the first
    srv = K.Server(pool_bytes=int(need * 1.5), group_size=16)
    try:
        t1 = srv.submit(op_big, pr_big.tau, v_big)
        t2 = srv.submit(op_big, pr_big.tau, v_big)
        running, waiting = srv.progress()
        announce(f"  after two submissions: running {running}, waiting {waiting}")
        res = _drain(srv, [t1, t2])
    finally:
        srv.close()
    for t in (t1, t2):
        assert rel(res[t][1], ref_big.cpu().numpy()) <= 1e-8


def test_served_gangs_match_alone():
    """Requests large enough to run on gangs of several groups (2, 4, 8, ... of
    16 workgroups), mixed with one-group requests, all in flight together."""
    import paper_1804_05126_amd as K
    prs = [W.adr2d_problem(s, p, tau, seed=5100 + i) for i, (s, p, tau) in
           enumerate([(96, 2, 1e-3), (300, 3, 2e-4), (40, 1, 1e-2), (512, 2, 1e-4), (128, 4, 5e-4)])]
    prs += [W.diffusion3d_problem(s, 2, 2e-4, seed=5200 + s, tol=1e-8) for s in (24, 48, 64)]
    ins = _inputs(prs)
    alone = []
    for pr, (op, vecs) in zip(prs, ins):
        w, st, status = K.phi_combination(op, pr.tau, vecs, tol=pr.tol)
        assert status == 0
        alone.append(w.cpu().numpy())
    srv = K.Server(pool_bytes=8 << 30, group_size=16, points_per_workgroup=1024)
    announce(f"served gangs: {srv.groups} groups of 16")
    try:
        tickets = [srv.submit(op, pr.tau, vecs, tol=pr.tol) for pr, (op, vecs) in zip(prs, ins)]
        res = _drain(srv, tickets)
    finally:
        srv.close()
    sizes = []
    for pr, a, t in zip(prs, alone, tickets):
        st, w = res[t]
        assert st["status"] == 0
        sizes.append(st["grid_blocks"])
        assert rel(w, a) <= 2e-8, (pr.name, rel(w, a))
    announce(f"  gang sizes (workgroups): {sizes}")
    assert max(sizes) >= 64 and min(sizes) == 16


def test_served_bitwise_alone_and_in_mix():
    """On a gang of a given size a request computes the same bits whether it
    runs alone on the server or among other requests (the reductions follow
    the gang's workgroup order, not the timing)."""
    import torch
    import paper_1804_05126_amd as K
    prs = _requests(12, seed=5301)
    ins = _inputs(prs)
    probe = [0, 3, 7]
    alone = {}
    srv = K.Server(pool_bytes=4 << 30, group_size=16)
    try:
        for i in probe:
            pr, (op, vecs) = prs[i], ins[i]
            t = srv.submit(op, pr.tau, vecs, tol=pr.tol)
            res = _drain(srv, [t])
            alone[i] = (res[t][0]["grid_blocks"], res[t][1])
        announce(f"served bitwise: alone done, gangs {[alone[i][0] for i in probe]}")
        tickets = [srv.submit(op, pr.tau, vecs, tol=pr.tol) for pr, (op, vecs) in zip(prs, ins)]
        res = _drain(srv, tickets)
    finally:
        srv.close()
    for i in probe:
        st, w = res[tickets[i]]
        assert st["grid_blocks"] == alone[i][0]
        assert np.array_equal(w, alone[i][1]), (prs[i].name, rel(w, alone[i][1]))


def test_served_first_use_of_every_queue_slot():
    """Regression test of the request hand-over: many small requests submitted
    together land on fresh groups, so each is read from a queue slot and a
    parameter block the launch has never read before (the case in which a
    launch that saw a tail before its block pointer or block contents read a
    null or uninitialised pointer).  Two servers in a row, the second on the
    mailbox the first gave back.  Every result must equal the dense Theorem-1
    result."""
    import paper_1804_05126_amd as K
    prs = [W.adr2d_problem(16 + 4 * (i % 5), 1 + i % 2, 1e-3 * (1 + i % 3), seed=5400 + i)
           for i in range(40)]
    ins = _inputs(prs)
    refs = [augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors) for pr in prs]
    for rep in range(2):
        srv = K.Server(pool_bytes=1 << 30, group_size=8)
        announce(f"served first use (server {rep}): {len(prs)} requests on {srv.groups} groups of 8")
        try:
            tickets = [srv.submit(op, pr.tau, vecs, tol=pr.tol) for pr, (op, vecs) in zip(prs, ins)]
            res = _drain(srv, tickets)
        finally:
            srv.close()
        for pr, ref, t in zip(prs, refs, tickets):
            st, w = res[t]
            assert st["status"] == 0, (rep, pr.name)
            assert rel(w, ref) <= 1e-8, (rep, pr.name, rel(w, ref))
