"""GPU parity of the batched form (many problems in one persistent launch).

Each problem of a batch must match the oracle exactly as a single solve does
(dense Theorem-1 result, relative 2-norm error <= 1e-8 at tol 1e-8, <= 1e-5
for the mixed form at tol 1e-6), whatever the group size, and agree with the
same problem solved alone.  Batches of 2-D (different sizes, p, tau and
coefficients, as in the batched workload's recipe) and of 3-D problems are
checked; operators of different families in one batch are refused.
"""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _small_batch(count, seed, precision="fp64", side_range=(16, 64)):
    return W.cfg4(count=count, seed=seed, precision=precision, side_range=side_range)


def _problems(prs, precision="fp64"):
    import paper_1804_05126_amd as K
    out = []
    for pr in prs:
        op = K.Operator.from_desc(pr.op, precision=precision)
        out.append(dict(op=op, tau=pr.tau, vectors=to_dev(pr.vectors), tol=pr.tol, m_init=pr.m_init, q=pr.q))
    return out


@pytest.mark.parametrize("group_size", [0, 8, 16])
def test_batch_2d_vs_dense(group_size):
    import paper_1804_05126_amd as K
    prs = _small_batch(12, seed=4001)
    announce(f"batch of 12 2-D problems, group_size={group_size}")
    ws, stats, status, plan = K.phi_batch(_problems(prs), group_size=group_size)
    announce(f"  plan (groups, group size) = {plan}")
    assert status == 0
    for pr, w, st in zip(prs, ws, stats):
        assert st["status"] == 0
        ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
        assert rel(w.cpu().numpy(), ref) <= 1e-8, (pr.name, st)


def test_batch_matches_single_solves():
    import paper_1804_05126_amd as K
    prs = _small_batch(8, seed=4002, side_range=(40, 120))
    probs = _problems(prs)
    announce("batch of 8 vs the same problems solved alone")
    ws, stats, status, plan = K.phi_batch(probs, group_size=8)
    assert status == 0
    for pr, pb, w in zip(prs, probs, ws):
        single, st, _ = K.phi_combination(pb["op"], pr.tau, pb["vectors"], tol=pr.tol)
        assert rel(w.cpu().numpy(), single.cpu().numpy()) <= 1e-8


def test_batch_mixed_vs_dense():
    import paper_1804_05126_amd as K
    prs = _small_batch(8, seed=4003, precision="mixed")
    announce("mixed batch of 8")
    ws, stats, status, plan = K.phi_batch(_problems(prs, precision="mixed"), group_size=8)
    assert status == 0
    for pr, w in zip(prs, ws):
        ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
        assert rel(w.cpu().numpy(), ref) <= 1e-5


def test_batch_3d_vs_dense():
    import paper_1804_05126_amd as K
    prs = [W.diffusion3d_problem(s, p, t, seed=4100 + s, tol=1e-8)
           for s, p, t in ((8, 1, 2e-3), (12, 2, 1e-3), (16, 3, 5e-4), (10, 4, 1e-3))]
    announce("batch of 4 3-D problems")
    ws, stats, status, plan = K.phi_batch(_problems(prs), group_size=8)
    assert status == 0
    for pr, w in zip(prs, ws):
        ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
        assert rel(w.cpu().numpy(), ref) <= 1e-8


def test_batch_refuses_mixed_families():
    import paper_1804_05126_amd as K
    prs = [_small_batch(1, seed=4004)[0], W.diffusion3d_problem(8, 1, 1e-3, seed=4005)]
    announce("batch with a 2-D and a 3-D operator")
    with pytest.raises(K.KiopsError):
        K.phi_batch(_problems(prs))


def test_batch_tune_picks_a_candidate():
    import paper_1804_05126_amd as K
    prs = _small_batch(16, seed=4006, side_range=(32, 96))
    announce("autotune over group sizes 8, 16")
    best, ms = K.batch_tune(_problems(prs), candidates=(8, 16))
    assert best in (8, 16) and ms > 0


def test_full_batch_workload_matches_single_solves_and_oracle():
    """The batched workload at its full size, in the configuration bench.py
    times (256 problems, group size autotuned there, 16 here): every result
    agrees with the same problem solved alone, and the three smallest agree
    with the oracle's full-Arnoldi route."""
    import paper_1804_05126_amd as K
    from oracle.arnoldi import phi_combination_arnoldi
    prs = W.cfg4()
    probs = _problems(prs)
    announce(f"full batch: {len(prs)} problems, {sum(pr.n for pr in prs)} points")
    ws, stats, status, plan = K.phi_batch(probs, group_size=16)
    assert status == 0
    assert all(st["status"] == 0 for st in stats)
    for pr, pb, w in zip(prs, probs, ws):
        single, st, s1 = K.phi_combination(pb["op"], pr.tau, pb["vectors"], tol=pr.tol)
        assert s1 == 0
        assert rel(w.cpu().numpy(), single.cpu().numpy()) <= 2e-8, pr.name
    for i in sorted(range(len(prs)), key=lambda i: prs[i].n)[:3]:
        pr = prs[i]
        ref = phi_combination_arnoldi(operators.make_apply(pr.op), pr.tau, pr.vectors, tol_o=1e-12)
        assert rel(ws[i].cpu().numpy(), ref) <= 1e-8, (pr.name, rel(ws[i].cpu().numpy(), ref))


def test_batch_dominant_problem_gets_own_group():
    """Two problems, one with nearly all of the work: the plan gives it a
    group of its own (larger than the shared groups) and both results still
    match the same problems solved alone (the small one also the dense route)."""
    import paper_1804_05126_amd as K
    big = W.adr2d_problem(256, 3, 2e-2, seed=4201)
    small = W.adr2d_problem(16, 2, 1e-2, seed=4202)
    probs = _problems([big, small])
    announce("batch of a dominant and a small problem")
    ws, stats, status, plan = K.phi_batch(probs, group_size=8)
    assert status == 0
    assert stats[0]["grid_blocks"] > 8 and stats[1]["grid_blocks"] == 8, (stats[0]["grid_blocks"], stats[1]["grid_blocks"])
    for pr, pb, w in zip((big, small), probs, ws):
        single, st, s1 = K.phi_combination(pb["op"], pr.tau, pb["vectors"], tol=pr.tol)
        assert s1 == 0
        assert rel(w.cpu().numpy(), single.cpu().numpy()) <= 2e-8
    ref = augmented.phi_combination_dense(operators.dense(small.op), small.tau, small.vectors)
    assert rel(ws[1].cpu().numpy(), ref) <= 1e-8


def test_batch_reports_start_and_end_clocks():
    # each problem's device clocks: start before end, all inside the host's
    # wall time of the call; a single solve reports them too
    import time
    import torch
    import paper_1804_05126_amd as K
    prs = _small_batch(16, seed=4011)
    probs = _problems(prs)
    announce("batch of 16: per-problem start and end clocks")
    K.phi_batch(probs, group_size=8)             # warm: workspaces and code
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ws, stats, status, plan = K.phi_batch(probs, group_size=8)
    wall = time.perf_counter() - t0
    assert status == 0
    starts = [st["clock_start_s"] for st in stats]
    ends = [st["clock_end_s"] for st in stats]
    assert all(e > s > 0.0 for s, e in zip(starts, ends))
    span = max(ends) - min(starts)
    announce(f"  device span {span * 1e3:.3f} ms, host wall {wall * 1e3:.3f} ms")
    assert 0.0 < span <= wall
    _, st, _ = K.phi_combination(probs[0]["op"], prs[0].tau, probs[0]["vectors"], tol=prs[0].tol)
    assert st["clock_end_s"] > st["clock_start_s"] > 0.0


@pytest.mark.parametrize("tile_rows", [8, 4])
def test_batch_short_tiles_vs_dense(tile_rows):
    # the tile heights the shape autotuner may pick: every problem still matches
    # the dense Theorem-1 result, including sides that are not multiples of the
    # tile (the problems of cfg4's recipe at 16..64 points a side)
    import paper_1804_05126_amd as K
    prs = _small_batch(12, seed=4001)
    announce(f"batch of 12 2-D problems, 64 x {tile_rows} tiles")
    for gs in (8, 16):
        ws, stats, status, plan = K.phi_batch(_problems(prs), group_size=gs, tile_rows=tile_rows)
        assert status == 0
        for pr, w, st in zip(prs, ws, stats):
            assert st["status"] == 0
            ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
            assert rel(w.cpu().numpy(), ref) <= 1e-8, (pr.name, gs, st)


def test_batch_short_tiles_match_single_solves_mixed():
    import paper_1804_05126_amd as K
    prs = _small_batch(8, seed=4002, side_range=(40, 120))
    probs = _problems(prs)
    announce("batch of 8, 64 x 4 tiles, vs the same problems solved alone")
    ws, stats, status, plan = K.phi_batch(probs, group_size=8, tile_rows=4)
    assert status == 0
    for pr, pb, w in zip(prs, probs, ws):
        single, st, _ = K.phi_combination(pb["op"], pr.tau, pb["vectors"], tol=pr.tol)
        assert rel(w.cpu().numpy(), single.cpu().numpy()) <= 1e-8
    mprs = _small_batch(8, seed=4003, precision="mixed")
    announce("mixed batch of 8, 64 x 8 tiles")
    ws, stats, status, plan = K.phi_batch(_problems(mprs, precision="mixed"), group_size=8, tile_rows=8)
    assert status == 0
    for pr, w in zip(mprs, ws):
        ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
        assert rel(w.cpu().numpy(), ref) <= 1e-5


def test_batch_tune_shape_picks_a_candidate_pair():
    import paper_1804_05126_amd as K
    prs = _small_batch(10, seed=4004)
    announce("shape autotuner over group sizes (8, 16) and tile rows (16, 8, 4)")
    gs, rows, ms = K.batch_tune_shape(_problems(prs), group_sizes=(8, 16), tile_rows=(16, 8, 4))
    assert gs in (8, 16) and rows in (16, 8, 4) and ms > 0.0
    # 3-D batches have one tile shape: the pair reports the default rows
    prs3 = [W.diffusion3d_problem(s, 2, 1e-3, seed=4200 + s, tol=1e-8) for s in (8, 10)]
    gs, rows, ms = K.batch_tune_shape(_problems(prs3), group_sizes=(8,), tile_rows=(4, 8))
    assert gs == 8 and rows == 16


def test_batch_rejects_invalid_tile_rows():
    import paper_1804_05126_amd as K
    prs = _small_batch(2, seed=4005)
    for bad in (5, 32, -4):
        with pytest.raises(K.KiopsError) as e:
            K.phi_batch(_problems(prs), group_size=8, tile_rows=bad)
        assert "INVALID_ARG" in str(e.value)
