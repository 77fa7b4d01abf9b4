"""The entry point that allocates nothing (kiops_phi_combination_noalloc).

It runs the same solver with the library's fixed scratch array as the
workspace.  Two calls in a row (the second on a smaller problem, so the array
holds the first call's larger contents) are compared with the ordinary entry
point kiops_phi_combination on the same inputs (rel. 2-norm <= 1e-12: the same
kernels in the same order) and with the exact result of the dense oracle
(<= 1e-8 at tol 1e-8).  A problem whose workspace exceeds the array is
refused with KIOPS_ERR_OUT_OF_MEMORY, and the call allocates no device
memory through torch's allocator.
"""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _case(side, p, tau, seed):
    return W.adr2d_problem(side, p, tau, seed=seed)


def test_noalloc_matches_plain_entry_point_twice():
    import torch
    import paper_1804_05126_amd as K
    for side, p, tau, seed in ((48, 3, 2e-2, 71), (32, 2, 1e-2, 72)):   # second call: smaller input
        pr = _case(side, p, tau, seed)
        announce(f"noalloc {side}x{side} p={p} tau={tau}")
        op = K.Operator.from_desc(pr.op)
        vecs = to_dev(pr.vectors)
        ref_w, ref_st, _ = K.phi_combination(op, pr.tau, vecs, tol=1e-8)
        out = torch.empty(pr.n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        before, reserved = torch.cuda.memory_allocated(), torch.cuda.memory_reserved()
        w, st, status = K.phi_combination_noalloc(op, pr.tau, vecs, out, tol=1e-8)
        torch.cuda.synchronize()
        # nothing was allocated through torch during the call (a temporary of
        # an earlier statement may be released meanwhile)
        assert torch.cuda.memory_allocated() <= before and torch.cuda.memory_reserved() == reserved
        assert status == 0
        got, plain = w.cpu().numpy(), ref_w.cpu().numpy()
        e_plain = rel(got, plain)
        dense = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
        e_dense = rel(got, dense)
        announce(f"  vs plain entry point {e_plain:.2e} (bitwise {np.array_equal(got, plain)}), "
                 f"vs dense oracle {e_dense:.2e}; matvecs {st['matvecs']} / {ref_st['matvecs']}")
        assert e_plain <= 1e-12
        assert e_dense <= 1e-8
        assert st["matvecs"] == ref_st["matvecs"] and st["substeps"] == ref_st["substeps"]


def test_noalloc_refuses_problems_beyond_its_array():
    import torch
    import paper_1804_05126_amd as K
    pr = _case(512, 2, 1e-3, 73)            # 129 basis vectors of 2 MiB: beyond 128 MiB
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    out = torch.zeros(pr.n, dtype=torch.float64, device="cuda")
    announce(f"noalloc refusal: workspace {op.workspace_bytes(2) / 2**20:.0f} MiB")
    _, _, status = K.phi_combination_noalloc(op, pr.tau, vecs, out, tol=1e-8, check=False)
    assert status == 2                      # KIOPS_ERR_OUT_OF_MEMORY
    assert float(out.abs().max()) == 0.0    # nothing ran
