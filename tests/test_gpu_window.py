"""GPU parity across IOP windows (Algorithm 2 with window q = 1 … 4, and the
full window q = 0, i.e. full Arnoldi): the 512^2 ADR operator of the 2-D
workload with a constant reaction, whose exact phi-combination the oracle
computes by the periodic DFT.  Every window must meet the accuracy of the
default q = 2; the number of products it takes is reported."""

import pytest

import workloads as W
from oracle import spectral

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tau", [1e-2, 1e-1])
@pytest.mark.parametrize("q", [1, 2, 3, 4, 0])
def test_window_vs_dft(q, tau):
    import paper_1804_05126_amd as K
    pr = W.cfg2(512, tau, q=q, constant_reaction=-0.5)
    op = K.Operator.from_desc(pr.op)
    w, st, status = K.phi_combination(op, pr.tau, to_dev(pr.vectors), tol=pr.tol, m_init=pr.m_init, q=q)
    assert status == 0
    ref = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    err = rel(w.cpu().numpy(), ref)
    announce(f"512^2 tau {tau} q {q}: products {st['matvecs']} substeps {st['substeps']} "
             f"rejections {st['rejections']} error {err:.2e}")
    assert err <= 1e-8
