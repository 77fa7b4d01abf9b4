"""Loss of orthogonality of the basis at m = 128 (512^2 ADR problem, p = 3):
the device's full window (q = 0: classical Gram-Schmidt with a Gram-matrix
correction from one set of inner products per step) beside the oracle's
Arnoldi process with classical Gram-Schmidt applied twice (CGS2), on the same
augmented matrix and start vector (B scaled by nu, trailing entries by mu,
Eqs. (48)-(49)); the IOP window q = 2 is reported for comparison (its basis is
not orthogonal by design, Section 3.3)."""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators
from oracle.arnoldi import arnoldi_basis
from oracle.iop import IOPBasis

from gpu_helpers import announce, to_dev

pytestmark = pytest.mark.gpu


def test_orthogonality_at_m128():
    import torch
    import paper_1804_05126_amd as K
    m = 128
    pr = W.cfg2(512, 1e-2)
    p = len(pr.vectors) - 1
    op = K.Operator.from_desc(pr.op)
    vecs = to_dev(pr.vectors)
    loss = {}
    for q in (0, 2):
        V, H, j, beta, nu = K.iop_basis(op, vecs, m, q)
        assert j == m
        G = V @ V.T
        loss[q] = float((G - torch.eye(m + 1, dtype=G.dtype, device=G.device)).abs().max())
    nu_o, mu_o = augmented.b_norm_scaling(pr.vectors)
    Bcols = [pr.vectors[p - c] for c in range(p)]
    ob = IOPBasis(operators.make_apply(pr.op), Bcols, nu_o, pr.vectors[0],
                  mu_o * augmented.trailing_entries(p, 0.0), 0, m)
    Vo, Ho, k, happy = arnoldi_basis(ob.apply_aug, ob.V[0].copy(), m)
    assert k == m and not happy
    loss_cgs2 = float(np.abs(Vo @ Vo.T - np.eye(m + 1)).max())
    announce(f"max |I - V^T V| at m = {m}: device q=0 {loss[0]:.3e}, oracle CGS2 {loss_cgs2:.3e}, "
             f"device IOP q=2 {loss[2]:.3e}")
    assert loss[0] <= 1e-10
    assert loss_cgs2 <= 1e-12
