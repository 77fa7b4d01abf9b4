"""Pins of the oracle's general (per-cell weights) stencil form.

  * the whole-array form and the entry-by-entry sparse assembly agree for
    random weights (2-D and 3-D, with axes of size 1 and 2, where a
    neighbour is the cell itself or both neighbours coincide);
  * weights written from the coefficient form (diffusivity field, advection,
    reaction) give the coefficient-form operator.
"""

import numpy as np
import pytest

import workloads as W
from oracle import operators


@pytest.mark.parametrize("shape", [(7, 5, 1), (5, 4, 3), (6, 1, 1), (2, 3, 1), (4, 2, 2)])
def test_weights_apply_matches_sparse_assembly(shape):
    nx, ny, nz = shape
    n = nx * ny * nz
    g = np.random.default_rng(nx * 100 + ny * 10 + nz)
    nw = 5 if nz == 1 else 7
    desc = W.StencilDesc(nx=nx, ny=ny, nz=nz, h=0.1, weights=g.standard_normal((nw, n)))
    M = operators.stencil_sparse(desc)
    for _ in range(3):
        u = g.standard_normal(n)
        assert np.allclose(operators.stencil_apply(desc, u), M @ u, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape", [(8, 6, 1), (5, 4, 3)])
def test_weights_from_coefficients_reproduce_the_operator(shape):
    nx, ny, nz = shape
    n = nx * ny * nz
    g = np.random.default_rng(5)
    h = 0.125
    kap = g.uniform(0.5, 2.0, n)
    adv = (1.5, -2.0, 0.7)
    r = g.uniform(-3, 0, n)
    coef = W.StencilDesc(nx=nx, ny=ny, nz=nz, h=h, kappa=kap, adv=adv, reaction=r)
    K = kap.reshape(nz, ny, nx)
    nw = 5 if nz == 1 else 7
    Wt = np.zeros((nw, n))
    Wt[0] = r
    for d, (axis, size) in enumerate(((2, nx), (1, ny), (0, nz))[: (nw - 1) // 2]):
        if size == 1:
            continue
        kp = (0.5 * (K + np.roll(K, -1, axis=axis))).reshape(-1)
        km = (0.5 * (K + np.roll(K, 1, axis=axis))).reshape(-1)
        Wt[0] -= (kp + km) / h ** 2
        Wt[1 + 2 * d] = kp / h ** 2 - adv[d] / (2 * h)
        Wt[2 + 2 * d] = km / h ** 2 + adv[d] / (2 * h)
    gen = W.StencilDesc(nx=nx, ny=ny, nz=nz, h=h, weights=Wt)
    u = g.standard_normal(n)
    a = operators.stencil_apply(coef, u)
    b = operators.stencil_apply(gen, u)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())
