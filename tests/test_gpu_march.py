"""GPU parity of the row-marching 5-point pass (large 2-D grids) against the oracle.

The library picks the marching pass for large constant-diffusivity 2-D grids
with IOP windows of one or two vectors (the 2048^2 workloads run on it); the
environment variable KIOPS_MARCH=2 selects it for any size, so that ragged
strips (width not a multiple of 256), short and odd row chunks (both march
directions) and tiny grids are compared here with the oracle's Algorithm 2
basis and with exact results.  KIOPS_MARCH=0 selects the tile pass.
"""

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators
from oracle.arnoldi import phi_combination_arnoldi
from oracle.iop import iop_basis as oracle_iop

from gpu_helpers import announce, rel, to_dev

pytestmark = pytest.mark.gpu


def _desc(nx, ny, g):
    n = nx * ny
    return W.StencilDesc(nx=nx, ny=ny, nz=1, h=1.0 / max(nx, ny), diff=1e-2, adv=(10.0, -7.0, 0.0),
                         reaction=g.uniform(-1, 0, n))


CASES = [
    # (nx, ny, p, q, m, seed): strips of 256 and ragged ones, one or several row chunks
    (300, 100, 3, 2, 25, 21),   # two strips (256 + 44), three chunks (down, up, down)
    (256, 37, 2, 1, 20, 22),    # one strip, one chunk, window of one
    (520, 70, 0, 2, 20, 23),    # three strips (the last of 8 columns), p = 0
    (257, 65, 4, 2, 24, 24),    # a strip of one column
    (270, 3, 2, 2, 12, 25),     # three rows (halo rows wrap onto the chunk)
    (300, 1, 1, 2, 10, 26),     # one row
]


@pytest.mark.parametrize("nx,ny,p,q,m,seed", CASES)
def test_march_iop_basis_matches_oracle(nx, ny, p, q, m, seed, monkeypatch):
    import paper_1804_05126_amd as K
    monkeypatch.setenv("KIOPS_MARCH", "2")
    g = np.random.Generator(np.random.PCG64(seed))
    desc = _desc(nx, ny, g)
    n = desc.n
    vecs = [g.standard_normal(n) for _ in range(p + 1)]
    announce(f"march iop {nx}x{ny} p={p} q={q} m={m}")
    op = K.Operator.from_desc(desc)
    basis, H, j, beta, nu = K.iop_basis(op, to_dev(vecs), m, q)
    nu_o, mu_o = augmented.b_norm_scaling(vecs)
    Vo, Ho, jo, bdo, beta_o = oracle_iop(operators.make_apply(desc), [vecs[p - c] for c in range(p)], nu_o,
                                         vecs[0], mu_o * augmented.trailing_entries(p, 0.0), m, q)
    assert nu == nu_o
    assert j == jo and not bdo
    assert beta == pytest.approx(beta_o, rel=1e-13)
    Hd = H.cpu().numpy()
    assert np.max(np.abs(Hd - Ho)) <= 1e-9 * np.max(np.abs(Ho))
    Vd = basis.cpu().numpy()
    assert np.max(np.abs(Vd - Vo)) <= 1e-8, np.max(np.abs(Vd - Vo))
    assert np.max(np.abs(Vd[:4] - Vo[:4])) <= 1e-12


@pytest.mark.parametrize("nx,ny,p,tau,precision", [(300, 100, 3, 5e-3, "fp64"), (520, 70, 2, 2e-2, "fp64"),
                                                   (256, 96, 1, 1e-2, "mixed"), (300, 100, 4, 5e-3, "mixed")])
def test_march_solve_vs_arnoldi(nx, ny, p, tau, precision, monkeypatch):
    import paper_1804_05126_amd as K
    g = np.random.Generator(np.random.PCG64(nx + 7 * ny + p))
    desc = _desc(nx, ny, g)
    vecs = [g.standard_normal(desc.n) for _ in range(p + 1)]
    tol, bound = (1e-8, 1e-8) if precision == "fp64" else (1e-6, 1e-5)
    announce(f"march solve {nx}x{ny} p={p} tau={tau} {precision}")
    ref = phi_combination_arnoldi(operators.make_apply(desc), tau, vecs, tol_o=1e-12)
    res = {}
    for mode in ("2", "0"):      # marching pass, then the tile pass
        monkeypatch.setenv("KIOPS_MARCH", mode)
        op = K.Operator.from_desc(desc, precision=precision)
        w, st, _ = K.phi_combination(op, tau, to_dev(vecs), tol=tol)
        res[mode] = (w.cpu().numpy(), st)
        announce(f"  KIOPS_MARCH={mode}: rel err {rel(res[mode][0], ref):.3e}, matvecs {st['matvecs']}, "
                 f"grid {st['grid_blocks']}")
    assert rel(res["2"][0], ref) <= bound
    assert rel(res["0"][0], ref) <= bound


def test_march_in_place_and_deterministic(monkeypatch):
    import torch
    import paper_1804_05126_amd as K
    monkeypatch.setenv("KIOPS_MARCH", "2")
    g = np.random.Generator(np.random.PCG64(31))
    desc = _desc(300, 100, g)
    vecs = to_dev([g.standard_normal(desc.n) for _ in range(3)])
    op = K.Operator.from_desc(desc)
    a, _, _ = K.phi_combination(op, 1e-2, vecs, tol=1e-8)
    b, _, _ = K.phi_combination(op, 1e-2, vecs, tol=1e-8)
    assert torch.equal(a, b)
    b0 = vecs[0].clone()
    K.phi_combination(op, 1e-2, [b0] + vecs[1:], tol=1e-8, out=b0)
    assert torch.equal(b0, a)
