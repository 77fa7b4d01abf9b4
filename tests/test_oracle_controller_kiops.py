"""Pins of the oracle's Algorithm 4 (hand-derived decision table) and of its
Algorithm 1 (the method run on the CPU) against the exact results."""

import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import augmented, operators, spectral
from oracle.controller import ControllerState, decide
from oracle.kiops import kiops

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "controller_cases.json")


def load_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def _state(case):
    s = dict(T_end=1.0, tol=1e-8, m_min=10, m_max=128, T_now=0.0)
    s.update(case["state"])
    return ControllerState(**s)


@pytest.mark.parametrize("case", load_cases(), ids=lambda c: c["name"])
def test_controller_golden(case):
    d = decide(_state(case), case["j"], case["eps"], case["breakdown"])
    e = case["expect"]
    assert d.accept == e["accept"]
    assert d.m_new == e["m_new"]
    assert d.branch == e["branch"]
    assert d.tau_new == pytest.approx(e["tau_new"], rel=1e-12)


def test_controller_nonfinite_raises():
    st = ControllerState(T_end=1.0, tol=1e-8, tau=1.0, m=10)
    with pytest.raises(FloatingPointError):
        decide(st, 10, float("nan"), False)


# ------------------------------------------------------------- Algorithm 1

def test_kiops_cfg1_vs_dense():
    pr = W.cfg1()
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    w, st = kiops(operators.make_apply(pr.op), pr.tau, pr.vectors, tol=pr.tol)
    assert np.linalg.norm(w - ref) <= 1e-8 * np.linalg.norm(ref)
    assert st.substeps >= 1 and st.matvecs >= 10


@pytest.mark.parametrize("tau", [1e-3, 1e-2])
def test_kiops_stiff_2d_vs_dft(tau):
    pr = W.adr2d_problem(64, 3, tau, seed=21, constant_reaction=-0.5)
    ref = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    w, st = kiops(operators.make_apply(pr.op), pr.tau, pr.vectors, tol=1e-8)
    assert np.linalg.norm(w - ref) <= 1e-8 * np.linalg.norm(ref)


def test_kiops_reaches_mmax_and_substeps():
    pr = W.adr2d_problem(64, 2, 5e-2, seed=22, constant_reaction=-0.2)
    ref = spectral.phi_combination_fft(pr.op, pr.tau, pr.vectors)
    w, st = kiops(operators.make_apply(pr.op), pr.tau, pr.vectors, tol=1e-8, m_max=40)
    assert st.substeps > 1
    assert any(t[1] == 40 for t in st.trace)
    assert np.linalg.norm(w - ref) <= 1e-8 * np.linalg.norm(ref)


def test_kiops_zero_operator_is_polynomial():
    g = np.random.Generator(np.random.PCG64(4))
    vecs = [g.standard_normal(30) for _ in range(2)]
    w, st = kiops(lambda x: 0.0 * x, 0.5, vecs, tol=1e-10)
    ref = vecs[0] + 0.5 * vecs[1]
    assert np.allclose(w, ref, rtol=1e-12, atol=1e-12)
    assert st.breakdowns >= 1


def test_kiops_tau_zero_returns_b0():
    pr = W.cfg1()
    w, st = kiops(operators.make_apply(pr.op), 0.0, pr.vectors)
    assert np.array_equal(w, pr.vectors[0]) and st.matvecs == 0


def test_kiops_linearity_and_shift_identity():
    """Two half steps with the shifted vectors b_k <- sum_l t1^l/l! b_{k+l}
    (the form of Eq. (7)) reproduce one full step, within tolerance."""
    pr = W.adr2d_problem(24, 3, 2e-2, seed=23)
    ap = operators.make_apply(pr.op)
    tol = 1e-10
    full, _ = kiops(ap, pr.tau, pr.vectors, tol=tol)
    t1 = 0.4 * pr.tau
    w1, _ = kiops(ap, t1, pr.vectors, tol=tol)
    p = pr.p
    shifted = [w1] + [sum(t1 ** l / math.factorial(l) * pr.vectors[k + l] for l in range(p - k + 1))
                      for k in range(1, p + 1)]
    w2, _ = kiops(ap, pr.tau - t1, shifted, tol=tol)
    assert np.linalg.norm(w2 - full) <= 1e-8 * np.linalg.norm(full)
    two, _ = kiops(ap, pr.tau, [2.0 * v for v in pr.vectors], tol=tol)
    assert np.linalg.norm(two - 2.0 * full) <= 1e-8 * np.linalg.norm(full)


def test_kiops_normalisation_does_not_change_result():
    pr = W.adr2d_problem(20, 4, 1e-2, seed=24)
    ap = operators.make_apply(pr.op)
    ref = augmented.phi_combination_dense(operators.dense(pr.op), pr.tau, pr.vectors)
    a, _ = kiops(ap, pr.tau, pr.vectors, tol=1e-9, normalize_B=True)
    b, _ = kiops(ap, pr.tau, pr.vectors, tol=1e-9, normalize_B=False)
    assert np.linalg.norm(a - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.linalg.norm(b - ref) <= 1e-8 * np.linalg.norm(ref)
