"""Pins of the oracle's several-output-times route (Algorithm 1 with an array
of times, Task I and Task II).

Task II at each T_k is sum_i T_k^i phi_i(T_k A) b_i; Task I multiplies it by
(1 / T_k)^p, which leaves phi_p(T_k A) b_p when only b_p is nonzero.  Both are
checked against scalar closed forms of phi_1, phi_2 on a diagonal A (written
out here from phi_0(z) = e^z, phi_{k+1}(z) = (phi_k(z) - 1/k!) / z), and
against the semigroup property of the exponential.
"""

import math

import numpy as np
import pytest

from oracle import augmented


def _phi(k, z):
    v = math.exp(z)
    for j in range(k):
        v = (v - 1.0 / math.factorial(j)) / z
    return v


def _setup(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    a = -g.uniform(0.5, 3.0, n)            # moderate |z| keeps the recurrence accurate
    return a, np.diag(a), [g.standard_normal(n) for _ in range(3)]


def test_task2_times_match_scalar_closed_forms():
    a, A, b = _setup(7, 11)
    times = [0.05, 0.2, 0.7, 1.3]
    got = augmented.phi_combination_times(A, times, b, task=2)
    for t, w in zip(times, got):
        ref = np.array([_phi(0, t * ai) * b[0][i] + t * _phi(1, t * ai) * b[1][i] + t * t * _phi(2, t * ai) * b[2][i]
                        for i, ai in enumerate(a)])
        assert np.max(np.abs(w - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_task1_single_phi_p():
    a, A, b = _setup(6, 12)
    vecs = [np.zeros(6), np.zeros(6), b[2]]        # only b_2: Task I gives phi_2(T A) b_2
    times = [0.1, 0.5, 2.0]
    got = augmented.phi_combination_times(A, times, vecs, task=1)
    for t, w in zip(times, got):
        ref = np.array([_phi(2, t * ai) * b[2][i] for i, ai in enumerate(a)])
        assert np.max(np.abs(w - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_times_semigroup_p0():
    g = np.random.Generator(np.random.PCG64(13))
    A = g.standard_normal((9, 9)) - 3.0 * np.eye(9)
    b0 = g.standard_normal(9)
    t1, t2 = 0.3, 0.8
    w1, w2 = augmented.phi_combination_times(A, [t1, t2], [b0], task=2)
    w21 = augmented.phi_combination_times(A, [t2 - t1], [w1], task=2)[0]
    assert np.max(np.abs(w2 - w21)) <= 1e-12 * np.max(np.abs(w2))


@pytest.mark.parametrize("task", [1, 2])
def test_task_scaling_relation(task):
    a, A, b = _setup(5, 14)
    times = [0.25, 1.0]
    t2 = augmented.phi_combination_times(A, times, b, task=2)
    got = augmented.phi_combination_times(A, times, b, task=task)
    for t, x, y in zip(times, got, t2):
        expect = y * (1.0 / t) ** 2 if task == 1 else y
        assert np.array_equal(x, expect)
