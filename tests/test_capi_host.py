"""CPU checks of the C ABI: the library loads, exports every function that
include/kiops.h declares, and its controller (the same code the device runs
once per attempt) reproduces the hand-derived decision table."""

import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kiops.h")


def _lib():
    from paper_1804_05126_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libkiops.so not built (run __graft_entry__.build())")
    return L, L.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:kiops_status|const char\*)\s+(kiops_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("kiops_create_operator", "kiops_destroy_operator", "kiops_workspace_bytes",
                     "kiops_set_workspace", "kiops_phi_combination", "kiops_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    bound = {n for n, _, _ in L.SIGNATURES}
    assert set(declared_functions()) <= bound


def test_status_strings():
    _, lib = _lib()
    assert lib.kiops_status_string(0) == b"ok"
    assert lib.kiops_status_string(5) == b"substep limit reached"
    assert lib.kiops_status_string(99) == b"unknown status"


def test_null_arguments_rejected_without_device():
    L, lib = _lib()
    out = ctypes.c_void_p()
    assert lib.kiops_create_operator(None, None, ctypes.byref(out)) == 1
    d = L.OperatorDesc()
    d.kind = L.OP_STENCIL2D_5PT
    d.nx, d.ny, d.nz, d.h = 8, 8, 2, 0.1          # 2-D operator with nz != 1
    assert lib.kiops_create_operator(ctypes.byref(d), None, ctypes.byref(out)) == 1
    d.nz, d.h = 1, -1.0                           # negative spacing
    assert lib.kiops_create_operator(ctypes.byref(d), None, ctypes.byref(out)) == 1
    assert lib.kiops_phi_combination(None, 1.0, 0, None, 1e-8, 10, 2, None, None, None) == 1
    assert lib.kiops_destroy_operator(None) == 1
    # batch shape tuner: empty candidate lists, missing outputs or an unaligned
    # workspace are refused before any device call
    gs, rows = (ctypes.c_int * 2)(8, 16), (ctypes.c_int * 1)(16)
    bg, br, bms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    args = (0, None, None)
    assert lib.kiops_batch_tune_shape(*args, None, 0, rows, 1, ctypes.c_void_p(256), 1 << 20, None,
                                      ctypes.byref(bg), ctypes.byref(br), ctypes.byref(bms)) == 1
    assert lib.kiops_batch_tune_shape(*args, gs, 2, rows, 0, ctypes.c_void_p(256), 1 << 20, None,
                                      ctypes.byref(bg), ctypes.byref(br), ctypes.byref(bms)) == 1
    assert lib.kiops_batch_tune_shape(*args, gs, 2, rows, 1, ctypes.c_void_p(256), 1 << 20, None,
                                      None, ctypes.byref(br), ctypes.byref(bms)) == 1
    assert lib.kiops_batch_tune_shape(*args, gs, 2, rows, 1, ctypes.c_void_p(100), 1 << 20, None,
                                      ctypes.byref(bg), ctypes.byref(br), ctypes.byref(bms)) == 1
    assert lib.kiops_batch_tune_shape(*args, gs, 2, rows, 1, ctypes.c_void_p(256), 1 << 20, None,
                                      ctypes.byref(bg), ctypes.byref(br), ctypes.byref(bms)) == 1   # no problems


def test_grid_size_product_overflow_rejected():
    # each side within 2^30, but nx*ny*nz = 2^66 wraps a 64-bit product
    L, lib = _lib()
    out = ctypes.c_void_p()
    d = L.OperatorDesc()
    d.kind = L.OP_STENCIL3D_7PT
    d.nx = d.ny = d.nz = 1 << 22
    d.h = 1.0
    assert lib.kiops_create_operator(ctypes.byref(d), None, ctypes.byref(out)) == 1
    d.nx = d.ny = d.nz = 1 << 11                  # 2^33 points: 8 N reaches 4 GiB
    assert lib.kiops_create_operator(ctypes.byref(d), None, ctypes.byref(out)) == 1
    assert not out.value


def test_stream_probe_rejects_bad_arguments_without_device():
    _, lib = _lib()
    arr = (ctypes.c_void_p * 1)(16)
    assert lib.kiops_stream_probe(None, 1, ctypes.c_void_p(16), 64, 8, None) == 1
    assert lib.kiops_stream_probe(arr, 0, ctypes.c_void_p(16), 64, 8, None) == 1
    assert lib.kiops_stream_probe(arr, 1, None, 64, 8, None) == 1
    assert lib.kiops_stream_probe(arr, 1, ctypes.c_void_p(16), 63, 8, None) == 1      # odd n
    assert lib.kiops_stream_probe(arr, 1, ctypes.c_void_p(24), 64, 8, None) == 1      # misaligned dst


GOLDEN = os.path.join(ROOT, "tests", "golden", "controller_cases.json")


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_device_controller_golden(case):
    _lib()
    import paper_1804_05126_amd as K
    st = dict(T_end=1.0, tol=1e-8, m_min=10, m_max=128, T_now=0.0, have_old=0)
    for k, v in case["state"].items():
        st[k] = int(v) if k == "have_old" else v
    d = K.controller_decide(st, case["j"], case["eps"], case["breakdown"])
    e = case["expect"]
    assert d["accept"] == e["accept"]
    assert d["m_new"] == e["m_new"]
    assert d["branch"] == e["branch"]
    assert d["tau_new"] == pytest.approx(e["tau_new"], rel=1e-12)


def test_device_controller_matches_oracle_on_random_inputs():
    """The device controller and the oracle's Algorithm 4 are written apart;
    on random states away from rounding ties they must decide alike."""
    _lib()
    import math
    import numpy as np
    import paper_1804_05126_amd as K
    from oracle.controller import ControllerState, decide
    g = np.random.Generator(np.random.PCG64(77))
    for _ in range(2000):
        m_max = int(g.choice([40, 128]))
        j = int(g.integers(10, m_max + 1))
        tau = float(10 ** g.uniform(-4, 0))
        have_old = bool(g.uniform() < 0.5)
        st = dict(T_end=1.0, tol=1e-8, T_now=float(g.uniform(0, 1 - tau)) if tau < 1 else 0.0,
                  tau=tau, m_min=10, m_max=m_max, m=j, have_old=int(have_old),
                  tau_old=tau * float(g.choice([1.0, 2.0, 3.0])), eps_old=float(10 ** g.uniform(-14, 0)),
                  omega_old=float(10 ** g.uniform(-3, 6)), m_old=int(g.integers(10, m_max + 1)))
        eps = float(10 ** g.uniform(-16, 0))
        d = K.controller_decide(st, j, eps, False)
        cs = ControllerState(T_end=1.0, tol=1e-8, m_min=10, m_max=m_max, T_now=st["T_now"], tau=tau,
                             m=j, have_old=have_old, tau_old=st["tau_old"], eps_old=st["eps_old"],
                             omega_old=st["omega_old"], m_old=st["m_old"])
        o = decide(cs, j, eps, False)
        assert d["accept"] == o.accept and d["branch"] == o.branch
        assert math.isclose(d["tau_new"], o.tau_new, rel_tol=1e-12)
        if d["m_new"] != o.m_new:
            # only a ceil() on an exact integer boundary may differ by rounding
            assert abs(d["m_new"] - o.m_new) == 1
