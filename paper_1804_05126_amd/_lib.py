"""ctypes view of the C ABI in include/kiops.h (marshalling only).

Loads ``libkiops.so`` from this package directory.  Nothing here computes;
every step of a solve runs in the HIP library.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkiops.so")

KIOPS_OK = 0
STATUS_NAMES = {
    0: "KIOPS_OK",
    1: "KIOPS_ERR_INVALID_ARG",
    2: "KIOPS_ERR_OUT_OF_MEMORY",
    3: "KIOPS_ERR_DEVICE",
    4: "KIOPS_ERR_NONFINITE",
    5: "KIOPS_ERR_NOT_CONVERGED",
    6: "KIOPS_ERR_BUDGET",
    7: "KIOPS_ERR_UNSUPPORTED",
}

OP_STENCIL2D_5PT = 0
OP_STENCIL3D_7PT = 1
OP_CSR = 2
FP64 = 0
MIXED = 1
M_MAX_LIMIT = 128
P_MAX = 8
EXPM_SCRATCH_DOUBLES = 9 * 144 * 144
PASS_NAMES = {0: "Stencil2D", 1: "Stencil2DWide", 2: "Stencil2DMarch", 3: "Stencil3D", 4: "CsrOp", 5: "WeightsOp"}


class OperatorDesc(C.Structure):
    _fields_ = [
        ("kind", C.c_int),
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("h", C.c_double),
        ("diff", C.c_double),
        ("kappa", C.c_void_p),
        ("adv", C.c_double * 3),
        ("reaction", C.c_void_p),
        ("nrows", C.c_int64), ("nnz", C.c_int64),
        ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
        ("precision", C.c_int),
        ("weights", C.c_void_p),
    ]


class Options(C.Structure):
    _fields_ = [("m_min", C.c_int32), ("m_max", C.c_int32), ("max_substeps", C.c_int32),
                ("estimate", C.c_int32), ("tile_rows", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [
        ("m_last", C.c_int32), ("substeps", C.c_int32), ("rejections", C.c_int32),
        ("expms", C.c_int32), ("breakdowns", C.c_int32), ("grid_blocks", C.c_int32),
        ("matvecs", C.c_int64),
        ("last_omega", C.c_double), ("t_reached", C.c_double), ("alg_bytes", C.c_double),
        ("beta_last", C.c_double),
        ("time_work_s", C.c_double), ("time_wait_s", C.c_double), ("time_epilogue_s", C.c_double),
        ("time_expm_s", C.c_double), ("arrive_max_s", C.c_double), ("arrive_mean_s", C.c_double),
        ("barriers", C.c_int64),
        ("release_max_s", C.c_double), ("release_mean_s", C.c_double),
        ("status", C.c_int32), ("m_max", C.c_int32),
        ("time_reduce_s", C.c_double), ("time_publish_s", C.c_double), ("time_serial_s", C.c_double),
        ("pass_kind", C.c_int32), ("reserved3", C.c_int32),
        ("clock_start_s", C.c_double), ("clock_end_s", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class CtrlIn(C.Structure):
    _fields_ = [
        ("T_end", C.c_double), ("tol", C.c_double), ("T_now", C.c_double), ("tau", C.c_double),
        ("m_min", C.c_int32), ("m_max", C.c_int32), ("m", C.c_int32), ("have_old", C.c_int32),
        ("tau_old", C.c_double), ("eps_old", C.c_double), ("omega_old", C.c_double),
        ("m_old", C.c_int32), ("reserved", C.c_int32),
    ]


class CtrlOut(C.Structure):
    _fields_ = [("accept", C.c_int32), ("m_new", C.c_int32), ("branch", C.c_int32),
                ("reserved", C.c_int32), ("tau_new", C.c_double), ("omega", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("op", C.c_void_p), ("tau", C.c_double), ("p", C.c_int32), ("q", C.c_int32),
                ("V", C.POINTER(C.c_void_p)), ("tol", C.c_double), ("m_init", C.c_int32),
                ("reserved", C.c_int32), ("w", C.c_void_p)]


BRANCH_NAMES = {0: "breakdown", 1: "tau_reject", 2: "tau_accept", 3: "m_reject", 4: "m_accept",
                -1: "nonfinite"}

# (name, restype, argtypes) of every exported entry point of include/kiops.h
SIGNATURES = [
    ("kiops_create_operator", C.c_int, [C.POINTER(OperatorDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("kiops_destroy_operator", C.c_int, [C.c_void_p]),
    ("kiops_workspace_bytes", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(Options),
                                        C.POINTER(C.c_size_t)]),
    ("kiops_set_workspace", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("kiops_phi_combination", C.c_int, [C.c_void_p, C.c_double, C.c_int, C.POINTER(C.c_void_p),
                                        C.c_double, C.c_int, C.c_int, C.POINTER(Options),
                                        C.c_void_p, C.POINTER(Stats)]),
    ("kiops_phi_combination_noalloc", C.c_int, [C.c_void_p, C.c_double, C.c_int, C.POINTER(C.c_void_p),
                                                C.c_double, C.c_int, C.c_int, C.POINTER(Options),
                                                C.c_void_p, C.POINTER(Stats)]),
    ("kiops_phi_combination_times", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_int, C.c_int,
                                              C.POINTER(C.c_void_p), C.c_double, C.c_int, C.c_int,
                                              C.POINTER(Options), C.POINTER(C.c_void_p), C.POINTER(Stats)]),
    ("kiops_status_string", C.c_char_p, [C.c_int]),
    ("kiops_device_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("kiops_apply", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("kiops_iop_basis", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p), C.c_int, C.c_int,
                                  C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]),
    ("kiops_small_expm", C.c_int, [C.c_int, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    ("kiops_stream_probe", C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p, C.c_int64, C.c_int,
                                     C.c_void_p]),
    ("kiops_controller_decide", C.c_int, [C.POINTER(CtrlIn), C.c_int, C.c_double, C.c_int,
                                          C.POINTER(CtrlOut)]),
    ("kiops_batch_plan", C.c_int, [C.c_int, C.POINTER(Problem), C.POINTER(Options), C.c_int,
                                   C.POINTER(C.c_size_t), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("kiops_phi_batch", C.c_int, [C.c_int, C.POINTER(Problem), C.POINTER(Options), C.c_int, C.c_void_p,
                                  C.c_size_t, C.c_void_p, C.POINTER(Stats)]),
    ("kiops_batch_tune", C.c_int, [C.c_int, C.POINTER(Problem), C.POINTER(Options), C.POINTER(C.c_int),
                                   C.c_int, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_int),
                                   C.POINTER(C.c_double)]),
    ("kiops_batch_tune_shape", C.c_int, [C.c_int, C.POINTER(Problem), C.POINTER(Options), C.POINTER(C.c_int),
                                         C.c_int, C.POINTER(C.c_int), C.c_int, C.c_void_p, C.c_size_t,
                                         C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                         C.POINTER(C.c_double)]),
    ("kiops_server_fixed_bytes", C.c_int, [C.c_int, C.POINTER(C.c_size_t), C.POINTER(C.c_int)]),
    ("kiops_server_create", C.c_int, [C.c_int, C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_void_p)]),
    ("kiops_server_submit", C.c_int, [C.c_void_p, C.POINTER(Problem), C.POINTER(C.c_int64)]),
    ("kiops_server_progress", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("kiops_server_result", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int), C.POINTER(Stats)]),
    ("kiops_server_destroy", C.c_int, [C.c_void_p]),
]

_lib = None


class KiopsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}")


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same soname; importing it first
    # makes this library bind to that one runtime instead of loading a second
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != KIOPS_OK:
        raise KiopsError(status, where)
