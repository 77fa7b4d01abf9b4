"""MI355X (gfx950) KIOPS phi-combination library: Python binding.

    w = phi_0(tau A) b_0 + tau phi_1(tau A) b_1 + ... + tau^p phi_p(tau A) b_p

(Gaudreault, Rainwater & Tokman, J. Comput. Phys. 372 (2018), Eq. (4)),
computed by the device-resident adaptive Krylov/IOP solver in ``libkiops.so``.
PyTorch supplies device memory and the stream; this module only marshals
arguments into the C ABI of ``include/kiops.h``.  There is no CPU fallback:
without the built library or a GPU every entry point raises.
"""

from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

from . import _lib
from ._lib import KiopsError  # noqa: F401

__all__ = ["Operator", "phi_combination", "phi_combination_noalloc", "phi_batch", "batch_tune", "Server", "iop_basis", "small_expm",
           "stream_probe", "controller_decide", "apply", "KiopsError"]


def _torch():
    import torch
    return torch


def _ptr(t) -> int:
    return int(t.data_ptr())


def _require_cuda_f64(t, n: Optional[int], name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} entries")


class Operator:
    """A stencil or CSR operator bound to a stream, with its workspace.

    Coefficient tensors are borrowed (the Operator keeps references): leave them
    unchanged during a call that uses the operator; between calls their
    contents may be rewritten in place (a Jacobian's reaction field updated
    every time step), and the next call reads the new values."""

    def __init__(self, kind: str, *, nx: int = 0, ny: int = 0, nz: int = 1, h: float = 1.0,
                 diff: float = 0.0, kappa=None, adv=(0.0, 0.0, 0.0), reaction=None, weights=None,
                 rowptr=None, col=None, val=None, precision: str = "fp64", stream=None):
        torch = _torch()
        lib = _lib.load()
        d = _lib.OperatorDesc()
        kinds = {"stencil2d": _lib.OP_STENCIL2D_5PT, "stencil3d": _lib.OP_STENCIL3D_7PT,
                 "csr": _lib.OP_CSR}
        if kind not in kinds:
            raise ValueError(f"unknown operator kind {kind}")
        d.kind = kinds[kind]
        d.precision = {"fp64": _lib.FP64, "mixed": _lib.MIXED}[precision]
        self._keep = []
        if kind == "csr":
            n = int(rowptr.numel()) - 1
            for t, nm, dt in ((rowptr, "rowptr", torch.int32), (col, "col", torch.int32),
                              (val, "val", torch.float64)):
                if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                    raise TypeError(f"{nm} must be a contiguous device tensor of {dt}")
            d.nrows, d.nnz = n, int(col.numel())
            d.rowptr, d.col, d.val = _ptr(rowptr), _ptr(col), _ptr(val)
            self._keep += [rowptr, col, val]
            self.n = n
        else:
            d.nx, d.ny, d.nz, d.h, d.diff = int(nx), int(ny), int(nz), float(h), float(diff)
            d.adv[0], d.adv[1], d.adv[2] = (float(a) for a in adv)
            self.n = int(nx) * int(ny) * int(nz)
            if kappa is not None:
                _require_cuda_f64(kappa, self.n, "kappa")
                d.kappa = _ptr(kappa)
                self._keep.append(kappa)
            if reaction is not None:
                _require_cuda_f64(reaction, self.n, "reaction")
                d.reaction = _ptr(reaction)
                self._keep.append(reaction)
            if weights is not None:   # general form: [5|7][N] per-cell weights
                nw = 5 if kind == "stencil2d" else 7
                _require_cuda_f64(weights, nw * self.n, "weights")
                d.weights = _ptr(weights)
                self._keep.append(weights)
        self.kind = kind
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._desc = d
        handle = C.c_void_p()
        _lib.check(lib.kiops_create_operator(C.byref(d), C.c_void_p(self.stream.cuda_stream),
                                             C.byref(handle)), "kiops_create_operator")
        self._h = handle
        self._ws = None
        self._lib = lib

    @classmethod
    def from_desc(cls, desc, device="cuda", precision: Optional[str] = None, stream=None):
        """Build from a workloads.StencilDesc / CsrDesc (numpy data copied to the device)."""
        torch = _torch()
        prec = precision or "fp64"
        if getattr(desc, "kind", None) == "csr":
            return cls("csr", rowptr=torch.as_tensor(desc.rowptr, dtype=torch.int32, device=device),
                       col=torch.as_tensor(desc.col, dtype=torch.int32, device=device),
                       val=torch.as_tensor(desc.val, dtype=torch.float64, device=device),
                       precision=prec, stream=stream)
        f = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64, device=device)  # noqa: E731
        wts = getattr(desc, "weights", None)
        return cls(desc.kind, nx=desc.nx, ny=desc.ny, nz=desc.nz, h=desc.h, diff=desc.diff,
                   kappa=f(desc.kappa), adv=desc.adv, reaction=f(desc.reaction),
                   weights=None if wts is None else f(wts).reshape(-1).contiguous(),
                   precision=prec, stream=stream)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.kiops_destroy_operator(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_info(self):
        cu, g = C.c_int(), C.c_int()
        _lib.check(self._lib.kiops_device_info(self._h, C.byref(cu), C.byref(g)), "kiops_device_info")
        return cu.value, g.value

    def workspace_bytes(self, p: int, q: int = 2, m_min: int = 0, m_max: int = 0,
                        max_substeps: int = 0) -> int:
        o = _lib.Options(m_min, m_max, max_substeps, 0)
        out = C.c_size_t()
        _lib.check(self._lib.kiops_workspace_bytes(self._h, p, q, C.byref(o), C.byref(out)),
                   "kiops_workspace_bytes")
        return out.value

    def ensure_workspace(self, nbytes: int):
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = _ptr(self._ws)
        aligned = (base + 255) // 256 * 256
        _lib.check(self._lib.kiops_set_workspace(self._h, C.c_void_p(aligned),
                                                 self._ws.numel() - (aligned - base)),
                   "kiops_set_workspace")


def _vec_ptrs(vectors: Sequence, n: int):
    arr = (C.c_void_p * len(vectors))()
    for k, v in enumerate(vectors):
        _require_cuda_f64(v, n, f"V[{k}]")
        arr[k] = _ptr(v)
    return arr


def phi_combination(op: Operator, tau: float, vectors: Sequence, tol: float = 1e-8,
                    m_init: int = 10, q: int = 2, m_min: int = 0, m_max: int = 0,
                    max_substeps: int = 0, out=None, check: bool = True, estimate: int = 0):
    """w = sum_k tau^k phi_k(tau A) vectors[k]; returns (w, stats dict, status).
    estimate: 0 the one-term error estimate (Eq. (36)), 1 the first two terms
    of Eq. (35), 2 the corrected scheme (KIOPS_ESTIMATE_*)."""
    torch = _torch()
    p = len(vectors) - 1
    V = _vec_ptrs(vectors, op.n)
    w = out if out is not None else torch.empty(op.n, dtype=torch.float64, device="cuda")
    _require_cuda_f64(w, op.n, "w")
    op.ensure_workspace(op.workspace_bytes(p, q, m_min, m_max, max_substeps))
    o = _lib.Options(m_min, m_max, max_substeps, int(estimate))
    st = _lib.Stats()
    status = op._lib.kiops_phi_combination(op._h, float(tau), p, V, float(tol), int(m_init), int(q),
                                           C.byref(o), C.c_void_p(_ptr(w)), C.byref(st))
    if check:
        _lib.check(status, "kiops_phi_combination")
    return w, st.as_dict(), status


def phi_combination_noalloc(op: Operator, tau: float, vectors: Sequence, out, tol: float = 1e-8,
                            m_init: int = 10, q: int = 2, m_min: int = 0, m_max: int = 0,
                            max_substeps: int = 0, check: bool = True):
    """phi_combination through the entry point that allocates nothing (the
    library's fixed scratch array is the workspace; the output buffer `out`
    is the caller's).  Returns (out, stats dict, status)."""
    p = len(vectors) - 1
    V = _vec_ptrs(vectors, op.n)
    _require_cuda_f64(out, op.n, "w")
    o = _lib.Options(m_min, m_max, max_substeps, 0)
    st = _lib.Stats()
    status = op._lib.kiops_phi_combination_noalloc(op._h, float(tau), p, V, float(tol), int(m_init), int(q),
                                                   C.byref(o), C.c_void_p(_ptr(out)), C.byref(st))
    if check:
        _lib.check(status, "kiops_phi_combination_noalloc")
    return out, st.as_dict(), status


def phi_combination_times(op: Operator, times: Sequence[float], vectors: Sequence, task: int = 2,
                          tol: float = 1e-8, m_init: int = 10, q: int = 2, m_min: int = 0, m_max: int = 0,
                          max_substeps: int = 0, outs=None, check: bool = True, estimate: int = 0):
    """Several output times T_1 < ... < T_n in one integration (Algorithms 1 and 3):
    outs[k] = sum_i T_k^i phi_i(T_k A) vectors[i] (task 2), times (1/T_k)^p for
    task 1.  Returns (list of w, stats dict, status)."""
    torch = _torch()
    p = len(vectors) - 1
    V = _vec_ptrs(vectors, op.n)
    n = len(times)
    if outs is None:
        outs = [torch.empty(op.n, dtype=torch.float64, device="cuda") for _ in range(n)]
    if len(outs) != n:
        raise ValueError("one output per time")
    for o in outs:
        _require_cuda_f64(o, op.n, "outs")
    op.ensure_workspace(op.workspace_bytes(p, q, m_min, m_max, max_substeps))
    o = _lib.Options(m_min, m_max, max_substeps, int(estimate))
    st = _lib.Stats()
    T = (C.c_double * n)(*[float(t) for t in times])
    Wp = (C.c_void_p * n)(*[_ptr(x) for x in outs])
    status = op._lib.kiops_phi_combination_times(op._h, n, T, int(task), p, V, float(tol), int(m_init), int(q),
                                                 C.byref(o), Wp, C.byref(st))
    if check:
        _lib.check(status, "kiops_phi_combination_times")
    return outs, st.as_dict(), status


_batch_ws = {}


def _batch_problems(problems):
    """Marshal (op, tau, vectors, tol, m_init, q, out) entries into kiops_problem structs."""
    torch = _torch()
    arr = (_lib.Problem * len(problems))()
    keep, outs = [], []
    for i, pr in enumerate(problems):
        op, tau, vectors = pr["op"], pr["tau"], pr["vectors"]
        V = _vec_ptrs(vectors, op.n)
        w = pr.get("out")
        if w is None:
            w = torch.empty(op.n, dtype=torch.float64, device="cuda")
        _require_cuda_f64(w, op.n, "w")
        arr[i].op = op._h.value
        arr[i].tau = float(tau)
        arr[i].p = len(vectors) - 1
        arr[i].q = int(pr.get("q", 2))
        arr[i].V = C.cast(V, C.POINTER(C.c_void_p))
        arr[i].tol = float(pr.get("tol", 1e-8))
        arr[i].m_init = int(pr.get("m_init", 10))
        arr[i].w = _ptr(w)
        keep.append(V)
        outs.append(w)
    return arr, keep, outs


def _batch_workspace(nbytes: int):
    torch = _torch()
    ws = _batch_ws.get("ws")
    if ws is None or ws.numel() < nbytes + 256:
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        _batch_ws["ws"] = ws
    base = _ptr(ws)
    aligned = (base + 255) // 256 * 256
    return aligned, ws.numel() - (aligned - base)


def phi_batch(problems: Sequence[dict], group_size: int = 0, m_min: int = 0, m_max: int = 0,
              max_substeps: int = 0, stream=None, tile_rows: int = 0):
    """Batched form: every problem (a dict with op, tau, vectors and optionally
    tol, m_init, q, out) solved in one persistent launch.  Returns
    (list of w, list of stats dicts, status, plan) with plan = (groups,
    group_size): the number of groups and the size of the shared groups (a
    problem with a large share of the work runs on a larger group of its own;
    stats[i]["grid_blocks"] is the size of the group that solved problem i).
    tile_rows: rows of the 2-D tile pass's tiles (16 (0), 8 or 4)."""
    torch = _torch()
    lib = _lib.load()
    arr, keep, outs = _batch_problems(problems)
    o = _lib.Options(m_min, m_max, max_substeps, 0, int(tile_rows))
    nbytes, groups, gs = C.c_size_t(), C.c_int(), C.c_int()
    _lib.check(lib.kiops_batch_plan(len(problems), arr, C.byref(o), int(group_size), C.byref(nbytes),
                                    C.byref(groups), C.byref(gs)), "kiops_batch_plan")
    ws, wsb = _batch_workspace(nbytes.value)
    stats = (_lib.Stats * len(problems))()
    s = stream if stream is not None else torch.cuda.current_stream()
    status = lib.kiops_phi_batch(len(problems), arr, C.byref(o), int(group_size), C.c_void_p(ws), wsb,
                                 C.c_void_p(s.cuda_stream), stats)
    return outs, [st.as_dict() for st in stats], status, (groups.value, gs.value)


def batch_tune(problems: Sequence[dict], candidates=(8, 16, 32, 64), m_min: int = 0, m_max: int = 0,
               stream=None, tile_rows: int = 0):
    """Autotuner of the batched form: the fastest group size among candidates and its time (ms)."""
    torch = _torch()
    lib = _lib.load()
    arr, keep, outs = _batch_problems(problems)
    o = _lib.Options(m_min, m_max, 0, 0, int(tile_rows))
    need = 0
    for c in candidates:
        nbytes, groups, gs = C.c_size_t(), C.c_int(), C.c_int()
        _lib.check(lib.kiops_batch_plan(len(problems), arr, C.byref(o), int(c), C.byref(nbytes),
                                        C.byref(groups), C.byref(gs)), "kiops_batch_plan")
        need = max(need, nbytes.value)
    ws, wsb = _batch_workspace(need)
    cand = (C.c_int * len(candidates))(*candidates)
    best, best_ms = C.c_int(), C.c_double()
    s = stream if stream is not None else torch.cuda.current_stream()
    _lib.check(lib.kiops_batch_tune(len(problems), arr, C.byref(o), cand, len(candidates), C.c_void_p(ws), wsb,
                                    C.c_void_p(s.cuda_stream), C.byref(best), C.byref(best_ms)),
               "kiops_batch_tune")
    return best.value, best_ms.value


def batch_tune_shape(problems: Sequence[dict], group_sizes=(8, 16, 32, 64), tile_rows=(16, 8, 4),
                     m_min: int = 0, m_max: int = 0, stream=None):
    """Autotuner over batch shapes: the fastest (group size, tile rows) pair
    among the candidates and its time (ms)."""
    torch = _torch()
    lib = _lib.load()
    arr, keep, outs = _batch_problems(problems)
    need = 0
    for r in tile_rows:
        o = _lib.Options(m_min, m_max, 0, 0, int(r))
        for c in group_sizes:
            nbytes, groups, gs = C.c_size_t(), C.c_int(), C.c_int()
            _lib.check(lib.kiops_batch_plan(len(problems), arr, C.byref(o), int(c), C.byref(nbytes),
                                            C.byref(groups), C.byref(gs)), "kiops_batch_plan")
            need = max(need, nbytes.value)
    ws, wsb = _batch_workspace(need)
    o = _lib.Options(m_min, m_max, 0, 0, 0)
    gcand = (C.c_int * len(group_sizes))(*group_sizes)
    rcand = (C.c_int * len(tile_rows))(*tile_rows)
    bg, br, bms = C.c_int(), C.c_int(), C.c_double()
    s = stream if stream is not None else torch.cuda.current_stream()
    _lib.check(lib.kiops_batch_tune_shape(len(problems), arr, C.byref(o), gcand, len(group_sizes), rcand,
                                          len(tile_rows), C.c_void_p(ws), wsb, C.c_void_p(s.cuda_stream),
                                          C.byref(bg), C.byref(br), C.byref(bms)),
               "kiops_batch_tune_shape")
    return bg.value, br.value, bms.value


class Server:
    """Served form: a long-lived launch that runs admitted requests on gangs of
    groups of workgroups (continuous batching).  pool_bytes is the HBM budget
    for the requests' workspaces; a request gets the smallest power-of-two gang
    of groups giving each workgroup at most points_per_workgroup grid points.
    While a server is open, do not synchronise the whole device
    (torch.cuda.synchronize) and do not run one-solve or batched launches: both
    need every CU and would wait for the server."""

    def __init__(self, pool_bytes: int, group_size: int = 16, points_per_workgroup: int = 0):
        torch = _torch()
        self._lib = lib = _lib.load()
        fixed, groups = C.c_size_t(), C.c_int()
        _lib.check(lib.kiops_server_fixed_bytes(int(group_size), C.byref(fixed), C.byref(groups)),
                   "kiops_server_fixed_bytes")
        self.groups = groups.value
        total = fixed.value + int(pool_bytes)
        self._ws = torch.empty(total + 256, dtype=torch.uint8, device="cuda")
        base = _ptr(self._ws)
        aligned = (base + 255) // 256 * 256
        self.run_stream = torch.cuda.Stream()
        self.io_stream = torch.cuda.Stream()
        torch.cuda.current_stream().synchronize()
        h = C.c_void_p()
        _lib.check(lib.kiops_server_create(int(group_size), int(points_per_workgroup), C.c_void_p(aligned), total,
                                           C.c_void_p(self.run_stream.cuda_stream),
                                           C.c_void_p(self.io_stream.cuda_stream), C.byref(h)),
                   "kiops_server_create")
        self._h = h
        self._keep = {}

    def submit(self, op: Operator, tau: float, vectors: Sequence, tol: float = 1e-8, m_init: int = 10,
               q: int = 2, out=None) -> int:
        torch = _torch()
        arr, keep, outs = _batch_problems([dict(op=op, tau=tau, vectors=vectors, tol=tol, m_init=m_init, q=q,
                                                out=out)])
        torch.cuda.current_stream().synchronize()     # inputs written on this stream are complete
        t = C.c_int64()
        _lib.check(self._lib.kiops_server_submit(self._h, arr, C.byref(t)), "kiops_server_submit")
        self._keep[t.value] = (op, list(vectors), outs[0], keep)
        return t.value

    def progress(self):
        r, w = C.c_int(), C.c_int()
        _lib.check(self._lib.kiops_server_progress(self._h, C.byref(r), C.byref(w)), "kiops_server_progress")
        return r.value, w.value

    def result(self, ticket: int):
        """(done, stats dict, w); after done the ticket is released."""
        d = C.c_int()
        st = _lib.Stats()
        _lib.check(self._lib.kiops_server_result(self._h, int(ticket), C.byref(d), C.byref(st)),
                   "kiops_server_result")
        if not d.value:
            return False, None, None
        op, vectors, w, keep = self._keep.pop(ticket)
        return True, st.as_dict(), w

    def close(self):
        if getattr(self, "_h", None):
            status = self._lib.kiops_server_destroy(self._h)
            self._h = None
            _lib.check(status, "kiops_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def iop_basis(op: Operator, vectors: Sequence, m: int, q: int = 2):
    """First-substep basis and H after m steps of Algorithm 2 (diagnostics).
    Returns (basis (j+1, N+p) or (j, N+p) after breakdown, H (m+1, m), j, beta, nu)."""
    torch = _torch()
    p = len(vectors) - 1
    V = _vec_ptrs(vectors, op.n)
    need = op.workspace_bytes(p, q, m_min=1, m_max=m) + 8 * op.n + 256
    op.ensure_workspace(need)
    basis = torch.zeros((m + 1, op.n + p), dtype=torch.float64, device="cuda")
    H = torch.zeros((m + 1, m), dtype=torch.float64, device="cuda")
    j, beta, nu = C.c_int(), C.c_double(), C.c_double()
    _lib.check(op._lib.kiops_iop_basis(op._h, p, V, m, q, C.c_void_p(_ptr(basis)), C.c_void_p(_ptr(H)),
                                       C.byref(j), C.byref(beta), C.byref(nu)), "kiops_iop_basis")
    return basis, H, j.value, beta.value, nu.value


def small_expm(Hs, tau: float, stream=None):
    """exp(tau Hs) for a device (n, n) float64 matrix by the device routine."""
    torch = _torch()
    lib = _lib.load()
    n = int(Hs.shape[0])
    Hs = Hs.contiguous()
    _require_cuda_f64(Hs, n * n, "Hs")
    F = torch.empty_like(Hs)
    scratch = torch.empty(_lib.EXPM_SCRATCH_DOUBLES, dtype=torch.float64, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    _lib.check(lib.kiops_small_expm(n, C.c_void_p(_ptr(Hs)), float(tau), C.c_void_p(_ptr(F)),
                                    C.c_void_p(_ptr(scratch)), C.c_void_p(s.cuda_stream)),
               "kiops_small_expm")
    return F


def apply(op: Operator, x, y=None):
    """y = A x (FP64) by the library's operator kernel, enqueued on the
    operator's stream; returns y (allocated when not given)."""
    torch = _torch()
    n = op.n
    _require_cuda_f64(x, n, "x")
    if y is None:
        y = torch.empty_like(x)
    _require_cuda_f64(y, n, "y")
    _lib.check(op._lib.kiops_apply(op._h, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y))), "kiops_apply")
    return y


def stream_probe(srcs: Sequence, dst, blocks: int, stream=None) -> None:
    """dst = sum(srcs) by the library's plain streaming kernel on `blocks`
    workgroups (enqueued on the stream, not waited for); a bandwidth probe."""
    torch = _torch()
    lib = _lib.load()
    n = int(dst.numel())
    _require_cuda_f64(dst, n, "dst")
    arr = (C.c_void_p * len(srcs))()
    for k, t in enumerate(srcs):
        _require_cuda_f64(t, n, f"src[{k}]")
        arr[k] = _ptr(t)
    s = stream if stream is not None else torch.cuda.current_stream()
    _lib.check(lib.kiops_stream_probe(arr, len(srcs), C.c_void_p(_ptr(dst)), n, int(blocks),
                                      C.c_void_p(s.cuda_stream)), "kiops_stream_probe")


def controller_decide(state: dict, j: int, eps: float, breakdown: bool) -> dict:
    """One decision of the device controller (host copy of the same code)."""
    lib = _lib.load()
    ci = _lib.CtrlIn()
    for k, v in state.items():
        setattr(ci, k, v)
    co = _lib.CtrlOut()
    _lib.check(lib.kiops_controller_decide(C.byref(ci), int(j), float(eps), int(bool(breakdown)),
                                           C.byref(co)), "kiops_controller_decide")
    return {"accept": bool(co.accept), "m_new": co.m_new, "branch": _lib.BRANCH_NAMES[co.branch],
            "tau_new": co.tau_new, "omega": co.omega}
