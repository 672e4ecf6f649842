"""Python binding of the MI355X Red-Light-Green-Light library (``librlgl.so``).

The functions below carry the names of the C ABI in ``include/rlgl.h`` and do
argument marshalling only; every step of the method runs in the HIP kernels.
PyTorch provides device memory (the graph arrays, the workspace, the output)
and the stream.  There is no fallback: importing this package fails when the
built library is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime that the library then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlgl.so")

RLGL_OK, RLGL_EINVAL, RLGL_ENOMEM, RLGL_EHIP = 0, -1, -2, -3
RLGL_EZERO_HISTORY, RLGL_ENOT_CONVERGED, RLGL_ENONFINITE, RLGL_EBUSY = -4, -5, -6, -7
SCHED_ALL, SCHED_THRESHOLD, SCHED_TOPK, SCHED_MAXC, SCHED_PC = 0, 1, 2, 3, 4
FP64, FP32C_FP64H, FP32C_KAHANH = 0, 1, 2
ROUTE_PUSH, ROUTE_PULL, ROUTE_AUTO = 0, 1, 2

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EZERO_HISTORY", -5: "ENOT_CONVERGED",
                -6: "ENONFINITE"}


class rlgl_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("csr_rowptr", ctypes.c_void_p), ("csr_col", ctypes.c_void_p), ("csr_val", ctypes.c_void_p),
                ("csc_colptr", ctypes.c_void_p), ("csc_row", ctypes.c_void_p), ("csc_val", ctypes.c_void_p),
                ("damping", ctypes.c_double)]


class rlgl_options(ctypes.Structure):
    _fields_ = [("sched", ctypes.c_int32), ("r", ctypes.c_double), ("k", ctypes.c_int64),
                ("theta_period", ctypes.c_int32), ("precision", ctypes.c_int32), ("route", ctypes.c_int32),
                ("pull_alpha", ctypes.c_double), ("check_period", ctypes.c_int32),
                ("record_green", ctypes.c_int32), ("refresh", ctypes.c_int32), ("relabel", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class rlgl_step_info(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("green", ctypes.c_int64), ("green_total", ctypes.c_int64),
                ("edges_pushed", ctypes.c_int64), ("l1_cash", ctypes.c_double), ("h_sum", ctypes.c_double),
                ("resid", ctypes.c_double), ("theta", ctypes.c_double), ("cash_sum", ctypes.c_double),
                ("status", ctypes.c_int32), ("last_route", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class rlgl_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("bytes_touched", ctypes.c_double), ("green_links", ctypes.c_int64)]


BATCH_LOCKSTEP = 1


class rlgl_batch_graphs(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int32), ("node_off", ctypes.c_void_p), ("edge_off", ctypes.c_void_p),
                ("damping", ctypes.c_void_p), ("csr_rowptr", ctypes.c_void_p), ("csr_col", ctypes.c_void_p),
                ("csr_val", ctypes.c_void_p), ("csc_colptr", ctypes.c_void_p), ("csc_row", ctypes.c_void_p),
                ("csc_val", ctypes.c_void_p), ("tol_l1", ctypes.c_void_p)]


class rlgl_batch_options(ctypes.Structure):
    _fields_ = [("sched", ctypes.c_int32), ("r", ctypes.c_double), ("precision", ctypes.c_int32),
                ("eps", ctypes.c_double), ("max_steps", ctypes.c_int64), ("refresh", ctypes.c_int32),
                ("wg_size", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("check_period", ctypes.c_int32), ("relabel", ctypes.c_int32)]


class rlgl_chain_result(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("edges_pushed", ctypes.c_int64), ("resid", ctypes.c_double),
                ("h_sum", ctypes.c_double), ("status", ctypes.c_int32), ("green_steps", ctypes.c_int32),
                ("start_us", ctypes.c_double), ("end_us", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class rlgl_pool_options(ctypes.Structure):
    _fields_ = [("sched", ctypes.c_int32), ("r", ctypes.c_double), ("precision", ctypes.c_int32),
                ("refresh", ctypes.c_int32), ("wg_size", ctypes.c_int32), ("max_chains", ctypes.c_int32),
                ("max_steps", ctypes.c_int64), ("route_per_cu", ctypes.c_int32)]


class rlgl_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("csr_rowptr", ctypes.c_void_p),
                ("csc_colptr", ctypes.c_void_p), ("csc_row", ctypes.c_void_p), ("damping", ctypes.c_double),
                ("tol_l1", ctypes.c_double)]


EXPORTED = ["rlgl_default_options", "rlgl_workspace_bytes", "rlgl_create", "rlgl_step", "rlgl_solve",
            "rlgl_destroy", "rlgl_last_error", "rlgl_reset", "rlgl_get_state", "rlgl_set_state",
            "rlgl_get_green", "rlgl_refresh", "rlgl_profile_enable", "rlgl_profile_read",
            "rlgl_batch_default_options", "rlgl_batch_workspace_bytes", "rlgl_batch_create", "rlgl_batch_solve",
            "rlgl_batch_autotune", "rlgl_batch_destroy",
            "rlgl_pool_default_options", "rlgl_pool_workspace_bytes", "rlgl_pool_footprint", "rlgl_pool_create",
            "rlgl_pool_admit", "rlgl_pool_advance", "rlgl_pool_launch", "rlgl_pool_wait", "rlgl_pool_poll",
            "rlgl_pool_result", "rlgl_pool_release", "rlgl_pool_destroy", "rlgl_validate_scratch_bytes",
            "rlgl_validate", "rlgl_step_mask", "rlgl_small_max_n", "rlgl_small_workspace_bytes",
            "rlgl_solve_small", "rlgl_solve_small_static", "rlgl_pull_plan", "rlgl_batch_chain_plan"]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"the HIP library {path} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    G, O, I = ctypes.POINTER(rlgl_graph), ctypes.POINTER(rlgl_options), ctypes.POINTER(rlgl_step_info)
    lib.rlgl_default_options.argtypes = [O]
    lib.rlgl_default_options.restype = None
    lib.rlgl_workspace_bytes.argtypes = [G, O]
    lib.rlgl_workspace_bytes.restype = ctypes.c_size_t
    lib.rlgl_validate_scratch_bytes.argtypes = [G]
    lib.rlgl_validate_scratch_bytes.restype = ctypes.c_size_t
    lib.rlgl_validate.argtypes = [G, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(f64)]
    lib.rlgl_validate.restype = i32
    lib.rlgl_create.argtypes = [G, O, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.rlgl_create.restype = i32
    lib.rlgl_step.argtypes = [vp, i32, I]
    lib.rlgl_step.restype = i32
    lib.rlgl_step_mask.argtypes = [vp, vp, I]
    lib.rlgl_step_mask.restype = i32
    lib.rlgl_solve.argtypes = [vp, f64, i64, vp, I]
    lib.rlgl_solve.restype = i32
    lib.rlgl_small_max_n.argtypes = [i32]
    lib.rlgl_small_max_n.restype = i32
    lib.rlgl_small_workspace_bytes.argtypes = [i32]
    lib.rlgl_small_workspace_bytes.restype = ctypes.c_size_t
    lib.rlgl_solve_small.argtypes = [G, O, f64, i64, vp, vp, ctypes.c_size_t, vp, I]
    lib.rlgl_solve_small.restype = i32
    lib.rlgl_solve_small_static.argtypes = [G, O, f64, i64, vp, vp, I]
    lib.rlgl_solve_small_static.restype = i32
    P64 = ctypes.POINTER(i64)
    lib.rlgl_pull_plan.argtypes = [vp, i32, i64, vp, i64, vp, i64, P64, P64]
    lib.rlgl_pull_plan.restype = i64
    lib.rlgl_batch_chain_plan.argtypes = [vp, i32, i64, vp, i64, vp, i64, P64, P64, P64]
    lib.rlgl_batch_chain_plan.restype = i64
    lib.rlgl_destroy.argtypes = [vp]
    lib.rlgl_destroy.restype = None
    lib.rlgl_last_error.argtypes = []
    lib.rlgl_last_error.restype = ctypes.c_char_p
    lib.rlgl_reset.argtypes = [vp]
    lib.rlgl_reset.restype = i32
    lib.rlgl_get_state.argtypes = [vp, vp, vp, I]
    lib.rlgl_get_state.restype = i32
    lib.rlgl_set_state.argtypes = [vp, vp, vp, f64, i64]
    lib.rlgl_set_state.restype = i32
    lib.rlgl_refresh.argtypes = [vp, I]
    lib.rlgl_refresh.restype = i32
    lib.rlgl_get_green.argtypes = [vp, vp]
    lib.rlgl_get_green.restype = i32
    lib.rlgl_profile_enable.argtypes = [vp, i32]
    lib.rlgl_profile_enable.restype = i32
    lib.rlgl_profile_read.argtypes = [vp, ctypes.POINTER(rlgl_kernel_stat), i32]
    lib.rlgl_profile_read.restype = i32
    BG, BO = ctypes.POINTER(rlgl_batch_graphs), ctypes.POINTER(rlgl_batch_options)
    lib.rlgl_batch_default_options.argtypes = [BO]
    lib.rlgl_batch_default_options.restype = None
    lib.rlgl_batch_workspace_bytes.argtypes = [BG, BO]
    lib.rlgl_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.rlgl_batch_create.argtypes = [BG, BO, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.rlgl_batch_create.restype = i32
    lib.rlgl_batch_solve.argtypes = [vp, vp, ctypes.POINTER(rlgl_chain_result), ctypes.POINTER(f64)]
    lib.rlgl_batch_solve.restype = i32
    lib.rlgl_batch_autotune.argtypes = [vp, vp, BO]
    lib.rlgl_batch_autotune.restype = i32
    lib.rlgl_batch_destroy.argtypes = [vp]
    lib.rlgl_batch_destroy.restype = None
    PO, RQ = ctypes.POINTER(rlgl_pool_options), ctypes.POINTER(rlgl_request)
    lib.rlgl_pool_default_options.argtypes = [PO]
    lib.rlgl_pool_default_options.restype = None
    lib.rlgl_pool_workspace_bytes.argtypes = [PO, ctypes.c_size_t]
    lib.rlgl_pool_workspace_bytes.restype = ctypes.c_size_t
    lib.rlgl_pool_footprint.argtypes = [PO, i32, i64]
    lib.rlgl_pool_footprint.restype = ctypes.c_size_t
    lib.rlgl_pool_create.argtypes = [PO, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.rlgl_pool_create.restype = i32
    lib.rlgl_pool_admit.argtypes = [vp, RQ, ctypes.POINTER(i32)]
    lib.rlgl_pool_admit.restype = i32
    lib.rlgl_pool_advance.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.rlgl_pool_advance.restype = i32
    lib.rlgl_pool_launch.argtypes = [vp, i32]
    lib.rlgl_pool_launch.restype = i32
    lib.rlgl_pool_wait.argtypes = [vp, ctypes.POINTER(i32)]
    lib.rlgl_pool_wait.restype = i32
    lib.rlgl_pool_poll.argtypes = [vp, ctypes.POINTER(i32), i32]
    lib.rlgl_pool_poll.restype = i32
    lib.rlgl_pool_result.argtypes = [vp, i32, ctypes.POINTER(rlgl_chain_result), ctypes.POINTER(vp)]
    lib.rlgl_pool_result.restype = i32
    lib.rlgl_pool_release.argtypes = [vp, i32]
    lib.rlgl_pool_release.restype = i32
    lib.rlgl_pool_destroy.argtypes = [vp]
    lib.rlgl_pool_destroy.restype = None
    return lib


_lib = load_library(os.environ.get("RLGL_LIBRARY", LIB_PATH))


class RlglError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {rlgl_last_error()}")


def _check(st: int, what: str, allow=()):
    if st != RLGL_OK and st not in allow:
        raise RlglError(st, what)
    return st


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


# ---------------------------------------------------------------- C names

def rlgl_default_options(**overrides) -> rlgl_options:
    o = rlgl_options()
    _lib.rlgl_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def rlgl_last_error() -> str:
    return _lib.rlgl_last_error().decode()


def rlgl_workspace_bytes(graph: rlgl_graph, opt: rlgl_options) -> int:
    return int(_lib.rlgl_workspace_bytes(ctypes.byref(graph), ctypes.byref(opt)))


def rlgl_validate_scratch_bytes(graph: rlgl_graph) -> int:
    return int(_lib.rlgl_validate_scratch_bytes(ctypes.byref(graph)))


def rlgl_validate(graph: rlgl_graph, precision: int, scratch, scratch_bytes: int, stream=None) -> float:
    """Raises RlglError when the graph breaks the contract; returns max |row sum - 1|."""
    dev = ctypes.c_double(0.0)
    st = _lib.rlgl_validate(ctypes.byref(graph), int(precision), _ptr(scratch), int(scratch_bytes),
                            _stream_handle(stream), ctypes.byref(dev))
    _check(st, "rlgl_validate")
    return dev.value


def rlgl_create(graph: rlgl_graph, opt: rlgl_options, workspace, ws_bytes: int, stream=None):
    ctx = ctypes.c_void_p()
    st = _lib.rlgl_create(ctypes.byref(graph), ctypes.byref(opt), _ptr(workspace), int(ws_bytes),
                          _stream_handle(stream), ctypes.byref(ctx))
    _check(st, "rlgl_create")
    return ctx


def rlgl_step(ctx, nsteps: int) -> rlgl_step_info:
    info = rlgl_step_info()
    _check(_lib.rlgl_step(ctx, int(nsteps), ctypes.byref(info)), "rlgl_step")
    return info


def rlgl_step_mask(ctx, mask) -> rlgl_step_info:
    """One step with the green set {i : mask[i] != 0} (device uint8 tensor or pointer)."""
    info = rlgl_step_info()
    _check(_lib.rlgl_step_mask(ctx, _ptr(mask), ctypes.byref(info)), "rlgl_step_mask")
    return info


def rlgl_solve(ctx, eps: float, max_steps: int, pi_out=None, raise_on_error: bool = True):
    info = rlgl_step_info()
    st = _lib.rlgl_solve(ctx, float(eps), int(max_steps), _ptr(pi_out), ctypes.byref(info))
    if raise_on_error:
        _check(st, "rlgl_solve")
    return st, info


def _plan(fn, colptr, batched: bool):
    """Runs a host-only plan builder on int32 column pointers (numpy)."""
    import numpy as np
    cp = np.ascontiguousarray(colptr, dtype=np.int32)
    n = cp.size - 1
    nnz = int(cp[-1]) if cp.size else 0
    n_long, n_pieces, bound = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    extra = [ctypes.byref(n_pieces)] if batched else []
    # first call sizes the output (RLGL_ENOMEM with zero capacity unless the plan is empty)
    cnt = fn(cp.ctypes.data, n, nnz, None, 0, None, 0, ctypes.byref(n_long), *extra, ctypes.byref(bound))
    if cnt < 0 and cnt != RLGL_ENOMEM:
        raise RlglError(int(cnt), "plan")
    cap_items = int(bound.value)
    items = np.zeros((max(cap_items, 1), 4), dtype=np.int32)
    longs = np.zeros(max(int(n_long.value), 1), dtype=np.int32)
    cnt = fn(cp.ctypes.data, n, nnz, items.ctypes.data, cap_items, longs.ctypes.data, int(n_long.value),
             ctypes.byref(n_long), *extra, ctypes.byref(bound))
    if cnt < 0:
        raise RlglError(int(cnt), "plan")
    out = {"items": items[:cnt], "long_cols": longs[:int(n_long.value)], "item_bound": int(bound.value)}
    if batched:
        out["n_pieces"] = int(n_pieces.value)
    return out


def rlgl_pull_plan(colptr) -> dict:
    """The single-chain pull plan of CSC column pointers (host numpy array)."""
    return _plan(_lib.rlgl_pull_plan, colptr, False)


def rlgl_batch_chain_plan(colptr) -> dict:
    """The batched engine's plan of one chain's CSC column pointers (host numpy array)."""
    return _plan(_lib.rlgl_batch_chain_plan, colptr, True)


def rlgl_small_max_n(precision: int) -> int:
    return int(_lib.rlgl_small_max_n(int(precision)))


def rlgl_small_workspace_bytes(n: int) -> int:
    return int(_lib.rlgl_small_workspace_bytes(int(n)))


def rlgl_solve_small(graph: rlgl_graph, opt: rlgl_options, eps: float, max_steps: int, pi_out, workspace,
                     ws_bytes: int, stream=None, raise_on_error: bool = True):
    info = rlgl_step_info()
    st = _lib.rlgl_solve_small(ctypes.byref(graph), ctypes.byref(opt), float(eps), int(max_steps), _ptr(pi_out),
                               _ptr(workspace), int(ws_bytes), _stream_handle(stream), ctypes.byref(info))
    if raise_on_error:
        _check(st, "rlgl_solve_small")
    return st, info


RLGL_SMALL_STATIC_BYTES = 512 * 1024


def rlgl_solve_small_static(graph: rlgl_graph, opt: rlgl_options, eps: float, max_steps: int, pi_out, stream=None,
                            raise_on_error: bool = True):
    """rlgl_solve_small on the library's static device workspace (no allocation)."""
    info = rlgl_step_info()
    st = _lib.rlgl_solve_small_static(ctypes.byref(graph), ctypes.byref(opt), float(eps), int(max_steps),
                                      _ptr(pi_out), _stream_handle(stream), ctypes.byref(info))
    if raise_on_error:
        _check(st, "rlgl_solve_small_static")
    return st, info


def rlgl_destroy(ctx) -> None:
    _lib.rlgl_destroy(ctx)


def rlgl_reset(ctx) -> None:
    _check(_lib.rlgl_reset(ctx), "rlgl_reset")


def rlgl_get_state(ctx, C_out=None, H_out=None) -> rlgl_step_info:
    info = rlgl_step_info()
    _check(_lib.rlgl_get_state(ctx, _ptr(C_out), _ptr(H_out), ctypes.byref(info)), "rlgl_get_state")
    return info


def rlgl_set_state(ctx, C, H, h_sum: float, t: int) -> None:
    _check(_lib.rlgl_set_state(ctx, _ptr(C), _ptr(H), float(h_sum), int(t)), "rlgl_set_state")


def rlgl_refresh(ctx) -> rlgl_step_info:
    info = rlgl_step_info()
    _check(_lib.rlgl_refresh(ctx, ctypes.byref(info)), "rlgl_refresh")
    return info


def rlgl_get_green(ctx, mask_out) -> None:
    _check(_lib.rlgl_get_green(ctx, _ptr(mask_out)), "rlgl_get_green")


def rlgl_profile_enable(ctx, on: bool) -> None:
    _check(_lib.rlgl_profile_enable(ctx, 1 if on else 0), "rlgl_profile_enable")


def rlgl_profile_read(ctx):
    buf = (rlgl_kernel_stat * 8)()
    m = _lib.rlgl_profile_read(ctx, buf, 8)
    if m < 0:
        raise RlglError(m, "rlgl_profile_read")
    return {buf[i].name.decode(): {"launches": buf[i].launches, "ms": buf[i].ms, "bytes": buf[i].bytes,
                                   "bytes_touched": buf[i].bytes_touched, "green_links": buf[i].green_links}
            for i in range(m)}


def rlgl_batch_default_options(**overrides) -> rlgl_batch_options:
    o = rlgl_batch_options()
    _lib.rlgl_batch_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def rlgl_batch_workspace_bytes(graphs: rlgl_batch_graphs, opt: rlgl_batch_options) -> int:
    return int(_lib.rlgl_batch_workspace_bytes(ctypes.byref(graphs), ctypes.byref(opt)))


def rlgl_batch_create(graphs: rlgl_batch_graphs, opt: rlgl_batch_options, workspace, ws_bytes: int, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.rlgl_batch_create(ctypes.byref(graphs), ctypes.byref(opt), _ptr(workspace), int(ws_bytes),
                                  _stream_handle(stream), ctypes.byref(h)), "rlgl_batch_create")
    return h


def rlgl_batch_solve(handle, pi_out, n_chains: int, raise_on_error: bool = True):
    res = (rlgl_chain_result * n_chains)()
    ms = ctypes.c_double(0.0)
    st = _lib.rlgl_batch_solve(handle, _ptr(pi_out), res, ctypes.byref(ms))
    if raise_on_error:
        _check(st, "rlgl_batch_solve")
    return st, [r.as_dict() for r in res], ms.value


def rlgl_batch_autotune(handle, pi_out) -> rlgl_batch_options:
    best = rlgl_batch_options()
    _check(_lib.rlgl_batch_autotune(handle, _ptr(pi_out), ctypes.byref(best)), "rlgl_batch_autotune")
    return best


def rlgl_batch_destroy(handle) -> None:
    _lib.rlgl_batch_destroy(handle)


def rlgl_pool_default_options(**overrides) -> rlgl_pool_options:
    o = rlgl_pool_options()
    _lib.rlgl_pool_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def rlgl_pool_workspace_bytes(opt: rlgl_pool_options, arena_bytes: int) -> int:
    return int(_lib.rlgl_pool_workspace_bytes(ctypes.byref(opt), int(arena_bytes)))


def rlgl_pool_footprint(opt: rlgl_pool_options, n: int, nnz: int) -> int:
    return int(_lib.rlgl_pool_footprint(ctypes.byref(opt), int(n), int(nnz)))


def rlgl_pool_create(opt: rlgl_pool_options, workspace, ws_bytes: int, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.rlgl_pool_create(ctypes.byref(opt), _ptr(workspace), int(ws_bytes), _stream_handle(stream),
                                 ctypes.byref(h)), "rlgl_pool_create")
    return h


def rlgl_pool_admit(handle, req: rlgl_request):
    """Slot of the admitted chain, or None when the pool is full right now."""
    slot = ctypes.c_int32(-1)
    st = _lib.rlgl_pool_admit(handle, ctypes.byref(req), ctypes.byref(slot))
    if st == RLGL_EBUSY:
        return None
    _check(st, "rlgl_pool_admit")
    return slot.value


def rlgl_pool_advance(handle, iterations: int) -> int:
    running = ctypes.c_int32(0)
    _check(_lib.rlgl_pool_advance(handle, int(iterations), ctypes.byref(running)), "rlgl_pool_advance")
    return running.value


def rlgl_pool_launch(handle, iterations: int) -> None:
    _check(_lib.rlgl_pool_launch(handle, int(iterations)), "rlgl_pool_launch")


def rlgl_pool_wait(handle) -> int:
    running = ctypes.c_int32(0)
    _check(_lib.rlgl_pool_wait(handle, ctypes.byref(running)), "rlgl_pool_wait")
    return running.value


def rlgl_pool_poll(handle, max_slots: int = 1024):
    buf = (ctypes.c_int32 * max_slots)()
    m = _lib.rlgl_pool_poll(handle, buf, max_slots)
    if m < 0:
        raise RlglError(m, "rlgl_pool_poll")
    return [buf[i] for i in range(m)]


def rlgl_pool_result(handle, slot: int):
    r = rlgl_chain_result()
    ptr = ctypes.c_void_p()
    _check(_lib.rlgl_pool_result(handle, int(slot), ctypes.byref(r), ctypes.byref(ptr)), "rlgl_pool_result")
    return r.as_dict(), ptr.value


def rlgl_pool_release(handle, slot: int) -> None:
    _check(_lib.rlgl_pool_release(handle, int(slot)), "rlgl_pool_release")


def rlgl_pool_destroy(handle) -> None:
    _lib.rlgl_pool_destroy(handle)


def _stream_handle(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------ convenience layer

class DeviceGraph:
    """Device copies (torch tensors) of a chain's CSR and CSC arrays.

    ``rowptr``/``col`` (and optionally ``colptr``/``row``/``perm``) are host
    arrays; ``val`` is 1/outdeg per stored link as float64 (or None for the
    implicit form).  Values are stored as float64 for FP64 and float32
    otherwise.
    """

    def __init__(self, n, rowptr, col, damping, val=None, colptr=None, row=None, perm=None, precision=FP32C_FP64H,
                 device="cuda"):
        import numpy as np
        vdt = torch.float64 if precision == FP64 else torch.float32
        self.n = int(n)
        self.nnz = int(rowptr[-1])
        self.damping = float(damping)
        self.precision = precision
        self.rowptr = torch.from_numpy(np.ascontiguousarray(rowptr, dtype=np.int32)).to(device)
        self.col = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).to(device)
        self.val = None if val is None else torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).to(
            device=device, dtype=vdt)
        self.colptr = self.row = self.cval = None
        if colptr is not None:
            self.colptr = torch.from_numpy(np.ascontiguousarray(colptr, dtype=np.int32)).to(device)
            self.row = torch.from_numpy(np.ascontiguousarray(row, dtype=np.int32)).to(device)
            if val is not None:
                cv = np.ascontiguousarray(np.asarray(val, dtype=np.float64)[perm])
                self.cval = torch.from_numpy(cv).to(device=device, dtype=vdt)

    @classmethod
    def from_workload(cls, g, precision=FP32C_FP64H, with_csc=True, explicit_val=True, device="cuda"):
        val = g.val() if explicit_val else None
        if with_csc:
            colptr, row, perm = g.csc()
        else:
            colptr = row = perm = None
        return cls(g.n, g.rowptr, g.col, g.c, val, colptr, row, perm, precision, device)

    def validate(self, stream=None) -> float:
        """rlgl_validate on these arrays (scratch from torch); returns max |row sum - 1|."""
        g = self.struct()
        nbytes = rlgl_validate_scratch_bytes(g)
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.rowptr.device)
        return rlgl_validate(g, self.precision, scratch, nbytes, stream)

    def struct(self) -> rlgl_graph:
        return rlgl_graph(self.n, self.nnz, _ptr(self.rowptr), _ptr(self.col), _ptr(self.val),
                          _ptr(self.colptr), _ptr(self.row), _ptr(self.cval), self.damping)


class Solver:
    """Owns one context, its workspace tensor and an output buffer."""

    def __init__(self, dg: DeviceGraph, stream=None, **options):
        options.setdefault("precision", dg.precision)
        self.dg = dg
        self.graph = dg.struct()
        self.opt = rlgl_default_options(**options)
        self.ws_bytes = rlgl_workspace_bytes(self.graph, self.opt)
        if self.ws_bytes == 0:
            raise RlglError(RLGL_EINVAL, "rlgl_workspace_bytes")
        dev = dg.rowptr.device
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.stream = stream
        self.ctx = rlgl_create(self.graph, self.opt, self.workspace, self.ws_bytes, stream)
        self.pi = torch.empty(dg.n, dtype=torch.float64, device=dev)

    def step(self, nsteps: int = 1) -> dict:
        return rlgl_step(self.ctx, nsteps).as_dict()

    def step_mask(self, mask) -> dict:
        """One step whose green set is {i : mask[i] != 0} (uint8 tensor of n on the device)."""
        if mask.dtype != torch.uint8 or mask.numel() != self.dg.n or not mask.is_cuda:
            raise ValueError("mask must be a device uint8 tensor of n entries")
        return rlgl_step_mask(self.ctx, mask.contiguous()).as_dict()

    def solve(self, eps: float, max_steps: int = 1_000_000, raise_on_error: bool = True):
        st, info = rlgl_solve(self.ctx, eps, max_steps, self.pi, raise_on_error)
        return st, info.as_dict()

    def reset(self):
        rlgl_reset(self.ctx)

    def refresh(self) -> dict:
        return rlgl_refresh(self.ctx).as_dict()

    def state(self):
        dev = self.dg.rowptr.device
        C = torch.empty(self.dg.n, dtype=torch.float64, device=dev)
        H = torch.empty(self.dg.n, dtype=torch.float64, device=dev)
        info = rlgl_get_state(self.ctx, C, H)
        return C, H, info.as_dict()

    def set_state(self, C, H, h_sum=float("nan"), t: int = 2):
        rlgl_set_state(self.ctx, C, H, h_sum, t)

    def green(self):
        m = torch.empty(self.dg.n, dtype=torch.uint8, device=self.dg.rowptr.device)
        rlgl_get_green(self.ctx, m)
        return m

    def close(self):
        if self.ctx is not None:
            rlgl_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SmallSolver:
    """One-workgroup solves of a small chain (rlgl_solve_small): the options,
    a workspace tensor and an output buffer."""

    def __init__(self, dg: DeviceGraph, stream=None, **options):
        options.setdefault("precision", dg.precision)
        self.dg = dg
        self.graph = dg.struct()
        self.opt = rlgl_default_options(**options)
        self.ws_bytes = rlgl_small_workspace_bytes(dg.n)
        dev = dg.rowptr.device
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.stream = stream
        self.pi = torch.empty(dg.n, dtype=torch.float64, device=dev)

    def solve(self, eps: float, max_steps: int = 1_000_000, raise_on_error: bool = True):
        st, info = rlgl_solve_small(self.graph, self.opt, eps, max_steps, self.pi, self.workspace, self.ws_bytes,
                                    self.stream, raise_on_error)
        return st, info.as_dict()


class DeviceBatch:
    """Concatenated device arrays of many chains (CSR and CSC, local node ids).

    ``graphs`` is a sequence of objects with ``n``, ``rowptr``, ``col``, ``c``,
    ``val(dtype)`` and ``csc()`` (as ``workloads.Graph``).
    """

    def __init__(self, graphs, precision=FP32C_KAHANH, explicit_val=False, device="cuda", tol_l1=None):
        import numpy as np
        self.tol_l1 = None if tol_l1 is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(tol_l1, dtype=np.float64), (len(graphs),)))
        vdt = np.float64 if precision == FP64 else np.float32
        self.precision = precision
        self.n_chains = len(graphs)
        ns = np.array([g.n for g in graphs], dtype=np.int64)
        ms = np.array([int(g.rowptr[-1]) for g in graphs], dtype=np.int64)
        self.node_off = np.zeros(self.n_chains + 1, dtype=np.int64)
        np.cumsum(ns, out=self.node_off[1:])
        self.edge_off = np.zeros(self.n_chains + 1, dtype=np.int64)
        np.cumsum(ms, out=self.edge_off[1:])
        self.damping = np.array([g.c for g in graphs], dtype=np.float64)
        self.total_n = int(self.node_off[-1])
        self.total_nnz = int(self.edge_off[-1])
        rp, cl, cp, rw, vv, cv = [], [], [], [], [], []
        for g in graphs:
            colptr, row, perm = g.csc()
            rp.append(np.asarray(g.rowptr, dtype=np.int32))
            cl.append(np.asarray(g.col, dtype=np.int32))
            cp.append(np.asarray(colptr, dtype=np.int32))
            rw.append(np.asarray(row, dtype=np.int32))
            if explicit_val:
                v = g.val(np.float64)
                vv.append(v.astype(vdt))
                cv.append(v[perm].astype(vdt))
        cat = lambda xs, dt: torch.from_numpy(np.ascontiguousarray(np.concatenate(xs), dtype=dt)).to(device)
        self.rowptr = cat(rp, np.int32)
        self.col = cat(cl, np.int32)
        self.colptr = cat(cp, np.int32)
        self.row = cat(rw, np.int32)
        self.val = cat(vv, vdt) if explicit_val else None
        self.cval = cat(cv, vdt) if explicit_val else None

    def struct(self) -> rlgl_batch_graphs:
        return rlgl_batch_graphs(self.n_chains, self.node_off.ctypes.data, self.edge_off.ctypes.data,
                                 self.damping.ctypes.data, _ptr(self.rowptr), _ptr(self.col), _ptr(self.val),
                                 _ptr(self.colptr), _ptr(self.row), _ptr(self.cval),
                                 None if self.tol_l1 is None else self.tol_l1.ctypes.data)


class BatchSolver:
    """One batched context over a DeviceBatch: workspace, output and results."""

    def __init__(self, db: DeviceBatch, stream=None, **options):
        options.setdefault("precision", db.precision)
        self.db = db
        self.graphs = db.struct()
        self.opt = rlgl_batch_default_options(**options)
        self.ws_bytes = rlgl_batch_workspace_bytes(self.graphs, self.opt)
        if self.ws_bytes == 0:
            raise RlglError(RLGL_EINVAL, "rlgl_batch_workspace_bytes")
        dev = db.rowptr.device
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.handle = rlgl_batch_create(self.graphs, self.opt, self.workspace, self.ws_bytes, stream)
        self.pi = torch.empty(db.total_n, dtype=torch.float64, device=dev)

    def solve(self, raise_on_error: bool = True):
        return rlgl_batch_solve(self.handle, self.pi, self.db.n_chains, raise_on_error)

    def autotune(self) -> dict:
        best = rlgl_batch_autotune(self.handle, self.pi)
        return {name: getattr(best, name) for name, _ in best._fields_}

    def chain_pi(self, k: int):
        return self.pi[int(self.db.node_off[k]):int(self.db.node_off[k + 1])]

    def close(self):
        if self.handle is not None:
            rlgl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostChain:
    """A request held in page-locked host memory: CSR row pointers (the
    out-degrees), the CSC and the damping, as ``rlgl_request`` wants them."""

    def __init__(self, g, tol_l1: float = 1e-6):
        import numpy as np
        colptr, row, _ = g.csc()
        self.n, self.nnz, self.c, self.tol_l1, self.name = g.n, g.nnz, float(g.c), float(tol_l1), g.name

        def pinned(a):
            t = torch.empty(len(a), dtype=torch.int32, pin_memory=True)
            t.numpy()[:] = np.asarray(a, dtype=np.int32)
            return t

        self.rowptr = pinned(g.rowptr)
        self.colptr = pinned(colptr)
        self.row = pinned(row) if self.nnz > 0 else None

    def request(self) -> rlgl_request:
        return rlgl_request(self.n, self.nnz, self.rowptr.data_ptr(), self.colptr.data_ptr(),
                            None if self.row is None else self.row.data_ptr(), self.c, self.tol_l1)


class Pool:
    """A serving pool: workspace tensor (control records + arena) and handle."""

    def __init__(self, arena_bytes: int, stream=None, device="cuda", **options):
        self.opt = rlgl_pool_default_options(**options)
        self.ws_bytes = rlgl_pool_workspace_bytes(self.opt, arena_bytes)
        if self.ws_bytes == 0:
            raise RlglError(RLGL_EINVAL, "rlgl_pool_workspace_bytes")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.handle = rlgl_pool_create(self.opt, self.workspace, self.ws_bytes, stream)
        self.requests = {}

    def footprint(self, n: int, nnz: int) -> int:
        return rlgl_pool_footprint(self.opt, n, nnz)

    def admit(self, hc: HostChain):
        """Slot of the admitted chain, or None when no slot or memory is free."""
        req = hc.request()
        slot = rlgl_pool_admit(self.handle, req)
        if slot is not None:
            self.requests[slot] = hc  # keeps the host arrays alive until release
        return slot

    def advance(self, iterations: int = 4) -> int:
        return rlgl_pool_advance(self.handle, iterations)

    def launch(self, iterations: int = 4) -> None:
        rlgl_pool_launch(self.handle, iterations)

    def wait(self) -> int:
        return rlgl_pool_wait(self.handle)

    def poll(self):
        return rlgl_pool_poll(self.handle)

    def result(self, slot: int):
        """(outcome dict, pi_hat as a float64 view into the workspace)."""
        res, ptr = rlgl_pool_result(self.handle, slot)
        n = self.requests[slot].n
        off = ptr - self.workspace.data_ptr()
        pi = self.workspace[off:off + 8 * n].view(torch.float64)
        return res, pi

    def release(self, slot: int) -> None:
        rlgl_pool_release(self.handle, slot)
        self.requests.pop(slot, None)

    def close(self):
        if self.handle is not None:
            rlgl_pool_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
