"""Reference oracle for the Red-Light-Green-Light (RLGL) method.

TEST INFRASTRUCTURE ONLY.  Plain, serial FP64 statements of what the method
computes (Avrachenkov, Brown, Litvak, "Red Light Green Light Method for
Solving Large Markov Chains", arXiv 2008.02710).  Only ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark import this package.  It shares
no code with the HIP library and never imports it.

Contents
  * ctypes wrappers over ``rlgl_oracle.c``: the chain product ``route`` (the
    M_t P of the cash recursion, Sec. 2.1 eq. (6)), green-set selection,
    Algorithm 1 step by step and to its stop test, power iteration (Sec. 2.3.1
    and the PI reference of Sec. 6), and the residual ||pi - pi P||_1.
  * ``dense_P``: the transition matrix written out densely (tiny chains).
  * ``stationary_dense``: pi = pi P, sum(pi) = 1 by a linear solve (Sec. 2.1).
  * ``stationary_gth``: the Grassmann-Taksar-Heyman elimination cited in
    Sec. 1.1, free of subtractions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rlgl_oracle.c")
_LIB = os.path.join(_HERE, "librlgl_oracle.so")

ALL, THRESHOLD, TOPK, MAXC, PC = 0, 1, 2, 3, 4
OK, EINVAL, ENOMEM, EZERO_HISTORY, ENOT_CONVERGED, ENONFINITE = 0, -1, -2, -4, -5, -6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
             "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Chain(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("c", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("steps", ctypes.c_int64), ("green_total", ctypes.c_int64),
                ("edges_pushed", ctypes.c_int64), ("l1_cash", ctypes.c_double), ("h_sum", ctypes.c_double),
                ("resid", ctypes.c_double), ("theta", ctypes.c_double), ("cash_sum", ctypes.c_double),
                ("status", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        pc = ctypes.POINTER(_Chain)
        lib.orc_route.argtypes = [pc, vp, vp]
        lib.orc_route.restype = None
        lib.orc_theta.argtypes = [i32, vp, f64]
        lib.orc_theta.restype = f64
        lib.orc_select.argtypes = [i32, vp, i32, f64, i64, vp]
        lib.orc_select.restype = i64
        lib.orc_init.argtypes = [pc, vp, vp, vp, ctypes.POINTER(f64), ctypes.POINTER(i64)]
        lib.orc_init.restype = None
        lib.orc_step.argtypes = [pc, vp, vp, vp, ctypes.POINTER(f64), ctypes.POINTER(i64), vp]
        lib.orc_step.restype = None
        lib.orc_select_pc.argtypes = [i32, vp, ctypes.c_uint64, i64, vp]
        lib.orc_select_pc.restype = i64
        lib.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_splitmix64.restype = ctypes.c_uint64
        lib.orc_solve.argtypes = [pc, vp, i32, f64, i64, i32, f64, i64, ctypes.c_uint64, vp, vp, vp,
                                  ctypes.POINTER(Info)]
        lib.orc_solve.restype = i32
        lib.orc_power_iteration.argtypes = [pc, f64, i64, vp, ctypes.POINTER(i64)]
        lib.orc_power_iteration.restype = i32
        lib.orc_power_iteration_omp.argtypes = [pc, f64, i64, vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
        lib.orc_power_iteration_omp.restype = i32
        lib.orc_gso_pr.argtypes = [pc, vp, f64, i64, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        lib.orc_gso_pr.restype = i32
        lib.orc_residual.argtypes = [pc, vp]
        lib.orc_residual.restype = f64
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Chain:
    """A chain P = c W + (1-c)/N 1 1^T with dangling rows uniform (see module doc).

    ``rowptr``/``col``/``val`` is the CSR of W; ``val`` None means 1/outdeg.
    Arrays are converted to the oracle's own types (int64 rowptr, int32 col,
    float64 val) and kept alive by this object.
    """

    def __init__(self, rowptr, col, val=None, c: float = 1.0):
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = None if val is None else np.ascontiguousarray(val, dtype=np.float64)
        self.n = int(self.rowptr.shape[0] - 1)
        self.c = float(c)
        if self.val is not None and self.val.shape[0] != self.col.shape[0]:
            raise ValueError("val and col differ in length")
        self._s = _Chain(self.n, _ptr(self.rowptr), _ptr(self.col), _ptr(self.val), self.c)

    @property
    def outdeg(self):
        return np.diff(self.rowptr)

    def ref(self):
        return ctypes.byref(self._s)


def route(ch: Chain, M) -> np.ndarray:
    """Return M P (the routed cash of eq. (6))."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    out = np.zeros(ch.n, dtype=np.float64)
    _load().orc_route(ch.ref(), _ptr(M), _ptr(out))
    return out


def theta(C, r: float = 1.0) -> float:
    C = np.ascontiguousarray(C, dtype=np.float64)
    return float(_load().orc_theta(C.shape[0], _ptr(C), float(r)))


def splitmix64(seed: int, index: int) -> int:
    """Output number `index` of splitmix64 started at `seed`."""
    return int(_load().orc_splitmix64(seed & (2 ** 64 - 1), index & (2 ** 64 - 1)))


def select(C, sched: int, theta_value: float = 0.0, k: int = 1, seed: int = 0, t: int = 0) -> np.ndarray:
    """Green mask (bool array) chosen from the cash snapshot C (of step t for
    PC, whose draws also use the seed)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    mask = np.zeros(C.shape[0], dtype=np.uint8)
    if sched == PC:
        g = _load().orc_select_pc(C.shape[0], _ptr(C), seed & (2 ** 64 - 1), int(t), _ptr(mask))
        return mask.astype(bool)
    g = _load().orc_select(C.shape[0], _ptr(C), int(sched), float(theta_value), int(k), _ptr(mask))
    if g < 0:
        raise ValueError("bad selection arguments")
    return mask.astype(bool)


class State:
    """RLGL state (C_t, H_t, H_t 1) advanced step by step (Algorithm 1)."""

    def __init__(self, ch: Chain, M0=None):
        self.ch = ch
        self.C = np.zeros(ch.n, dtype=np.float64)
        self.H = np.zeros(ch.n, dtype=np.float64)
        self._M = np.zeros(ch.n, dtype=np.float64)
        hs = ctypes.c_double(0.0)
        ed = ctypes.c_int64(0)
        m0 = None if M0 is None else np.ascontiguousarray(M0, dtype=np.float64)
        _load().orc_init(ch.ref(), _ptr(m0), _ptr(self.C), _ptr(self.H), ctypes.byref(hs), ctypes.byref(ed))
        self.hsum = hs.value
        self.edges = ed.value
        self.t = 1

    @classmethod
    def from_arrays(cls, ch: Chain, C, H, hsum: float, t: int = 2, edges: int = 0):
        s = cls.__new__(cls)
        s.ch = ch
        s.C = np.array(C, dtype=np.float64)
        s.H = np.array(H, dtype=np.float64)
        s._M = np.zeros(ch.n, dtype=np.float64)
        s.hsum = float(hsum)
        s.edges = int(edges)
        s.t = int(t)
        return s

    def step_mask(self, mask):
        mask = np.ascontiguousarray(np.asarray(mask, dtype=bool).astype(np.uint8))
        hs = ctypes.c_double(self.hsum)
        ed = ctypes.c_int64(self.edges)
        _load().orc_step(self.ch.ref(), _ptr(mask), _ptr(self.C), _ptr(self.H), ctypes.byref(hs),
                         ctypes.byref(ed), _ptr(self._M))
        self.hsum = hs.value
        self.edges = ed.value
        self.t += 1

    def step(self, sched: int, r: float = 1.0, k: int = 1, theta_value=None, seed: int = 0):
        th = theta(self.C, r) if (sched == THRESHOLD and theta_value is None) else (theta_value or 0.0)
        mask = select(self.C, sched, th, k, seed=seed, t=self.t)
        self.step_mask(mask)
        return mask, th

    @property
    def l1(self):
        return float(np.abs(self.C).sum())

    @property
    def resid(self):
        return self.l1 / abs(self.hsum)

    @property
    def pi_hat(self):
        return self.H / self.hsum


def solve(ch: Chain, sched: int = ALL, eps: float = 1e-10, max_steps: int = 10 ** 7, r: float = 1.0, k: int = 1,
          theta_period: int = 1, M0=None, want_state: bool = False, seed: int = 0):
    """Algorithm 1 to its stop test.  Returns (status, pi_hat, info dict[, C, H])."""
    pi = np.zeros(ch.n, dtype=np.float64)
    C = np.zeros(ch.n, dtype=np.float64) if want_state else None
    H = np.zeros(ch.n, dtype=np.float64) if want_state else None
    info = Info()
    m0 = None if M0 is None else np.ascontiguousarray(M0, dtype=np.float64)
    st = _load().orc_solve(ch.ref(), _ptr(m0), int(sched), float(r), int(k), int(theta_period), float(eps),
                           int(max_steps), seed & (2 ** 64 - 1), _ptr(pi), _ptr(C), _ptr(H), ctypes.byref(info))
    if want_state:
        return st, pi, info.as_dict(), C, H
    return st, pi, info.as_dict()


def power_iteration(ch: Chain, tol: float, max_iter: int = 100000):
    """x_{k+1} = x_k P from the uniform vector until ||x_{k+1}-x_k||_1 <= tol."""
    x = np.zeros(ch.n, dtype=np.float64)
    it = ctypes.c_int64(0)
    st = _load().orc_power_iteration(ch.ref(), float(tol), int(max_iter), _ptr(x), ctypes.byref(it))
    return st, x, it.value


def power_iteration_omp(ch: Chain, tol: float, max_iter: int = 100000):
    """The power iteration on every host core (OpenMP), a CPU baseline:
    (status, x, iterations, threads)."""
    x = np.zeros(ch.n, dtype=np.float64)
    it = ctypes.c_int64(0)
    th = ctypes.c_int32(0)
    st = _load().orc_power_iteration_omp(ch.ref(), float(tol), int(max_iter), _ptr(x), ctypes.byref(it),
                                         ctypes.byref(th))
    return st, x, it.value, th.value


def gso_pr(ch: Chain, eps: float, max_steps: int = 10 ** 8, s=None):
    """Algorithm 2 (GSo-PR): (status, H, C, steps, edges); pi_hat = H."""
    H = np.zeros(ch.n, dtype=np.float64)
    C = np.zeros(ch.n, dtype=np.float64)
    sv = None if s is None else np.ascontiguousarray(s, dtype=np.float64)
    steps = ctypes.c_int64(0)
    edges = ctypes.c_int64(0)
    st = _load().orc_gso_pr(ch.ref(), _ptr(sv), float(eps), int(max_steps), _ptr(H), _ptr(C), ctypes.byref(steps),
                            ctypes.byref(edges))
    return st, H, C, steps.value, edges.value


def reference_pagerank(ch: Chain, l1_target: float = 1e-13, max_iter: int = 100000):
    """FP64 power iteration stopped at ||x_{k+1}-x_k||_1 <= l1_target (1-c).

    For c < 1 the Dobrushin coefficient of P is at most c (Sec. 3.2), so the
    last iterate is within l1_target of pi* in L1.
    """
    if ch.c >= 1.0:
        raise ValueError("the error certificate needs c < 1")
    st, x, it = power_iteration(ch, l1_target * (1.0 - ch.c), max_iter)
    if st != OK:
        raise RuntimeError(f"power iteration did not converge (status {st})")
    return x, it


def residual(ch: Chain, pi) -> float:
    """||pi - pi P||_1 in FP64."""
    pi = np.ascontiguousarray(pi, dtype=np.float64)
    return float(_load().orc_residual(ch.ref(), _ptr(pi)))


def dense_P(ch: Chain) -> np.ndarray:
    """The transition matrix as a dense array (tiny chains only)."""
    n = ch.n
    W = np.zeros((n, n), dtype=np.float64)
    deg = ch.outdeg
    for i in range(n):
        for e in range(ch.rowptr[i], ch.rowptr[i + 1]):
            W[i, ch.col[e]] += (ch.val[e] if ch.val is not None else 1.0 / deg[i])
    P = ch.c * W + (1.0 - ch.c) / n
    P[deg == 0, :] = 1.0 / n
    return P


def stationary_dense(P: np.ndarray) -> np.ndarray:
    """Solve pi (I - P) = 0 with sum(pi) = 1: the last equation is replaced by
    the normalisation, and the system is solved by LU (numpy.linalg.solve)."""
    n = P.shape[0]
    A = (np.eye(n) - P).T.copy()
    A[-1, :] = 1.0
    b = np.zeros(n)
    b[-1] = 1.0
    return np.linalg.solve(A, b)


def stationary_gth(P: np.ndarray) -> np.ndarray:
    """Grassmann-Taksar-Heyman: censor states n-1, ..., 1 one at a time, then
    rebuild pi by forward substitution.  Only additions, multiplications and
    divisions of non-negative numbers are used."""
    A = np.array(P, dtype=np.float64)
    n = A.shape[0]
    for m in range(n - 1, 0, -1):
        s = A[m, :m].sum()
        A[:m, m] /= s
        A[:m, :m] += np.outer(A[:m, m], A[m, :m])
    x = np.zeros(n)
    x[0] = 1.0
    for j in range(1, n):
        x[j] = x[:j] @ A[:j, j]
    return x / x.sum()
