"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package draws graphs and lays them out; it holds none of the RLGL
method's arithmetic.  The random draws are counter-based (``gen.c``), so a
graph is a pure function of its parameters and seed.

Workloads (the paper's own graphs are public web crawls that are not shipped
here; these synthetic families cover the same range of sizes, densities and
degree skew as its Table 1):

  * ``poisson_uniform``: out-degree Poisson(lam)+1, targets uniform.
  * ``chung_lu``: directed Chung-Lu power law, independent in/out rank
    weights w(rank) ~ (rank+1)^(-1/(gamma-1)), optional forced dangling nodes.
  * ``rmat``: Graph500-style R-MAT with a seeded relabelling.
  * ``batch_chains`` / ``serving_pool``: many Chung-Lu chains of log-uniform size.

Every stored link of node i carries P_ij = 1/outdeg(i) (duplicates add up).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libwlgen.so")

# stream ids of the counter-based generator
S_DEG, S_TGT, S_PERM_OUT, S_PERM_IN, S_DANGLING, S_SRC, S_DST, S_RMAT, S_RELABEL, S_META = range(10)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64, u64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.wl_poisson.argtypes = [i64, f64, i32, u64, u64, vp]
        lib.wl_uniform_int.argtypes = [i64, i64, u64, u64, vp]
        lib.wl_uniform01.argtypes = [i64, u64, u64, vp]
        lib.wl_categorical.argtypes = [i64, vp, i64, u64, u64, vp]
        lib.wl_permutation.argtypes = [i64, u64, u64, vp]
        lib.wl_rmat.argtypes = [i32, i64, f64, f64, f64, u64, u64, vp, vp]
        lib.wl_relabel.argtypes = [i64, vp, vp]
        lib.wl_bucket.argtypes = [i64, i64, vp, vp, vp, vp, vp]
        lib.wl_bucket.restype = i32
        lib.wl_transpose.argtypes = [i64, vp, vp, vp, vp, vp]
        lib.wl_transpose.restype = i32
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


@dataclass
class Graph:
    """Link matrix W in CSR with P_ij = 1/outdeg(i) per stored link, plus the
    damping c of the Google-matrix chain built on it."""
    n: int
    rowptr: np.ndarray  # int64 [n+1]
    col: np.ndarray  # int32 [nnz]
    c: float
    name: str = ""
    params: dict = field(default_factory=dict)
    _csc: tuple | None = None
    weights: np.ndarray | None = None  # explicit W_ij per stored link (float64); None: 1/outdeg(i)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @property
    def outdeg(self) -> np.ndarray:
        return np.diff(self.rowptr)

    @property
    def n_dangling(self) -> int:
        return int((self.outdeg == 0).sum())

    def val(self, dtype=np.float64) -> np.ndarray:
        """W_ij of every stored link: the explicit weights, or 1/outdeg(i),
        computed in float64 then cast."""
        if self.weights is not None:
            return self.weights.astype(dtype)
        deg = self.outdeg
        inv = np.zeros(self.n, dtype=np.float64)
        nz = deg > 0
        inv[nz] = 1.0 / deg[nz]
        return np.repeat(inv, deg).astype(dtype)

    def csc(self):
        """(colptr int64 [n+1], row int32 [nnz], perm int64 [nnz]) with
        row[p] the source of in-link p and perm[p] its CSR position."""
        if self._csc is None:
            colptr = np.empty(self.n + 1, dtype=np.int64)
            row = np.empty(self.nnz, dtype=np.int32)
            perm = np.empty(self.nnz, dtype=np.int64)
            rc = _load().wl_transpose(self.n, _p(self.rowptr), _p(self.col), _p(colptr), _p(row), _p(perm))
            if rc != 0:
                raise RuntimeError(f"transpose failed ({rc})")
            self._csc = (colptr, row, perm)
        return self._csc


def from_edges(n: int, src, dst, c: float, name="", params=None) -> Graph:
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    rowptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(src.shape[0], dtype=np.int32)
    rc = _load().wl_bucket(n, src.shape[0], _p(src), _p(dst), _p(rowptr), _p(col), None)
    if rc != 0:
        raise ValueError(f"edge list out of range ({rc})")
    return Graph(n, rowptr, col, float(c), name, dict(params or {}))


def poisson_uniform(n: int = 10000, lam: float = 8.0, c: float = 0.85, seed: int = 0) -> Graph:
    """Out-degree Poisson(lam)+1 (so no dangling node), targets uniform with
    replacement (self-loops and multi-links kept)."""
    lib = _load()
    deg = np.empty(n, dtype=np.int32)
    lib.wl_poisson(n, lam, 1, seed, S_DEG, _p(deg))
    m = int(deg.sum(dtype=np.int64))
    col = np.empty(m, dtype=np.int32)
    lib.wl_uniform_int(m, n, seed, S_TGT, _p(col))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=rowptr[1:])
    return Graph(n, rowptr, col, float(c), "poisson_uniform",
                 dict(n=n, lam=lam, c=c, seed=seed, generator="poisson_uniform"))


def _rank_cdf(n: int, gamma: float, perm: np.ndarray, zero=None) -> np.ndarray:
    w_rank = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    w = w_rank[perm]
    if zero is not None:
        w[zero] = 0.0
    return np.cumsum(w)


def chung_lu(n: int, gamma: float, mean_deg: float, dangling_frac: float = 0.0, c: float = 0.85, seed: int = 0,
             name: str = "chung_lu") -> Graph:
    """Directed Chung-Lu multigraph with m = round(mean_deg*n) links.  Node v
    has out-weight w(rank_out(v)) and in-weight w(rank_in(v)), the two ranks
    from independent seeded permutations; a seeded choice of
    floor(dangling_frac*n) nodes gets out-weight 0 (they become dangling)."""
    lib = _load()
    m = int(round(mean_deg * n))
    perm_out = np.empty(n, dtype=np.int32)
    perm_in = np.empty(n, dtype=np.int32)
    lib.wl_permutation(n, seed, S_PERM_OUT, _p(perm_out))
    lib.wl_permutation(n, seed, S_PERM_IN, _p(perm_in))
    zero = None
    nd = int(math.floor(dangling_frac * n))
    if nd > 0:
        pd = np.empty(n, dtype=np.int32)
        lib.wl_permutation(n, seed, S_DANGLING, _p(pd))
        zero = pd[:nd]
    cdf_out = _rank_cdf(n, gamma, perm_out, zero)
    cdf_in = _rank_cdf(n, gamma, perm_in)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    lib.wl_categorical(n, _p(cdf_out), m, seed, S_SRC, _p(src))
    lib.wl_categorical(n, _p(cdf_in), m, seed, S_DST, _p(dst))
    return from_edges(n, src, dst, c, name,
                      dict(n=n, gamma=gamma, mean_deg=mean_deg, dangling_frac=dangling_frac, c=c, seed=seed,
                           m=m, generator="chung_lu"))


def rmat(scale: int = 24, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, cq: float = 0.19,
         c: float = 0.85, seed: int = 0) -> Graph:
    """R-MAT with 2^scale nodes and edge_factor*2^scale links, then a seeded
    relabelling of the node ids (Graph500 style, no noise)."""
    lib = _load()
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    lib.wl_rmat(scale, m, a, b, cq, seed, S_RMAT, _p(src), _p(dst))
    perm = np.empty(n, dtype=np.int32)
    lib.wl_permutation(n, seed, S_RELABEL, _p(perm))
    lib.wl_relabel(m, _p(perm), _p(src))
    lib.wl_relabel(m, _p(perm), _p(dst))
    g = from_edges(n, src, dst, c, "rmat",
                   dict(scale=scale, edge_factor=edge_factor, a=a, b=b, c_quadrant=cq, c=c, seed=seed,
                        generator="rmat"))
    del src, dst
    return g


def log_uniform_sizes(count: int, lo: float, hi: float, seed: int, stream: int) -> np.ndarray:
    u = np.empty(count, dtype=np.float64)
    _load().wl_uniform01(count, seed, stream, _p(u))
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def uniform_values(count: int, lo: float, hi: float, seed: int, stream: int) -> np.ndarray:
    u = np.empty(count, dtype=np.float64)
    _load().wl_uniform01(count, seed, stream, _p(u))
    return lo + u * (hi - lo)


def batch_chains(count: int = 512, n_lo: float = 1e3, n_hi: float = 2e5, gamma: float = 2.3,
                 mean_deg: float = 10.0, c_lo: float = 0.8, c_hi: float = 0.95, seed: int = 4,
                 with_csc: bool = False):
    """Independent chains: n log-uniform in [n_lo, n_hi], Chung-Lu with
    exponent gamma and the given mean degree (natural dangling nodes), damping
    uniform in [c_lo, c_hi]."""
    sizes = log_uniform_sizes(count, n_lo, n_hi, seed, S_META)
    cs = uniform_values(count, c_lo, c_hi, seed, S_META + 1)

    def one(k):
        g = chung_lu(int(sizes[k]), gamma, mean_deg, 0.0, float(cs[k]), seed=seed * 100003 + 17 * k + 1,
                     name=f"chain{k}")
        if with_csc:
            g.csc()
        return g

    # the C generators release the GIL: chains are drawn on all host cores
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, range(count)))


def largest_scc(g: Graph, c: float = 1.0, name: str = "") -> Graph:
    """The chain restricted to the largest strongly connected component of
    g's link graph: its states renumbered 0..m-1 in their original order and
    the links among them (multiplicity kept), with damping c (c = 1: the
    undamped stationary distribution).  Every state of a component with more
    than one state keeps at least one out-link, so there is no dangling state."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg
    A = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col, g.rowptr), shape=(g.n, g.n))
    _, lab = cg.connected_components(A, directed=True, connection="strong")
    keep = lab == np.bincount(lab).argmax()
    new = np.full(g.n, -1, dtype=np.int64)
    m = int(keep.sum())
    new[keep] = np.arange(m)
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.outdeg)
    inside = keep[src] & keep[g.col]
    params = dict(g.params, scc_of=g.name, c=c)
    return from_edges(m, new[src[inside]].astype(np.int32), new[g.col[inside]].astype(np.int32), c,
                      name or f"{g.name}_scc", params)


def auxiliary_node_chain(g: Graph, c: float, name: str = "") -> Graph:
    """The (N+1)-state chain P^(0) of Sec. 2.4 on which RLGL is GSo-PR: state 0
    is the auxiliary node (self-loop c, then (1-c)/N to every state), state
    i+1 is g's state i (1-c back to 0, then c/outdeg(i) along each of its
    links).  Needs a graph without dangling states.  Explicit weights; used
    with damping 1 (the chain already carries the restart)."""
    n = g.n
    deg = g.outdeg
    if np.any(deg == 0):
        raise ValueError("the auxiliary-node chain needs a graph without dangling states")
    rowlen = np.concatenate([[n + 1], 1 + deg]).astype(np.int64)
    rowptr = np.zeros(n + 2, dtype=np.int64)
    np.cumsum(rowlen, out=rowptr[1:])
    total = int(rowptr[-1])
    col = np.empty(total, dtype=np.int32)
    w = np.empty(total, dtype=np.float64)
    col[:n + 1] = np.arange(n + 1, dtype=np.int32)
    w[0] = c
    w[1:n + 1] = (1.0 - c) / n
    first = np.zeros(total, dtype=bool)
    first[rowptr[1:n + 1]] = True
    first[:n + 1] = False
    rest = np.zeros(total, dtype=bool)
    rest[n + 1:] = True
    links = rest & ~first
    col[first] = 0
    w[first] = 1.0 - c
    col[links] = g.col + 1
    w[links] = c / np.repeat(deg, deg)
    return Graph(n + 1, rowptr, col, 1.0, name or f"{g.name}_aux", dict(g.params, aux_of=g.name, c_inner=c),
                 weights=w)


def poisson_arrivals(count: int, rate: float, seed: int, stream: int = S_META + 2) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate: cumulative
    exponential gaps -log(1 - u) / rate."""
    u = np.empty(count, dtype=np.float64)
    _load().wl_uniform01(count, seed, stream, _p(u))
    return np.cumsum(-np.log1p(-u) / rate)


def serving_pool(count: int = 128, n_lo: float = 1e3, n_hi: float = 1e6, gamma: float = 2.3, mean_deg: float = 12.0,
                 c: float = 0.85, seed: int = 5):
    """Chains the serving requests draw from: n log-uniform in [n_lo, n_hi],
    Chung-Lu with exponent gamma and the given mean degree (natural dangling
    nodes), damping c, CSC built."""
    sizes = log_uniform_sizes(count, n_lo, n_hi, seed, S_META)

    def one(k):
        g = chung_lu(int(sizes[k]), gamma, mean_deg, 0.0, c, seed=seed * 100003 + 17 * k + 1, name=f"req{k}")
        g.csc()
        return g

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, range(count)))


def request_draws(count: int, pool_size: int, seed: int, stream: int = S_META + 3) -> np.ndarray:
    """Which pool chain each request asks for (uniform, with replacement)."""
    out = np.empty(count, dtype=np.int32)
    _load().wl_uniform_int(count, pool_size, seed, stream, _p(out))
    return out.astype(np.int64)


def random_small(n: int, mean_deg: float, c: float, seed: int, dangling_frac: float = 0.0) -> Graph:
    """Small Chung-Lu test graph (gamma 2.5) used for parity cases."""
    return chung_lu(n, 2.5, mean_deg, dangling_frac, c, seed, name=f"small{n}")
