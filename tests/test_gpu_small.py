"""One-workgroup solves (rlgl_solve_small) against the oracle.

* RLGL_MaxC in FP64 routes the maximisers' cash in the order of the serial
  method, so the trajectory is the oracle's own: the same number of steps,
  the same links used and pi_hat equal bit for bit.
* The column route (ALL, THRESHOLD, PC) sums every column in the serial
  order except the restart pool: ALL takes exactly the oracle's steps and
  every rule reaches L1 <= 1e-10 (FP64) or 1e-6 (FP32 cash) against the FP64
  power-iteration reference.
* Edges: N = 1, no links, the capacity limit and one past it, bad arguments,
  max_steps = 0 and a step limit, Example 1's chain and the two-wheels chain
  (c = 1).
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import l1, oracle_chain, say, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2008_02710_amd as rl  # noqa: E402

PREC_NAMES = {rl.FP64: "fp64", rl.FP32C_FP64H: "fp32c_fp64h"}


def small(g, prec, explicit_val=True, **opts):
    dg = rl.DeviceGraph.from_workload(g, precision=prec, with_csc=True, explicit_val=explicit_val)
    return rl.SmallSolver(dg, **opts)


_cache = {}


def poisson(n):
    if n not in _cache:
        _cache[n] = workloads.poisson_uniform(n, 8.0, 0.85, seed=0)
    return _cache[n]


def reference(g):
    key = ("ref", g.name, g.n, g.nnz)
    if key not in _cache:
        _cache[key] = oracle.reference_pagerank(oracle_chain(g), 1e-13)[0]
    return _cache[key]


@pytest.mark.parametrize("n", [3000, 10000])
@pytest.mark.parametrize("explicit", [True, False], ids=["stored", "implied"])
def test_maxc_fp64_is_the_serial_trajectory(n, explicit):
    g = poisson(n)
    eps = 1e-10 * (1 - g.c)
    say("case maxc_serial", n, explicit)
    s = small(g, rl.FP64, explicit_val=explicit, sched=rl.SCHED_MAXC)
    st, info = s.solve(eps, max_steps=2_000_000)
    assert st == rl.RLGL_OK
    ost, opi, oinfo = oracle.solve(oracle_chain(g), oracle.MAXC, eps=eps)
    assert ost == oracle.OK
    assert info["t"] == oinfo["t"]
    assert info["edges_pushed"] == oinfo["edges_pushed"]
    assert info["green_total"] == oinfo["green_total"]
    pi = to_np(s.pi)
    assert np.array_equal(pi, opi), float(np.abs(pi - opi).max())
    assert l1(pi, reference(g)) <= 1e-10
    assert info["last_route"] == rl.ROUTE_PUSH


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H], ids=PREC_NAMES.get)
def test_all_green_steps_and_accuracy(prec):
    g = poisson(10000)
    eps = 1e-10 * (1 - g.c) if prec == rl.FP64 else 1e-6 * (1 - g.c)
    say("case all", PREC_NAMES[prec])
    s = small(g, prec, sched=rl.SCHED_ALL)
    st, info = s.solve(eps, max_steps=2000)
    assert st == rl.RLGL_OK
    ost, opi, oinfo = oracle.solve(oracle_chain(g), oracle.ALL, eps=eps)
    if prec == rl.FP64:
        assert info["t"] == oinfo["t"]
        assert info["edges_pushed"] == oinfo["edges_pushed"]
        assert l1(to_np(s.pi), opi) <= 1e-14
    else:
        assert abs(info["t"] - oinfo["t"]) <= 2
    assert l1(to_np(s.pi), reference(g)) <= (1e-10 if prec == rl.FP64 else 1e-6)


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H], ids=PREC_NAMES.get)
@pytest.mark.parametrize("sched", ["threshold", "threshold_r2", "pc"])
def test_column_rules_reach_the_reference(prec, sched):
    g = workloads.chung_lu(4000, 2.3, 8.0, 0.1, 0.85, seed=21, name="cl4000")
    tol = 1e-10 if prec == rl.FP64 else 1e-6
    eps = tol * (1 - g.c)
    say("case column", PREC_NAMES[prec], sched)
    if sched == "pc":
        opts = dict(sched=rl.SCHED_PC, seed=77)
    elif sched == "threshold_r2":
        opts = dict(sched=rl.SCHED_THRESHOLD, r=2.0, theta_period=2)
    else:
        opts = dict(sched=rl.SCHED_THRESHOLD)
    s = small(g, prec, **opts)
    st, info = s.solve(eps, max_steps=20000)
    assert st == rl.RLGL_OK
    ref = reference(g)
    assert l1(to_np(s.pi), ref) <= tol
    if sched == "threshold" and prec == rl.FP64:
        ost, _, oinfo = oracle.solve(oracle_chain(g), oracle.THRESHOLD, eps=eps)
        assert abs(info["t"] - oinfo["t"]) <= 2
    # the certified bound of the returned vector
    assert oracle.residual(oracle_chain(g), to_np(s.pi)) / (1 - g.c) <= tol * 1.0000001


def test_maxc_fp32_list_route():
    g = poisson(3000)
    say("case maxc_fp32")
    s = small(g, rl.FP32C_FP64H, sched=rl.SCHED_MAXC)
    st, info = s.solve(1e-6 * (1 - g.c), max_steps=1_000_000)
    assert st == rl.RLGL_OK
    assert l1(to_np(s.pi), reference(g)) <= 1e-6


def test_degenerate_and_closed_forms():
    for prec in (rl.FP64, rl.FP32C_FP64H):
        for n in (1, 5, 1500):
            say("case empty", n, PREC_NAMES[prec])
            g = workloads.from_edges(n, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.85)
            for sched in (rl.SCHED_ALL, rl.SCHED_THRESHOLD, rl.SCHED_MAXC):
                s = small(g, prec, sched=sched)
                st, info = s.solve(1e-12, max_steps=1000)
                assert st == rl.RLGL_OK
                assert np.abs(to_np(s.pi) - 1.0 / n).max() <= 1e-7
    # two-wheels, c = 1: pi = deg / 42
    say("case two_wheels")
    edges = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "two_wheels_edges.txt"),
                       dtype=np.int64) - 1
    g = workloads.from_edges(12, np.r_[edges[:, 0], edges[:, 1]], np.r_[edges[:, 1], edges[:, 0]], 1.0)
    for sched in (rl.SCHED_ALL, rl.SCHED_THRESHOLD, rl.SCHED_MAXC):
        s = small(g, rl.FP64, sched=sched)
        st, info = s.solve(1e-13, max_steps=100000)
        assert st == rl.RLGL_OK
        assert l1(to_np(s.pi), g.outdeg / 42.0) <= 1e-11


def test_capacity_and_errors():
    cap64 = rl.rlgl_small_max_n(rl.FP64)
    cap32 = rl.rlgl_small_max_n(rl.FP32C_FP64H)
    say("case capacity", cap64, cap32)
    assert cap64 >= 10000 and cap32 >= 2 * cap64 - 64
    g = workloads.poisson_uniform(cap64, 8.0, 0.85, seed=9)
    s = small(g, rl.FP64, sched=rl.SCHED_ALL)
    st, info = s.solve(1e-9 * (1 - g.c), max_steps=2000)
    assert st == rl.RLGL_OK
    assert l1(to_np(s.pi), reference(g)) <= 1e-9
    g1 = workloads.poisson_uniform(cap64 + 1, 8.0, 0.85, seed=9)
    s1 = small(g1, rl.FP64, sched=rl.SCHED_ALL)
    st, info = s1.solve(1e-9, raise_on_error=False)
    assert st == rl.RLGL_EINVAL and "capacity" in rl.rlgl_last_error()
    # top-k is not a rule of this solver; a short workspace; a missing CSC
    g = poisson(3000)
    s = small(g, rl.FP64, sched=rl.SCHED_TOPK, k=3)
    st, _ = s.solve(1e-9, raise_on_error=False)
    assert st == rl.RLGL_EINVAL
    s = small(g, rl.FP64, sched=rl.SCHED_ALL)
    st, _ = rl.rlgl_solve_small(s.graph, s.opt, 1e-9, 100, s.pi, s.workspace, s.ws_bytes - 512,
                                raise_on_error=False)
    assert st == rl.RLGL_ENOMEM
    gs = s.dg.struct()
    gs.csc_colptr = None
    st, _ = rl.rlgl_solve_small(gs, s.opt, 1e-9, 100, s.pi, s.workspace, s.ws_bytes, raise_on_error=False)
    assert st == rl.RLGL_EINVAL
    # max_steps = 0: not converged, pi_hat = H_1 / (H_1 1) = uniform still written
    st, info = rl.rlgl_solve_small(s.graph, s.opt, 1e-9, 0, s.pi, s.workspace, s.ws_bytes, raise_on_error=False)
    assert st == rl.RLGL_ENOT_CONVERGED and info.t == 1
    assert np.abs(to_np(s.pi) - 1.0 / g.n).max() <= 1e-15


def test_example1_and_step_limit():
    """Example 1's chain (c = 1) from the uniform M_0: MaxC stops at t = 5 as
    the serial method does, on pi* = (2/7, 1/7, 2/7, 2/7) (its zero-history
    case needs an imported state, which a one-launch solve does not take);
    then the step limit."""
    P = workloads.from_edges(4, [0, 0, 1, 2, 3], [1, 2, 2, 3, 0], 1.0)
    say("case example1")
    ref = np.array([2, 1, 2, 2]) / 7.0
    for sched, osched in ((rl.SCHED_MAXC, oracle.MAXC), (rl.SCHED_ALL, oracle.ALL),
                          (rl.SCHED_THRESHOLD, oracle.THRESHOLD)):
        s = small(P, rl.FP64, sched=sched)
        st, info = s.solve(1e-12, max_steps=100000)
        assert st == rl.RLGL_OK
        _, _, oinfo = oracle.solve(oracle_chain(P), osched, eps=1e-12)
        assert info["t"] == oinfo["t"]
        assert l1(to_np(s.pi), ref) <= 1e-11
    g = poisson(3000)
    s = small(g, rl.FP64, sched=rl.SCHED_MAXC)
    st, info = s.solve(1e-30, max_steps=50, raise_on_error=False)
    assert st == rl.RLGL_ENOT_CONVERGED and info["t"] == 51
    assert abs(to_np(s.pi).sum() - 1.0) < 1e-12
