"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times (threshold r = 1, FP32 cash with FP64 history, link weights
1/outdeg implied by the row pointers, AUTO route, relabelled layout), and
with FP32 link values stored per link:

  * Chung-Lu power law, N = 2^20, 16.8M links, exponent 2.1, 5% dangling;
  * R-MAT scale 24 (16.8M nodes, 268M links, a/b/c = 0.57/0.19/0.19).

Per graph: one green-light step from a device state against the oracle's
step on the very same state (green set bit for bit, C node by node within
the rounding its terms allow, H in L1), for a pull and a push step; and a
full solve whose pi_hat the oracle's FP64 residual certifies to L1 <= 1e-6
(the bound ||pi_hat - pi*||_1 <= ||pi_hat - pi_hat P||_1 / (1 - c), for
pi_hat summing to one).  Also the benchmark's headline configuration (the
all-green schedule in the relabelled layout, R-MAT with stored values) and
the top-k step at k = N/4 on the Chung-Lu graph.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import l1, say, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2008_02710_amd as rl  # noqa: E402

_cache = {}


def graph(name, stored=False):
    key = (name, stored)
    if key not in _cache:
        if name not in _cache:
            say("generating", name)
            if name == "chung_lu_2p20":
                g = workloads.chung_lu(1 << 20, 2.1, 16.0, 0.05, 0.85, seed=0, name=name)
            else:
                g = workloads.rmat(24, 16, 0.57, 0.19, 0.19, 0.85, seed=0)
                g.name = name
            g.csc()
            say("generated", name, g.n, g.nnz, "dangling", g.n_dangling)
            _cache[name] = (g, oracle.Chain(g.rowptr, g.col, g.val(), g.c))
        g, ch = _cache[name]
        dg = rl.DeviceGraph.from_workload(g, precision=rl.FP32C_FP64H, with_csc=True, explicit_val=stored)
        say("uploaded", name, "stored values" if stored else "implied values")
        _cache[key] = (g, dg, ch)
    return _cache[key]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("relabel,stored", [(0, False), (1, False), (1, True)])
@pytest.mark.parametrize("name", ["chung_lu_2p20", "rmat_s24"])
def test_full_size_solve_certified(name, relabel, stored):
    g, dg, ch = graph(name, stored)
    say("case full_solve", name, "relabel" if relabel else "", "stored" if stored else "")
    eps = (1 - g.c) * 1e-6
    s = rl.Solver(dg, sched=rl.SCHED_THRESHOLD, route=rl.ROUTE_AUTO, precision=rl.FP32C_FP64H, relabel=relabel)
    st, info = s.solve(eps, max_steps=100000)
    assert st == rl.RLGL_OK and info["resid"] < eps
    pi = to_np(s.pi)
    s.close()
    say("solved", name, info["t"], "steps")
    assert np.all(pi >= 0.0) and abs(pi.sum() - 1.0) < 1e-9
    cert = oracle.residual(ch, pi) / (1 - g.c)
    say("certified L1 bound", cert)
    assert cert <= 1e-6


@pytest.mark.timeout(900)
@pytest.mark.parametrize("route,relabel,stored", [("pull", 0, False), ("push", 0, False), ("pull", 1, False),
                                                  ("pull", 1, True)])
@pytest.mark.parametrize("name", ["chung_lu_2p20", "rmat_s24"])
def test_full_size_one_step_parity(name, route, relabel, stored):
    g, dg, ch = graph(name, stored)
    say("case full_step", name, route, "relabel" if relabel else "", "stored" if stored else "")
    s = rl.Solver(dg, sched=rl.SCHED_THRESHOLD, route=rl.ROUTE_AUTO, precision=rl.FP32C_FP64H, record_green=1)
    s.step(3)
    C, H, info0 = s.state()
    C, H = to_np(C).astype(np.float64), to_np(H)
    s.close()
    # the same state, one step with the route forced
    s = rl.Solver(dg, sched=rl.SCHED_THRESHOLD, precision=rl.FP32C_FP64H, record_green=1, relabel=relabel,
                  route=rl.ROUTE_PULL if route == "pull" else rl.ROUTE_PUSH)
    s.set_state(torch.from_numpy(C).cuda(), torch.from_numpy(H).cuda(), info0["h_sum"],
                t=info0["t"])
    info1 = s.step(1)
    mask = to_np(s.green()).astype(bool)
    theta = info1["theta"]
    assert theta == pytest.approx(oracle.theta(C), rel=1e-12)
    want = oracle.select(C, oracle.THRESHOLD, theta, 0)
    assert np.array_equal(mask, want), (int(mask.sum()), int(want.sum()))
    ost = oracle.State.from_arrays(ch, C, H, info0["h_sum"], t=info0["t"])
    moved = float(np.abs(C[want]).sum())
    ost.step_mask(want)
    C1, H1, info2 = s.state()
    s.close()
    # one float rounding per stored value and per add: 2e-6 of the moved mass
    assert l1(to_np(C1), ost.C) <= 2e-6 * moved
    check_elementwise(g, ch, C, want, to_np(C1), ost.C, stored)
    assert l1(to_np(H1), ost.H) <= 1e-15 * moved + 1e-300
    assert abs(info2["h_sum"] - ost.hsum) <= 1e-14
    say("step parity", name, route, "green", int(want.sum()), "moved", moved)


def check_elementwise(g, ch, C, want, C1, C1_oracle, stored):
    """Every node within the rounding its own terms allow: R_k bounds the sum
    of |terms| arriving at k (the route of |M| plus |C_k|); FP32 cash rounds
    each term and the result once (1.3e-7 R + 6e-8 |C_k|), FP32 stored link
    values differ from the oracle's FP64 1/outdeg by 6e-8 each, the FP64
    column sums add (in-degree + 4) roundings, and the restart share is summed
    in another order (u sum |M| on every node)."""
    M = np.where(want, C, 0.0)
    R = oracle.route(ch, np.abs(M)) + np.abs(C)
    indeg = np.diff(g.csc()[0]).astype(np.float64)
    pool_err = 2.3e-16 * float(np.abs(M).sum())
    bound = ((1.3e-7 + (6e-8 if stored else 0.0)) * R + 6e-8 * np.abs(C1_oracle)
             + (indeg + 4.0) * 2.3e-16 * R + pool_err)
    err = np.abs(C1 - C1_oracle)
    worst = int(np.argmax(err - bound))
    assert np.all(err <= bound + 1e-300), (worst, err[worst], bound[worst])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,stored", [("rmat_s24", True), ("chung_lu_2p20", False)])
def test_full_size_all_green_solve_certified(name, stored):
    """The benchmark's headline configuration: the all-green schedule in the
    relabelled layout (R-MAT with stored FP32 link values), AUTO route, FP32
    cash with FP64 history; the oracle's FP64 residual of pi_hat certifies
    L1 <= 1e-6, in about as many steps as power iteration takes (22 on both
    graphs to this target: c^t below the target's share)."""
    g, dg, ch = graph(name, stored)
    say("case full_all_green", name, "stored" if stored else "")
    eps = (1 - g.c) * 1e-6
    s = rl.Solver(dg, sched=rl.SCHED_ALL, route=rl.ROUTE_AUTO, precision=rl.FP32C_FP64H, relabel=1)
    st, info = s.solve(eps, max_steps=100000)
    assert st == rl.RLGL_OK and info["resid"] < eps
    pi = to_np(s.pi)
    s.close()
    assert np.all(pi >= 0.0) and abs(pi.sum() - 1.0) < 1e-9
    cert = oracle.residual(ch, pi) / (1 - g.c)
    say("solved", name, info["t"], "steps, certified L1 bound", cert)
    assert cert <= 1e-6
    assert info["t"] <= 30
    # every step routes every link of every node with cash (step 0 included)
    assert info["edges_pushed"] <= info["t"] * g.nnz


@pytest.mark.timeout(900)
def test_full_size_topk_step_parity():
    """The top-k step at the benchmark's size and k (Chung-Lu 2^20, k = N/4,
    the caller's numbering, pull): on a device state after three top-k steps
    the green set is the oracle's bit for bit (|C| descending, then smaller
    id), and the step matches the oracle's element by element."""
    g, dg, ch = graph("chung_lu_2p20", False)
    k = 262144
    say("case full_topk_step", k)
    s = rl.Solver(dg, sched=rl.SCHED_TOPK, k=k, precision=rl.FP32C_FP64H, record_green=1)
    s.step(3)
    C, H, info0 = s.state()
    C, H = to_np(C).astype(np.float64), to_np(H)
    s.close()
    s = rl.Solver(dg, sched=rl.SCHED_TOPK, k=k, precision=rl.FP32C_FP64H, record_green=1, route=rl.ROUTE_PULL)
    s.set_state(torch.from_numpy(C).cuda(), torch.from_numpy(H).cuda(), info0["h_sum"], t=info0["t"])
    info1 = s.step(1)
    mask = to_np(s.green()).astype(bool)
    want = oracle.select(C, oracle.TOPK, 0.0, k)
    assert int(want.sum()) == k
    assert np.array_equal(mask, want), (int(mask.sum()), int((mask != want).sum()))
    assert info1["green"] == k
    ost = oracle.State.from_arrays(ch, C, H, info0["h_sum"], t=info0["t"])
    moved = float(np.abs(C[want]).sum())
    ost.step_mask(want)
    C1, H1, info2 = s.state()
    s.close()
    assert l1(to_np(C1), ost.C) <= 2e-6 * moved
    check_elementwise(g, ch, C, want, to_np(C1), ost.C, False)
    assert l1(to_np(H1), ost.H) <= 1e-15 * moved + 1e-300
    say("topk step parity: green", k, "moved", moved)
