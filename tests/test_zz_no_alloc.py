"""rlgl_solve_small_static (the library's static device workspace, no
allocation) against rlgl_solve_small (the caller's workspace): the same
kernel on the same inputs gives the same result bit for bit, on two calls in
a row, the second on a smaller chain, so that nothing the first call left in
the shared array reaches the second.  Sizes beyond the static array are
rejected."""
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


def _pair(g, prec, eps, max_steps, **opts):
    dg = rl.DeviceGraph.from_workload(g, precision=prec, with_csc=True, explicit_val=True)
    ref = rl.SmallSolver(dg, **opts)
    st_ref, info_ref = ref.solve(eps, max_steps)
    pi_static = torch.full((g.n,), float("nan"), dtype=torch.float64, device="cuda")
    st, info = rl.rlgl_solve_small_static(ref.graph, ref.opt, eps, max_steps, pi_static)
    return (st_ref, info_ref, to_np(ref.pi)), (st, info.as_dict(), to_np(pi_static))


@pytest.mark.parametrize("order", ["large_then_small", "small_then_large"])
def test_static_workspace_matches_caller_workspace(order):
    big = workloads.poisson_uniform(10000, 8.0, 0.85, seed=0)
    little = workloads.chung_lu(2500, 2.5, 6.0, 0.1, 0.85, seed=3, name="small")
    cases = [(big, rl.FP64, rl.SCHED_MAXC, 1e-10 * 0.15, 2_000_000),
             (little, rl.FP32C_FP64H, rl.SCHED_THRESHOLD, 1e-6 * 0.15, 20000)]
    if order == "small_then_large":
        cases = cases[::-1]
    for g, prec, sched, eps, max_steps in cases:
        say("case static", order, g.n, prec, sched)
        (st0, i0, pi0), (st1, i1, pi1) = _pair(g, prec, eps, max_steps, sched=sched)
        assert st0 == rl.RLGL_OK and st1 == rl.RLGL_OK
        for key in ("t", "green_total", "edges_pushed", "l1_cash", "h_sum", "status", "last_route"):
            assert i0[key] == i1[key], key
        assert np.array_equal(pi0, pi1)
        ref, _ = oracle.reference_pagerank(oracle_chain(g), 1e-13)
        assert l1(pi1, ref) <= (1e-10 if prec == rl.FP64 else 1e-6)


def test_static_workspace_limits():
    # the largest n the static array holds
    n_max = 0
    while rl.rlgl_small_workspace_bytes(n_max + 1) <= rl.RLGL_SMALL_STATIC_BYTES:
        n_max += 1024
    while rl.rlgl_small_workspace_bytes(n_max) > rl.RLGL_SMALL_STATIC_BYTES:
        n_max -= 1
    cap32 = rl.rlgl_small_max_n(rl.FP32C_FP64H)
    say("case static_limits", n_max, cap32)
    assert n_max < cap32  # FP32 chains between the two are taken only with a caller workspace
    for n, ok in ((n_max, True), (n_max + 1, False)):
        g = workloads.poisson_uniform(n, 8.0, 0.85, seed=4)
        dg = rl.DeviceGraph.from_workload(g, precision=rl.FP32C_FP64H, with_csc=True, explicit_val=False)
        opt = rl.rlgl_default_options(sched=rl.SCHED_ALL, precision=rl.FP32C_FP64H)
        pi = torch.empty(n, dtype=torch.float64, device="cuda")
        st, info = rl.rlgl_solve_small_static(dg.struct(), opt, 1e-6 * 0.15, 2000, pi, raise_on_error=False)
        if ok:
            assert st == rl.RLGL_OK
            assert abs(to_np(pi).sum() - 1.0) < 1e-9
        else:
            assert st == rl.RLGL_EINVAL and "static" in rl.rlgl_last_error()
