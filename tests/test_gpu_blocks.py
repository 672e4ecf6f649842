"""rlgl_step_mask through the C ABI: a green set chosen by the caller, step by
step against the oracle's step on the same state, and the optimal block
schedule of Sec. 5.3 run on the GPU on the three-block mean-field SBM."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import l1, oracle_chain, say, to_np
from oracle import blocks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2008_02710_amd as rl  # noqa: E402


def device_graph(P, c, precision):
    """DeviceGraph of a dense transition matrix (stored link values)."""
    n = P.shape[0]
    rows, cols = np.nonzero(P)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))])
    val = P[rows, cols]
    perm = np.lexsort((rows, cols))  # CSC order: by column, then source
    colptr = np.concatenate([[0], np.cumsum(np.bincount(cols, minlength=n))])
    return rl.DeviceGraph(n, rowptr, cols, c, val, colptr, rows[perm], perm, precision)


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H], ids=["fp64", "fp32c"])
@pytest.mark.parametrize("route", [rl.ROUTE_PUSH, rl.ROUTE_PULL], ids=["push", "pull"])
def test_step_mask_matches_oracle(prec, route):
    g = workloads.chung_lu(2500, 2.5, 6.0, 0.1, 0.85, seed=17, name="mask")
    say("case step_mask", prec, route)
    dg = rl.DeviceGraph.from_workload(g, precision=prec, explicit_val=True)
    s = rl.Solver(dg, sched=rl.SCHED_THRESHOLD, route=route, precision=prec)
    ch = oracle_chain(g)
    s.step(2)
    rng = np.random.default_rng(3)
    for k in range(4):
        C, H, info = s.state()
        C, H = to_np(C).astype(np.float64), to_np(H)
        ost = oracle.State.from_arrays(ch, C, H, info["h_sum"], t=info["t"])
        mask = rng.random(g.n) < (0.05, 0.3, 0.7, 1.0)[k]
        moved = float(np.abs(C[mask]).sum())
        info1 = s.step_mask(torch.from_numpy(mask.astype(np.uint8)).cuda())
        ost.step_mask(mask)
        C1, H1, _ = s.state()
        tol = 1e-13 if prec == rl.FP64 else 2e-6
        assert l1(to_np(C1), ost.C) <= tol * moved + 1e-300, (k, int(mask.sum()))
        assert l1(to_np(H1), ost.H) <= 1e-14 * moved + 1e-300
        assert abs(info1["h_sum"] - ost.hsum) <= 1e-14
        assert info1["t"] == info["t"] + 1
    # the schedule is back after the masked steps
    st, res = s.solve((1 - g.c) * 1e-6 if prec != rl.FP64 else (1 - g.c) * 1e-10)
    assert st == rl.RLGL_OK
    s.close()


def test_step_mask_needs_callers_numbering():
    g = workloads.chung_lu(500, 2.5, 6.0, 0.0, 0.85, seed=2, name="mask_rl")
    say("case step_mask_relabel")
    dg = rl.DeviceGraph.from_workload(g)
    s = rl.Solver(dg, relabel=1)
    with pytest.raises(rl.RlglError) as e:
        s.step_mask(torch.ones(g.n, dtype=torch.uint8, device="cuda"))
    assert e.value.status == rl.RLGL_EINVAL
    s.close()


def test_optimal_block_schedule_on_gpu():
    """Sec. 5.3: the schedule computed by dynamic programming on the block
    cash, applied to the 80-state mean-field SBM on the GPU (FP64, undamped):
    each step against the oracle's step, the total cost as the block model
    predicts, far below power iteration's, and pi_hat against the exact pi."""
    (N, p, q) = ((50, 20, 10), 0.1, 0.01)
    eps = 1e-12
    say("case block_schedule")
    pol = blocks.Policy(N, p, q, eps, z1_max=12.0, n1=1200, n2=81)
    P = blocks.dense_chain(N, p, q)
    n = P.shape[0]
    dg = device_graph(P, 1.0, rl.FP64)
    s = rl.Solver(dg, precision=rl.FP64, route=rl.ROUTE_PULL)
    rows, cols = np.nonzero(P)
    ch = oracle.Chain(np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]), cols.astype(np.int32),
                      P[rows, cols], 1.0)
    blk = np.repeat(np.arange(3), N)
    kap = blocks.kappa(N, p, q)
    C, H, info = s.state()
    ost = oracle.State.from_arrays(ch, to_np(C), to_np(H), info["h_sum"], t=info["t"])
    cost, acts = 0.0, []
    # rounding is absolute: what the first steps leave stays while the cash shrinks
    scale = float(np.abs(to_np(C)).sum())
    for _ in range(1000):
        Cg = to_np(s.state()[0])
        if np.abs(Cg).sum() <= eps:
            break
        c = np.array([Cg[blk == j].mean() for j in range(3)])
        a = pol.action(c)
        acts.append(a)
        cost += kap[a]
        mask = np.isin(blk, blocks.ACTIONS[a])
        s.step_mask(torch.from_numpy(mask.astype(np.uint8)).cuda())
        ost.step_mask(mask)
        assert l1(to_np(s.state()[0]), ost.C) <= 1e-13 * scale
    C, H, info = s.state()
    assert np.abs(to_np(C)).sum() <= eps
    # the block model: the same actions reach eps at the same step, and the
    # schedule it derives on its own costs the same to within rounding of
    # the grid lookups
    c0 = np.array([(P.T @ np.full(n, 1.0 / n) - 1.0 / n)[blk == j].mean() for j in range(3)])
    replay = iter(acts)
    rep_cost, rep_steps, _ = blocks.run(c0, lambda c: next(replay), N, p, q, eps, max_steps=len(acts))
    assert rep_steps == len(acts) and rep_cost == cost
    model_cost, _, _ = blocks.run(c0, pol.action, N, p, q, eps)
    pi_cost, pi_steps, _ = blocks.run(c0, lambda c: 6, N, p, q, eps)
    assert abs(cost - model_cost) <= 0.02 * model_cost
    assert cost < pi_cost / 5 and len(acts) < pi_steps and 6 not in acts
    pi = to_np(H) / info["h_sum"]
    exact = oracle.stationary_gth(P)
    assert l1(pi, exact) <= 1e-9
    s.close()
