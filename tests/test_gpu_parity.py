"""Parity of the HIP path (through the C ABI) with the reference oracle.

Tolerances:
  * FP64 cash: single steps agree to 1e-14 of the moved mass; solves reach
    L1 <= 1e-10 against the FP64 power-iteration reference.
  * FP32 cash (FP64 or compensated history): single steps agree to 2e-6 of
    the moved mass (one float rounding per stored link plus one per atomic
    add, at most ~2^-23 relative each); solves reach L1 <= 1e-6.
  * The green set is compared bit for bit: the oracle selects on the very
    cash vector the device holds, with the threshold the device reports.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import l1, oracle_chain, say, solver, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2008_02710_amd as rl  # noqa: E402

PRECS = [rl.FP64, rl.FP32C_FP64H, rl.FP32C_KAHANH]
PREC_NAMES = {rl.FP64: "fp64", rl.FP32C_FP64H: "fp32c_fp64h", rl.FP32C_KAHANH: "fp32c_kahanh"}
SCHEDS = {"all": rl.SCHED_ALL, "threshold": rl.SCHED_THRESHOLD, "topk": rl.SCHED_TOPK, "maxc": rl.SCHED_MAXC,
          "pc": rl.SCHED_PC}
ORC_SCHED = {rl.SCHED_ALL: oracle.ALL, rl.SCHED_THRESHOLD: oracle.THRESHOLD, rl.SCHED_TOPK: oracle.TOPK,
             rl.SCHED_MAXC: oracle.MAXC, rl.SCHED_PC: oracle.PC}
PC_SEED = 0x5EED5EED1234
ROUTES = {"push": rl.ROUTE_PUSH, "pull": rl.ROUTE_PULL, "auto": rl.ROUTE_AUTO}


def tol_step(prec):
    return 1e-14 if prec == rl.FP64 else 2e-6


def tol_solve(prec):
    return 1e-10 if prec == rl.FP64 else 1e-6


_cache = {}


def small_graph():
    # 3 tiles of 1024 nodes with a ragged tail, 10% dangling, duplicates and self-loops
    if "small" not in _cache:
        _cache["small"] = workloads.chung_lu(2500, 2.5, 6.0, 0.1, 0.85, seed=3, name="small")
    return _cache["small"]


def hub_graph():
    # power-law exponent 2.1: out- and in-hubs with more than 4096 links
    if "hub" not in _cache:
        g = workloads.chung_lu(20000, 2.1, 16.0, 0.05, 0.85, seed=5, name="hub")
        assert g.outdeg.max() > 4096 and np.diff(g.csc()[0]).max() > 4096
        _cache["hub"] = g
    return _cache["hub"]


def reference(g):
    key = ("ref", g.name, g.n)
    if key not in _cache:
        _cache[key] = oracle.reference_pagerank(oracle_chain(g), 1e-13)[0]
    return _cache[key]


# ------------------------------------------------------------------- step 0

@pytest.mark.parametrize("prec", PRECS, ids=PREC_NAMES.get)
@pytest.mark.parametrize("route", ["push", "pull"])
def test_step0_matches_oracle(prec, route):
    g = small_graph()
    say("case step0", PREC_NAMES[prec], route)
    s = solver(g, prec, route=ROUTES[route], sched=rl.SCHED_ALL)
    C, H, info = s.state()
    st = oracle.State(oracle_chain(g))
    assert info["t"] == 1
    assert l1(to_np(C), st.C) <= tol_step(prec)
    assert l1(to_np(H), st.H) <= (1e-15 if prec == rl.FP64 else 1e-6)
    # M_0 = (1/N) 1 rounded to the cash type
    assert abs(info["h_sum"] - 1.0) <= (1e-12 if prec == rl.FP64 else 1e-7)
    assert info["edges_pushed"] == st.edges == int(g.outdeg[g.outdeg > 0].sum())
    s.close()


# ------------------------------------------------------------ one step

def _nontrivial_state(g, prec, steps=3):
    st = oracle.State(oracle_chain(g))
    for _ in range(steps):
        st.step(oracle.ALL)
    C = st.C.copy()
    if prec != rl.FP64:
        C = C.astype(np.float32).astype(np.float64)
    return C, st.H.copy(), st.hsum


@pytest.mark.parametrize("prec", PRECS, ids=PREC_NAMES.get)
@pytest.mark.parametrize("route", ["push", "pull", "auto"])
@pytest.mark.parametrize("sched", ["all", "threshold", "topk", "maxc", "pc"])
@pytest.mark.parametrize("which", ["small", "hub"])
def test_single_step_parity(prec, route, sched, which):
    _step_parity(prec, route, sched, which, relabel=0)


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_KAHANH], ids=PREC_NAMES.get)
@pytest.mark.parametrize("route", ["push", "pull"])
@pytest.mark.parametrize("sched", ["all", "threshold", "maxc"])
@pytest.mark.parametrize("which", ["small", "hub"])
def test_relabel_single_step_parity(prec, route, sched, which):
    """The relabelled layout: state in and out, the green mask and the step
    itself, all in the caller's numbering, against the oracle."""
    _step_parity(prec, route, sched, which, relabel=1)


def _step_parity(prec, route, sched, which, relabel):
    g = small_graph() if which == "small" else hub_graph()
    say("case single_step", which, PREC_NAMES[prec], route, sched, "relabel" if relabel else "")
    k = 97
    s = solver(g, prec, route=ROUTES[route], sched=SCHEDS[sched], k=k, record_green=1, relabel=relabel,
               seed=PC_SEED)
    C0, H0, hs0 = _nontrivial_state(g, prec)
    s.set_state(torch.from_numpy(C0).cuda(), torch.from_numpy(H0).cuda(), hs0, t=4)
    Cg, Hg, info0 = s.state()
    Cg, Hg = to_np(Cg), to_np(Hg)
    assert np.array_equal(Cg, C0)  # the state is representable in the cash type
    assert l1(Hg, H0) <= (0.0 if prec != rl.FP32C_KAHANH else 1e-13)
    assert info0["h_sum"] == hs0 and info0["t"] == 4
    info1 = s.step(1)
    mask = to_np(s.green()).astype(bool)
    theta = info1["theta"]
    osch = ORC_SCHED[SCHEDS[sched]]
    if osch == oracle.THRESHOLD:
        assert theta == pytest.approx(oracle.theta(Cg), rel=1e-12)
    want = oracle.select(Cg, osch, theta, k, seed=PC_SEED, t=4)
    assert np.array_equal(mask, want), (int(mask.sum()), int(want.sum()))
    assert info1["green"] == int(want.sum())
    ost = oracle.State.from_arrays(oracle_chain(g), Cg, Hg, info0["h_sum"], t=4)
    moved = float(np.abs(Cg[want]).sum())
    ost.step_mask(want)
    C1, H1, info2 = s.state()
    assert info2["t"] == 5
    assert l1(to_np(C1), ost.C) <= tol_step(prec) * moved + 1e-300
    # element by element: every node within the rounding its own terms allow
    # (R_k bounds the sum of |terms| arriving at k: route of |M|)
    M = np.where(want, Cg, 0.0)
    R = oracle.route(oracle_chain(g), np.abs(M)) + np.abs(Cg)
    indeg = np.diff(g.csc()[0]).astype(np.float64)
    # the restart share T/N is summed over all green nodes in another order:
    # its error is at most u sum |M| (N terms, divided by N) on every node
    pool_err = 2.3e-16 * float(np.abs(M).sum())
    if prec == rl.FP64:
        bound = (indeg + 4.0) * 2.3e-16 * R + pool_err
    else:
        bound = 1.3e-7 * R + 6e-8 * np.abs(ost.C) + (indeg + 4.0) * 2.3e-16 * R + pool_err
    err = np.abs(to_np(C1) - ost.C)
    worst = int(np.argmax(err - bound))
    assert np.all(err <= bound + 1e-300), (worst, err[worst], bound[worst])
    assert l1(to_np(H1), ost.H) <= (1e-15 * moved if prec == rl.FP64 else 1e-13 + 1e-7 * moved)
    assert abs(info2["h_sum"] - ost.hsum) <= 1e-14
    assert info2["l1_cash"] == pytest.approx(float(np.abs(to_np(C1)).sum()), rel=1e-12, abs=1e-300)
    s.close()


# ------------------------------------------------------------- refresh

@pytest.mark.parametrize("prec", PRECS, ids=PREC_NAMES.get)
@pytest.mark.parametrize("relabel", [0, 1])
@pytest.mark.parametrize("which", ["small", "hub"])
def test_refresh_matches_oracle(prec, relabel, which):
    """rlgl_refresh rebuilds C_t = H_t P - H_t (eq. (7) with C_0 = 0): against
    the oracle's route(H) - H in FP64, element by element, with long columns
    (the hub graph has columns of more than 4096 in-links) and in the
    relabelled layout; H itself is left unchanged."""
    g = small_graph() if which == "small" else hub_graph()
    say("case refresh", which, PREC_NAMES[prec], relabel)
    s = solver(g, prec, sched=rl.SCHED_THRESHOLD, relabel=relabel)
    s.step(6)
    _, H, info = s.state()
    H = to_np(H)
    s.refresh()
    C2, H2, info2 = s.state()
    C2, H2 = to_np(C2), to_np(H2)
    assert np.array_equal(H2, H) and info2["t"] == info["t"]
    ch = oracle_chain(g)
    want = oracle.route(ch, H) - H
    R = oracle.route(ch, np.abs(H)) + np.abs(H)
    indeg = np.diff(g.csc()[0]).astype(np.float64)
    # the restart share is summed over all nodes in another order: at most
    # u sum |H| on every node
    bound = (indeg + 4.0) * 2.3e-16 * R + 2.3e-16 * float(np.abs(H).sum())
    if prec != rl.FP64:
        # FP32 link values (relative 2^-24 each) and one rounding of the result
        bound = bound + 1.3e-7 * R + 6e-8 * np.abs(want)
    err = np.abs(C2 - want)
    worst = int(np.argmax(err - bound))
    assert np.all(err <= bound + 1e-300), (worst, err[worst], bound[worst])
    # the statistics the step records now describe the rebuilt cash
    assert info2["l1_cash"] == pytest.approx(float(np.abs(C2).sum()), rel=1e-12)
    s.close()


# --------------------------------------------------------------- solves

@pytest.mark.parametrize("prec", PRECS, ids=PREC_NAMES.get)
@pytest.mark.parametrize("sched", ["all", "threshold", "topk", "maxc", "pc"])
def test_solve_small(prec, sched):
    g = small_graph()
    say("case solve_small", PREC_NAMES[prec], sched)
    tol = tol_solve(prec)
    eps = (1 - g.c) * tol * 0.5
    s = solver(g, prec, sched=SCHEDS[sched], k=50, seed=PC_SEED)
    st, info = s.solve(eps)
    assert st == rl.RLGL_OK and info["resid"] < eps and info["t"] >= 2
    pi = to_np(s.pi)
    x = reference(g)
    assert l1(pi, x) <= tol, info
    assert abs(pi.sum() - 1.0) <= 1e-12
    ost, opi, oinfo = oracle.solve(oracle_chain(g), ORC_SCHED[SCHEDS[sched]], eps=eps, k=50, seed=PC_SEED)
    assert ost == oracle.OK
    if prec == rl.FP64 and sched in ("all", "pc"):
        assert abs(info["t"] - oinfo["t"]) <= 1
    else:
        assert info["t"] <= 2 * oinfo["t"] + 5
    s.close()


@pytest.mark.parametrize("route", ["push", "pull"])
def test_all_green_trajectory_is_power_iteration(route):
    """G_t = [N]: H_t = M_0 P^(t-1) and H_t 1 = 1, step by step (FP64)."""
    g = small_graph()
    say("case all_green_trajectory", route)
    s = solver(g, rl.FP64, sched=rl.SCHED_ALL, route=ROUTES[route])
    ost = oracle.State(oracle_chain(g))
    for t in range(1, 30):
        C, H, info = s.state()
        assert info["t"] == t
        # summation order differs (CSC gather or atomics vs the oracle's CSR
        # scatter): ~sqrt(in-degree) ulps on the hub nodes per step
        assert l1(to_np(H), ost.H) <= 2e-14 * t
        assert abs(info["h_sum"] - 1.0) <= 1e-13
        s.step(1)
        ost.step(oracle.ALL)
    s.close()


@pytest.mark.parametrize("route", ["push", "pull", "auto"])
@pytest.mark.parametrize("prec", [rl.FP32C_FP64H, rl.FP32C_KAHANH], ids=PREC_NAMES.get)
def test_solve_hub_graph(route, prec):
    g = hub_graph()
    say("case solve_hub", route, PREC_NAMES[prec])
    s = solver(g, prec, sched=rl.SCHED_THRESHOLD, route=ROUTES[route])
    st, info = s.solve((1 - g.c) * 0.5e-6)
    assert st == rl.RLGL_OK
    assert l1(to_np(s.pi), reference(g)) <= 1e-6
    s.close()


def test_implicit_values_match_explicit():
    g = hub_graph()
    say("case implicit_values")
    a = solver(g, rl.FP32C_FP64H, explicit_val=False, route=rl.ROUTE_AUTO)
    st, info = a.solve((1 - g.c) * 0.5e-6)
    assert st == rl.RLGL_OK
    assert l1(to_np(a.pi), reference(g)) <= 1e-6
    a.close()


def test_reset_repeats_the_solve():
    g = small_graph()
    say("case reset")
    s = solver(g, rl.FP64, sched=rl.SCHED_THRESHOLD, route=rl.ROUTE_PULL)
    st, a = s.solve(1e-12)
    pa = to_np(s.pi).copy()
    s.reset()
    st, b = s.solve(1e-12)
    assert a["t"] == b["t"] and a["edges_pushed"] == b["edges_pushed"]
    assert l1(pa, to_np(s.pi)) <= 1e-13
    s.close()


def test_push_and_pull_agree():
    g = hub_graph()
    say("case push_pull_agree")
    out = []
    for route in (rl.ROUTE_PUSH, rl.ROUTE_PULL):
        s = solver(g, rl.FP64, sched=rl.SCHED_ALL, route=route)
        s.step(12)
        C, H, info = s.state()
        out.append((to_np(C), to_np(H)))
        s.close()
    assert l1(out[0][0], out[1][0]) <= 1e-13
    assert l1(out[0][1], out[1][1]) <= 2e-13


# ---------------------------------------------------------- edge cases

def test_error_zero_history():
    """Example 1: C_1 = (-1, .5, .5, 0), H_1 = (1, 0, 0, 0); MaxC greens node 1
    and the history vanishes."""
    P = workloads.from_edges(4, [0, 0, 1, 2, 3], [1, 2, 2, 3, 0], 1.0)
    say("case zero_history")
    s = solver(P, rl.FP64, sched=rl.SCHED_MAXC)
    s.set_state(torch.tensor([-1.0, .5, .5, 0.0], dtype=torch.float64).cuda(),
                torch.tensor([1.0, 0, 0, 0], dtype=torch.float64).cuda(), 1.0, t=1)
    st, info = s.solve(1e-12, raise_on_error=False)
    assert st == rl.RLGL_EZERO_HISTORY and info["t"] == 2
    s.close()


def test_error_not_converged_and_nonfinite():
    g = small_graph()
    say("case not_converged")
    s = solver(g, rl.FP32C_FP64H, sched=rl.SCHED_THRESHOLD)
    st, info = s.solve(1e-30, max_steps=5, raise_on_error=False)
    assert st == rl.RLGL_ENOT_CONVERGED and info["t"] == 6
    assert abs(to_np(s.pi).sum() - 1.0) < 1e-9  # pi is still written
    say("case nonfinite")
    C = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    C[7] = float("nan")
    H = torch.full((g.n,), 1.0 / g.n, dtype=torch.float64, device="cuda")
    s.set_state(C, H, 1.0, t=3)
    st, info = s.solve(1e-9, raise_on_error=False)
    assert st == rl.RLGL_ENONFINITE
    s.close()


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H], ids=PREC_NAMES.get)
def test_degenerate_graphs(prec):
    say("case degenerate", PREC_NAMES[prec])
    # a single dangling node; an empty link set (every row dangling: uniform pi)
    for n in (1, 5, 1500):
        g = workloads.from_edges(n, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.85)
        s = solver(g, prec, sched=rl.SCHED_THRESHOLD)
        st, info = s.solve(1e-12)
        assert st == rl.RLGL_OK
        assert np.abs(to_np(s.pi) - 1.0 / n).max() <= 1e-7
        s.close()
    # two nodes pointing at each other, c = 1 (periodic chain, but the
    # all-green step lands exactly on pi* from the uniform start)
    g = workloads.from_edges(2, [0, 1], [1, 0], 1.0)
    s = solver(g, prec, sched=rl.SCHED_ALL)
    st, info = s.solve(1e-12)
    assert st == rl.RLGL_OK and np.allclose(to_np(s.pi), 0.5)
    s.close()


def test_two_wheels_closed_form():
    """Two-wheels graph, c = 1: pi = deg / 42."""
    import os
    say("case two_wheels")
    edges = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "two_wheels_edges.txt"),
                       dtype=np.int64) - 1
    g = workloads.from_edges(12, np.r_[edges[:, 0], edges[:, 1]], np.r_[edges[:, 1], edges[:, 0]], 1.0)
    ref = g.outdeg / 42.0
    for sched in (rl.SCHED_ALL, rl.SCHED_THRESHOLD, rl.SCHED_MAXC, rl.SCHED_TOPK):
        s = solver(g, rl.FP64, sched=sched, k=3)
        st, info = s.solve(1e-13)
        assert st == rl.RLGL_OK
        assert l1(to_np(s.pi), ref) <= 1e-11
        s.close()


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H], ids=PREC_NAMES.get)
@pytest.mark.parametrize("which", ["small", "hub"])
def test_relabel_solve_matches_plain(prec, which):
    """Relabelled and plain layouts: the same chain, the same stop, pi_hat
    in the caller's numbering within the precision's tolerance of each other
    and of the FP64 reference."""
    g = small_graph() if which == "small" else hub_graph()
    say("case relabel_solve", which, PREC_NAMES[prec])
    tol = tol_solve(prec)
    eps = (1 - g.c) * tol * 0.5
    out = []
    for relabel in (0, 1):
        s = solver(g, prec, sched=rl.SCHED_THRESHOLD, relabel=relabel)
        st, info = s.solve(eps)
        assert st == rl.RLGL_OK
        out.append((info, to_np(s.pi).copy()))
        s.close()
    (ia, pa), (ib, pb) = out
    assert abs(ia["t"] - ib["t"]) <= 1
    assert l1(pa, pb) <= 2 * tol
    assert l1(pb, reference(g)) <= tol
    assert abs(ia["edges_pushed"] - ib["edges_pushed"]) <= 0.01 * ia["edges_pushed"]


def scc_graph():
    # the largest strongly connected component of a power-law graph, c = 1
    if "scc" not in _cache:
        base = workloads.chung_lu(20000, 2.3, 8.0, 0.0, 1.0, seed=7, name="cl20k")
        _cache["scc"] = workloads.largest_scc(base, c=1.0)
    return _cache["scc"]


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H, rl.FP32C_KAHANH], ids=PREC_NAMES.get)
@pytest.mark.parametrize("relabel", [0, 1])
def test_undamped_largest_scc(prec, relabel):
    """c = 1 on the largest strongly connected component (18,012 states): no
    restart, so the residual no longer bounds the error by 1/(1-c); pi_hat is
    compared with FP64 power iteration run to ||x_{k+1} - x_k||_1 <= 1e-15,
    and the FP64 step count with the oracle's RLGL solve."""
    g = scc_graph()
    say("case undamped_scc", PREC_NAMES[prec], "relabel" if relabel else "", g.n, g.nnz)
    ch = oracle_chain(g)
    key = ("scc_ref",)
    if key not in _cache:
        st, x, it = oracle.power_iteration(ch, 1e-15, 100000)
        assert st == oracle.OK
        _cache[key] = x
    ref = _cache[key]
    eps, tol = (1e-11, 1e-10) if prec == rl.FP64 else (1e-7, 1e-6)
    s = solver(g, prec, sched=rl.SCHED_THRESHOLD, relabel=relabel)
    st, info = s.solve(eps)
    assert st == rl.RLGL_OK and info["resid"] < eps
    pi = to_np(s.pi)
    s.close()
    assert l1(pi, ref) <= tol
    if prec == rl.FP64:
        ost, _, oinfo = oracle.solve(ch, oracle.THRESHOLD, eps=eps)
        assert abs(info["t"] - oinfo["t"]) <= 2, (info["t"], oinfo["t"])


@pytest.mark.parametrize("route", ["push", "pull"])
def test_pc_trajectory_matches_oracle(route):
    """RLGL_PC in FP64: the device and the oracle draw the same green sets
    from the same seed, so their trajectories agree step by step."""
    g = small_graph()
    say("case pc_trajectory", route)
    s = solver(g, rl.FP64, sched=rl.SCHED_PC, route=ROUTES[route], seed=PC_SEED, record_green=1)
    st = oracle.State(oracle_chain(g))
    for t in range(1, 16):
        info = s.step(1)
        want, _ = st.step(oracle.PC, seed=PC_SEED)
        assert np.array_equal(to_np(s.green()).astype(bool), want), t
        C, H, _ = s.state()
        assert l1(to_np(C), st.C) <= 1e-13 * max(1.0, float(np.abs(st.C).sum())), t
        assert l1(to_np(H), st.H) <= 1e-13, t
    s.close()


@pytest.mark.parametrize("route", ["push", "pull"])
@pytest.mark.parametrize("r,period", [(2.0, 1), (1.0, 3), (2.0, 4)])
def test_threshold_order_and_stale_theta(route, r, period):
    """RLGL_Theta with r = 2 and with theta refreshed every `period` steps
    (Sec. 6 allows a threshold updated less often): each step's threshold is
    the oracle's power mean of the device's own cash when it is refreshed and
    the previous one otherwise, the green set matches bit for bit, and the FP64
    trajectory follows the oracle's."""
    g = small_graph()
    say("case threshold_variants", route, r, period)
    s = solver(g, rl.FP64, sched=rl.SCHED_THRESHOLD, r=r, theta_period=period, route=ROUTES[route], record_green=1)
    st = oracle.State(oracle_chain(g))
    th = None
    for t in range(1, 25):
        C, H, info0 = s.state()
        assert info0["t"] == t
        Cd = to_np(C).astype(np.float64)
        info = s.step(1)
        if (t - 1) % period == 0:
            assert info["theta"] == pytest.approx(oracle.theta(Cd, r), rel=1e-12), t
        else:
            assert info["theta"] == th, t
        th = info["theta"]
        want = oracle.select(Cd, oracle.THRESHOLD, th)
        assert np.array_equal(to_np(s.green()).astype(bool), want), t
        st.step_mask(want)
        C1, H1, _ = s.state()
        assert l1(to_np(C1), st.C) <= 1e-12, t
        assert l1(to_np(H1), st.H) <= 1e-12, t
    s.close()


@pytest.mark.parametrize("prec", [rl.FP32C_FP64H, rl.FP32C_KAHANH], ids=PREC_NAMES.get)
def test_threshold_order_two_solve(prec):
    g = hub_graph()
    say("case threshold_r2_solve", PREC_NAMES[prec])
    eps = (1 - g.c) * 0.5e-6
    s = solver(g, prec, sched=rl.SCHED_THRESHOLD, r=2.0, theta_period=2)
    st, info = s.solve(eps)
    assert st == rl.RLGL_OK
    assert l1(to_np(s.pi), reference(g)) <= 1e-6
    s.close()


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H], ids=PREC_NAMES.get)
@pytest.mark.parametrize("route", ["push", "pull", "auto"])
def test_auxiliary_node_chain_gives_pagerank(prec, route):
    """RLGL on the auxiliary-node chain P^(0) of Sec. 2.4 (damping 1, explicit
    weights; state 0 has N+1 out-links and N in-links, the hub paths of both
    routes) started from M_0 = e_0: pi^(0) = (1/2, pi*/2), with pi* the
    PageRank of the original chain."""
    c = 0.85
    base = workloads.poisson_uniform(6000, 8.0, c, seed=11)
    aux = workloads.auxiliary_node_chain(base, c)
    say("case aux_chain", PREC_NAMES[prec], route, aux.n, aux.nnz)
    ref = oracle.reference_pagerank(oracle_chain(base), 1e-13)[0]
    s = solver(aux, prec, sched=rl.SCHED_THRESHOLD, route=ROUTES[route])
    C1 = np.concatenate([[-(1 - c)], np.full(base.n, (1 - c) / base.n)])
    H1 = np.zeros(aux.n)
    H1[0] = 1.0
    s.set_state(torch.from_numpy(C1).cuda(), torch.from_numpy(H1).cuda(), 1.0, t=1)
    tol = 1e-10 if prec == rl.FP64 else 1e-6
    st, info = s.solve(tol * 0.05)
    assert st == rl.RLGL_OK
    pi = to_np(s.pi)
    s.close()
    assert abs(pi[0] - 0.5) <= tol
    assert l1(2.0 * pi[1:], ref) <= 2 * tol


@pytest.mark.parametrize("prec", PRECS, ids=PREC_NAMES.get)
@pytest.mark.parametrize("k", [1, 37, 600, 1249, 2500])
def test_topk_with_heavy_ties(prec, k):
    """Top-k on a cash vector of a few distinct magnitudes (zero included), k
    cutting through a tie group: the device's green set is the oracle's (|C|
    descending, then smaller id) bit for bit, for every precision."""
    g = small_graph()
    say("case topk_ties", PREC_NAMES[prec], k)
    rng = np.random.default_rng(k)
    levels = np.array([0.0, 0.00048828125, 0.0009765625, 0.001953125])  # exact in FP32
    C0 = levels[rng.integers(0, 4, g.n)] * rng.choice([-1.0, 1.0], g.n)
    H0 = np.full(g.n, 1.0 / g.n)
    s = solver(g, prec, sched=rl.SCHED_TOPK, k=k, record_green=1, route=rl.ROUTE_PULL)
    s.set_state(torch.from_numpy(C0).cuda(), torch.from_numpy(H0).cuda(), float(H0.sum()), t=4)
    s.step(1)
    mask = to_np(s.green()).astype(bool)
    want = oracle.select(C0, oracle.TOPK, 0.0, k)
    assert int(mask.sum()) == min(k, g.n)
    assert np.array_equal(mask, want)
    s.close()



_topk_big = {}


@pytest.mark.parametrize("prec", PRECS, ids=PREC_NAMES.get)
@pytest.mark.parametrize("case,k", [("levels", 1), ("levels", 777), ("levels", 150001), ("levels", 299999),
                                    ("low", 1000), ("low", 123457), ("equal", 1), ("equal", 200000),
                                    ("distinct", 50000), ("distinct", 400000)])
def test_topk_many_segments(prec, case, k):
    """Top-k on 300,000 nodes (256 candidate segments of 1,280 nodes): a few
    magnitudes (ties across many segments), keys that differ only in their
    last 9 bits, all magnitudes equal, all distinct, and k above N.  The
    green set is the oracle's bit for bit."""
    if "g" not in _topk_big:
        _topk_big["g"] = workloads.poisson_uniform(300000, 4.0, 0.85, seed=3)
    g = _topk_big["g"]
    say("case topk_segments", PREC_NAMES[prec], case, k)
    rng = np.random.default_rng(k)
    sign = rng.choice([-1.0, 1.0], g.n)
    if case == "levels":
        mag = np.array([0.0, 2.0 ** -12, 2.0 ** -11, 2.0 ** -10, 2.0 ** -9])[rng.integers(0, 5, g.n)]
    elif case == "low":
        mag = 1.0 + rng.integers(0, 512, g.n) * 2.0 ** -23  # the same top 22 key bits
    elif case == "equal":
        mag = np.full(g.n, 2.0 ** -18)
    else:
        mag = rng.integers(1, 2 ** 23, g.n) * 2.0 ** -40  # exact in FP32
    C0 = sign * mag
    H0 = np.full(g.n, 1.0 / g.n)
    s = solver(g, prec, sched=rl.SCHED_TOPK, k=k, record_green=1, route=rl.ROUTE_PULL)
    s.set_state(torch.from_numpy(C0).cuda(), torch.from_numpy(H0).cuda(), float(H0.sum()), t=4)
    s.step(1)
    mask = to_np(s.green()).astype(bool)
    s.close()
    want = oracle.select(C0, oracle.TOPK, 0.0, k)
    assert int(mask.sum()) == min(k, g.n)
    assert np.array_equal(mask, want)

# ------------------------------------------------------- pull plan edges

def _boundary_graph():
    """Columns whose in-degrees sit on the pull plan's limits (512 links per
    item, 64 columns per item): exactly 511, 512 and 513 in-links, 1024 and
    1025, runs of empty columns at item starts and ends, 64 and 65 one-link
    columns in a row, a column fed only by dangling-free sources."""
    rng = np.random.default_rng(123)
    n = 3000
    indeg = np.zeros(n, dtype=np.int64)
    spec = [0, 0, 512, 0, 513, 511, 0, 1, 1024, 1025, 0, 0, 0, 512, 512, 2, 0]
    indeg[:len(spec)] = spec
    pos = len(spec)
    indeg[pos:pos + 64] = 1
    pos += 64 + 3
    indeg[pos:pos + 65] = 1
    pos += 65
    indeg[pos:pos + 200] = 8
    pos += 200
    indeg[pos:] = rng.integers(0, 12, n - pos)
    dst = np.repeat(np.arange(n), indeg)
    src = rng.integers(0, n, dst.size)
    return workloads.from_edges(n, src, dst, 0.85, name="plan_edges")


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H], ids=PREC_NAMES.get)
@pytest.mark.parametrize("relabel", [0, 1])
def test_pull_plan_boundaries(prec, relabel):
    g = _boundary_graph()
    cp = g.csc()[0]
    deg = np.diff(cp)
    assert {511, 512, 513, 1024, 1025} <= set(deg.tolist())
    say("case plan_edges", PREC_NAMES[prec], relabel)
    s = solver(g, prec, route=rl.ROUTE_PULL, sched=rl.SCHED_ALL, record_green=1, relabel=relabel)
    C0, H0, hs0 = _nontrivial_state(g, prec)
    s.set_state(torch.from_numpy(C0).cuda(), torch.from_numpy(H0).cuda(), hs0, t=4)
    Cg, Hg, info0 = s.state()
    Cg, Hg = to_np(Cg), to_np(Hg)
    s.step(1)
    ost = oracle.State.from_arrays(oracle_chain(g), Cg, Hg, info0["h_sum"], t=4)
    moved = float(np.abs(Cg).sum())
    ost.step_mask(np.ones(g.n, dtype=bool))
    C1, H1, info2 = s.state()
    err = np.abs(to_np(C1) - ost.C)
    assert err.sum() <= tol_step(prec) * moved + 1e-300, np.argsort(err)[-5:]
    st, info = s.solve((1 - g.c) * tol_solve(prec) * 0.5)
    assert st == rl.RLGL_OK
    assert l1(to_np(s.pi), reference(g)) <= tol_solve(prec)
    s.close()


def _many_piece_graph():
    """Long columns cut into many pull pieces: 20000, 5000 and 1537 in-links
    (40, 10 and 4 pieces, the last one a single link), beside ordinary ones."""
    rng = np.random.default_rng(7)
    n = 25000
    indeg = rng.integers(0, 10, n)
    indeg[0], indeg[1], indeg[7] = 20000, 5000, 1537
    dst = np.repeat(np.arange(n), indeg)
    src = rng.integers(0, n, dst.size)
    return workloads.from_edges(n, src, dst, 0.85, name="many_pieces")


@pytest.mark.parametrize("prec", [rl.FP64, rl.FP32C_FP64H], ids=PREC_NAMES.get)
@pytest.mark.parametrize("relabel", [0, 1])
def test_long_columns_many_pieces(prec, relabel):
    """The column a piece completes is written in the same pass: every step
    of several in a row against the oracle (a count or sum left over from one
    pass would show in the next)."""
    g = _many_piece_graph()
    deg = np.diff(g.csc()[0])
    assert deg.max() == 20000 and (deg > 512).sum() >= 3
    say("case many_pieces", PREC_NAMES[prec], relabel)
    s = solver(g, prec, route=rl.ROUTE_PULL, sched=rl.SCHED_ALL, record_green=1, relabel=relabel)
    C0, H0, hs0 = _nontrivial_state(g, prec)
    s.set_state(torch.from_numpy(C0).cuda(), torch.from_numpy(H0).cuda(), hs0, t=4)
    for _ in range(4):
        Cg, Hg, info0 = s.state()
        Cg, Hg = to_np(Cg), to_np(Hg)
        ost = oracle.State.from_arrays(oracle_chain(g), Cg, Hg, info0["h_sum"], t=info0["t"])
        moved = float(np.abs(Cg).sum())
        s.step(1)
        ost.step_mask(np.ones(g.n, dtype=bool))
        C1, _, _ = s.state()
        err = np.abs(to_np(C1) - ost.C)
        assert err.sum() <= tol_step(prec) * moved + 1e-300, np.argsort(err)[-5:]
        assert err[[0, 1, 7]].max() <= tol_step(prec) * moved
    s.close()
