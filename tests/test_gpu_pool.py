"""Serving pool (continuous batching) through the C ABI: every result against
the oracle's FP64 reference, the same chain alone and in a mix of requests
admitted while it runs, admission bounded by the arena, slot reuse."""
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
from paper_2008_02710_amd.serving import serve  # noqa: E402

_cache = {}


def requests():
    if "g" not in _cache:
        sizes = workloads.log_uniform_sizes(10, 500, 40000, seed=21, stream=1)
        gs = [workloads.chung_lu(int(n), 2.3, 12.0, 0.0, 0.85, seed=300 + k, name=f"q{k}")
              for k, n in enumerate(sizes)]
        gs.append(workloads.chung_lu(20000, 2.1, 16.0, 0.05, 0.9, seed=5, name="hub"))
        gs.append(workloads.from_edges(1, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.85, name="one"))
        gs.append(workloads.from_edges(300, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.85, name="empty"))
        assert np.diff(gs[10].csc()[0]).max() > 2048
        _cache["g"] = gs
    return _cache["g"]


def reference(g):
    key = (g.name, g.n)
    if key not in _cache:
        _cache[key] = oracle.reference_pagerank(oracle_chain(g), 1e-13)[0]
    return _cache[key]


def drain(pool, slots):
    """Advances until every slot in `slots` finished; returns {slot: (res, pi copy)}."""
    got = {}
    for _ in range(100000):
        pool.advance(4)
        for s in pool.poll():
            res, pi = pool.result(s)
            got[s] = (res, to_np(pi).copy())
        if all(s in got for s in slots):
            return got
    raise AssertionError("pool did not drain")


@pytest.mark.parametrize("prec", [rl.FP32C_KAHANH, rl.FP64], ids=["fp32c_kahanh", "fp64"])
def test_pool_results_match_oracle(prec):
    gs = requests()
    tol = 1e-6 if prec != rl.FP64 else 1e-10
    say("case pool_oracle", prec, len(gs), "requests")
    pool = rl.Pool(256 << 20, precision=prec, max_chains=32)
    hcs = [rl.HostChain(g, tol_l1=tol) for g in gs]
    slots = [pool.admit(h) for h in hcs]
    assert None not in slots
    got = drain(pool, slots)
    for k, (g, s) in enumerate(zip(gs, slots)):
        res, pi = got[s]
        assert res["status"] == rl.RLGL_OK, (k, res)
        assert res["resid"] < tol * (1 - g.c), (k, res)
        assert l1(pi, reference(g)) <= tol, (k, g.n)
        cert = oracle.residual(oracle_chain(g), pi) / (1 - g.c)
        assert cert <= tol * 1.0001, (k, cert)
        assert 0.0 <= res["start_us"] <= res["end_us"]
        pool.release(s)
    pool.close()


def test_pool_alone_equals_mix():
    """A chain's result is the same when it runs alone and when requests are
    admitted and finish around it (mixed precision, within 2e-6 of each
    other and within 1e-6 of the FP64 reference)."""
    gs = requests()
    target = gs[10]  # the hub chain, long columns included
    say("case pool_alone_vs_mix")
    pool = rl.Pool(256 << 20, max_chains=8)
    h = rl.HostChain(target, tol_l1=1e-6)
    alone = drain(pool, [pool.admit(h)])
    (s0, (res_a, pi_a)), = alone.items()
    pool.release(s0)
    # the mix: three requests first, the target after a few iterations, more
    # requests while it runs
    others = [rl.HostChain(g, tol_l1=1e-6) for g in gs[:10]]
    live = [pool.admit(o) for o in others[:3]]
    pool.advance(3)
    st = pool.admit(h)
    pool.advance(2)
    live += [pool.admit(o) for o in others[3:7]]
    got = drain(pool, [st] + [s for s in live if s is not None])
    res_m, pi_m = got[st]
    assert res_a["status"] == res_m["status"] == rl.RLGL_OK
    assert l1(pi_a, pi_m) <= 2e-6
    ref = reference(target)
    assert l1(pi_a, ref) <= 1e-6 and l1(pi_m, ref) <= 1e-6
    assert abs(res_a["t"] - res_m["t"]) <= 2
    pool.close()


def test_pool_admission_by_footprint_and_slot_reuse():
    gs = requests()[:10]
    say("case pool_admission")
    opt = rl.rlgl_pool_default_options(max_chains=3)
    foot = [rl.rlgl_pool_footprint(opt, g.n, g.nnz) for g in gs]
    arena = int(max(foot) * 1.6)  # the largest chain fits, never two of the largest
    pool = rl.Pool(arena, max_chains=3)
    hcs = [rl.HostChain(g, tol_l1=1e-6) for g in gs]
    arrivals = [0.0] * len(gs)
    seen = {}

    def keep(i, res, pi):
        seen[i] = to_np(pi).copy()

    out = serve(pool, hcs, arrivals, iterations=4, on_result=keep)
    assert all(r is not None and r["status"] == rl.RLGL_OK for r in out)
    for i, g in enumerate(gs):
        assert l1(seen[i], reference(g)) <= 1e-6, i
    # all blocks came back: the whole arena is one free block again
    big = workloads.chung_lu(int(gs[int(np.argmax(foot))].n), 2.3, 12.0, 0.0, 0.85, seed=99)
    slot = pool.admit(rl.HostChain(big))
    assert slot is not None
    with pytest.raises(rl.RlglError) as e:
        pool.release(slot)  # still uploading or running
    assert e.value.status == rl.RLGL_EBUSY
    drain(pool, [slot])
    pool.release(slot)
    pool.close()


def test_pool_rejects_bad_requests():
    say("case pool_bad_requests")
    pool = rl.Pool(16 << 20, max_chains=2)
    g = requests()[0]
    h = rl.HostChain(g)
    req = h.request()
    req.damping = 1.5
    with pytest.raises(rl.RlglError):
        rl.rlgl_pool_admit(pool.handle, req)
    # c = 1: the L1 target tol (1 - c) would be 0, and no certificate exists
    req = h.request()
    req.damping = 1.0
    with pytest.raises(rl.RlglError) as e:
        rl.rlgl_pool_admit(pool.handle, req)
    assert e.value.status == rl.RLGL_EINVAL
    req = h.request()
    req.nnz = g.nnz + 1  # disagrees with rowptr[n]
    with pytest.raises(rl.RlglError):
        rl.rlgl_pool_admit(pool.handle, req)
    # larger than the arena: busy, nothing changed
    big = workloads.chung_lu(400000, 2.3, 12.0, 0.0, 0.85, seed=1)
    assert pool.admit(rl.HostChain(big)) is None
    s = pool.admit(h)
    assert s is not None
    drain(pool, [s])
    pool.release(s)
    pool.close()


def test_pool_reports_step_limit_per_request():
    """A pool whose step limit is too small for the tolerance reports
    RLGL_ENOT_CONVERGED for that request (pi_hat still written) and keeps
    serving the next one."""
    gs = requests()[:2]
    say("case pool_limit")
    pool = rl.Pool(64 << 20, max_chains=2, max_steps=3)
    hcs = [rl.HostChain(g, tol_l1=1e-12) for g in gs]
    slots = [pool.admit(h) for h in hcs]
    got = drain(pool, slots)
    for s in slots:
        res, pi = got[s]
        assert res["status"] == rl.RLGL_ENOT_CONVERGED and res["t"] == 4
        assert abs(pi.sum() - 1.0) < 1e-6
        pool.release(s)
    pool.close()


def test_pool_launch_wait_with_admissions_in_flight():
    """The split advance: requests admitted and results collected while
    iterations are in flight give the same answers; a second launch before
    the wait is refused."""
    gs = requests()[:8]
    say("case pool_launch_wait")
    pool = rl.Pool(128 << 20, max_chains=8)
    hcs = [rl.HostChain(g, tol_l1=1e-6) for g in gs]
    slots = {pool.admit(hcs[0]): 0, pool.admit(hcs[1]): 1}
    pool.launch(4)
    with pytest.raises(rl.RlglError) as e:
        pool.launch(4)
    assert e.value.status == rl.RLGL_EINVAL
    nxt = 2
    got = {}
    for _ in range(100000):
        if nxt < len(hcs):
            s = pool.admit(hcs[nxt])  # while the launch runs
            assert s is not None
            slots[s] = nxt
            nxt += 1
        pool.wait()
        for s in pool.poll():
            res, pi = pool.result(s)
            got[slots[s]] = (res, to_np(pi).copy())
            pool.release(s)
        if len(got) == len(hcs):
            break
        pool.launch(4)
    assert len(got) == len(hcs)
    for k, g in enumerate(gs):
        res, pi = got[k]
        assert res["status"] == rl.RLGL_OK, (k, res)
        assert l1(pi, reference(g)) <= 1e-6, k
    pool.close()
