"""Batched solves (the step-synchronous engine over many chains) vs the
oracle and vs the single-chain path, through the C ABI."""
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

PREC_NAMES = {rl.FP64: "fp64", rl.FP32C_FP64H: "fp32c_fp64h", rl.FP32C_KAHANH: "fp32c_kahanh"}


def mixed_chains():
    """Chains of uneven size: tiny, dangling-only, power-law with long
    columns (> 2048 in-links), log-uniform sizes, damping in [0.8, 0.95]."""
    gs = []
    sizes = workloads.log_uniform_sizes(18, 50, 30000, seed=9, stream=1)
    cs = workloads.uniform_values(18, 0.8, 0.95, seed=9, stream=2)
    for k in range(18):
        gs.append(workloads.chung_lu(int(sizes[k]), 2.3, 10.0, 0.0, float(cs[k]), seed=100 + k, name=f"m{k}"))
    gs.append(workloads.chung_lu(20000, 2.1, 16.0, 0.05, 0.85, seed=5, name="hub"))
    gs.append(workloads.from_edges(1, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.9, name="one"))
    gs.append(workloads.from_edges(700, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.85, name="empty"))
    gs.append(workloads.poisson_uniform(3000, 8.0, 0.9, seed=3))
    return gs


_cache = {}


def chains():
    if "g" not in _cache:
        _cache["g"] = mixed_chains()
        assert np.diff(_cache["g"][18].csc()[0]).max() > 2048
    return _cache["g"]


def reference(g):
    key = (g.name, g.n)
    if key not in _cache:
        _cache[key] = oracle.reference_pagerank(oracle_chain(g), 1e-13)[0]
    return _cache[key]


ENGINES = {"lockstep": rl.BATCH_LOCKSTEP}


@pytest.mark.parametrize("engine", list(ENGINES))
@pytest.mark.parametrize("prec", [rl.FP32C_KAHANH, rl.FP32C_FP64H, rl.FP64], ids=PREC_NAMES.get)
@pytest.mark.parametrize("sched", ["threshold", "all"])
def test_batch_matches_oracle(prec, sched, engine):
    gs = chains()
    say("case batch", PREC_NAMES[prec], sched, engine, len(gs), "chains")
    tol = 1e-10 if prec == rl.FP64 else 1e-6
    worst_c = max(g.c for g in gs)
    eps = (1 - worst_c) * tol * 0.5
    db = rl.DeviceBatch(gs, precision=prec)
    bs = rl.BatchSolver(db, sched={"threshold": rl.SCHED_THRESHOLD, "all": rl.SCHED_ALL}[sched], eps=eps,
                        wg_size=256, wg_per_cu=2, max_steps=20000, engine=ENGINES[engine])
    st, res, ms = bs.solve()
    assert st == rl.RLGL_OK
    for k, g in enumerate(gs):
        pi = to_np(bs.chain_pi(k))
        err = l1(pi, reference(g))
        assert res[k]["status"] == rl.RLGL_OK and res[k]["resid"] < eps, (k, res[k])
        assert err <= tol, (k, g.n, err, res[k])
        assert 0.0 <= res[k]["start_us"] <= res[k]["end_us"] <= ms * 1000.0 * 1.01 + 5.0
        if sched == "all" and prec == rl.FP64:
            # all-green is power iteration: the step count is the oracle's
            ost, _, oinfo = oracle.solve(oracle_chain(g), oracle.ALL, eps=eps)
            assert abs(res[k]["t"] - oinfo["t"]) <= 1, (k, res[k]["t"], oinfo["t"])
    bs.close()


@pytest.mark.parametrize("engine", list(ENGINES))
def test_batch_equals_single_chain_path(engine):
    """Each chain's result is the same alone (single-chain solve) and in the
    batch, within the mixed-precision tolerance."""
    gs = chains()
    say("case batch_vs_single", engine)
    eps = 0.05 * 1e-6
    db = rl.DeviceBatch(gs, precision=rl.FP32C_FP64H)
    bs = rl.BatchSolver(db, eps=eps, max_steps=20000, engine=ENGINES[engine])
    st, res, ms = bs.solve()
    assert st == rl.RLGL_OK
    for k, g in enumerate(gs):
        dg = rl.DeviceGraph.from_workload(g, precision=rl.FP32C_FP64H)
        s = rl.Solver(dg, sched=rl.SCHED_THRESHOLD, route=rl.ROUTE_PULL)
        sst, info = s.solve(eps, max_steps=20000)
        assert sst == rl.RLGL_OK
        assert l1(to_np(s.pi), to_np(bs.chain_pi(k))) <= 2e-6, k
        assert abs(info["t"] - res[k]["t"]) <= 3, (k, info["t"], res[k]["t"])
        s.close()
    bs.close()


def test_batch_autotune_and_repeat():
    gs = chains()
    say("case batch_autotune")
    db = rl.DeviceBatch(gs, precision=rl.FP32C_KAHANH)
    bs = rl.BatchSolver(db, eps=1e-7, max_steps=20000)
    best = bs.autotune()
    assert best["wg_size"] in (256, 512) and best["wg_per_cu"] in (0, 4, 8)
    assert best["engine"] == rl.BATCH_LOCKSTEP
    st, res, ms = bs.solve()
    assert st == rl.RLGL_OK
    pa = to_np(bs.pi).copy()
    st, res2, ms2 = bs.solve()
    assert [r["t"] for r in res] == [r["t"] for r in res2]
    assert l1(pa, to_np(bs.pi)) <= 1e-12
    bs.close()


@pytest.mark.parametrize("engine", list(ENGINES))
def test_batch_maxc_small_chains(engine):
    gs = [workloads.chung_lu(n, 2.3, 6.0, 0.0, 0.85, seed=n, name=f"s{n}") for n in (40, 120, 333)]
    say("case batch_maxc", engine)
    db = rl.DeviceBatch(gs, precision=rl.FP64)
    bs = rl.BatchSolver(db, sched=rl.SCHED_MAXC, eps=0.15e-10, wg_size=256, wg_per_cu=0, max_steps=200000,
                        engine=ENGINES[engine])
    st, res, ms = bs.solve()
    assert st == rl.RLGL_OK
    for k, g in enumerate(gs):
        assert l1(to_np(bs.chain_pi(k)), reference(g)) <= 1e-10
    bs.close()


@pytest.mark.parametrize("engine", list(ENGINES))
def test_batch_not_converged_reports_chain_status(engine):
    gs = chains()[:4]
    say("case batch_limit", engine)
    db = rl.DeviceBatch(gs, precision=rl.FP32C_KAHANH)
    bs = rl.BatchSolver(db, eps=1e-30, max_steps=3, engine=ENGINES[engine])
    st, res, ms = bs.solve(raise_on_error=False)
    assert st == rl.RLGL_ENOT_CONVERGED
    assert all(r["status"] == rl.RLGL_ENOT_CONVERGED and r["t"] == 4 for r in res)
    bs.close()


def test_batch_route_shapes_agree_and_tol_l1_certifies():
    """Per-chain L1 targets: each chain stops at ||C||_1/|H.1| < tol (1 - c_k),
    and the FP64 residual of its pi_hat certifies L1 <= tol.  The route
    launched one workgroup per plan item and strided over 8 workgroups per CU
    take the same number of steps up to the rounding order."""
    gs = chains()
    say("case batch_tol_l1")
    tols = [1e-6 if k % 2 else 3e-7 for k in range(len(gs))]
    db = rl.DeviceBatch(gs, precision=rl.FP32C_KAHANH, tol_l1=tols)
    out = {}
    shapes = {"per_item": 0, "strided": 8}
    for name, per_cu in shapes.items():
        bs = rl.BatchSolver(db, engine=rl.BATCH_LOCKSTEP, wg_per_cu=per_cu, max_steps=20000)
        st, res, ms = bs.solve()
        assert st == rl.RLGL_OK
        pis = [to_np(bs.chain_pi(k)).copy() for k in range(len(gs))]
        out[name] = (res, pis)
        bs.close()
    for k, g in enumerate(gs):
        for name in shapes:
            res, pis = out[name]
            cert = oracle.residual(oracle_chain(g), pis[k]) / (1 - g.c)
            assert cert <= tols[k], (name, k, cert)
            assert l1(pis[k], reference(g)) <= tols[k], (name, k)
        ta, tb = out["per_item"][0][k]["t"], out["strided"][0][k]["t"]
        assert abs(ta - tb) <= 2, (k, ta, tb)


def test_batch_rejects_l1_target_without_damping():
    """A per-chain L1 target certifies through 1/(1 - c): a chain with c = 1
    has no such bound (its residual target would be 0), so a batch that
    gives both is rejected before any work; without tol_l1 it runs on the
    residual target of the options."""
    g = workloads.largest_scc(workloads.chung_lu(3000, 2.3, 10.0, 0.0, 1.0, seed=3), c=1.0)
    say("case batch_damping_1", g.n, g.nnz)
    db = rl.DeviceBatch([g], precision=rl.FP32C_KAHANH, tol_l1=[1e-6])
    with pytest.raises(rl.RlglError) as e:
        rl.BatchSolver(db, engine=rl.BATCH_LOCKSTEP)
    assert e.value.status == rl.RLGL_EINVAL
    db = rl.DeviceBatch([g], precision=rl.FP32C_KAHANH)
    bs = rl.BatchSolver(db, engine=rl.BATCH_LOCKSTEP, eps=1e-8, max_steps=20000)
    st, res, _ = bs.solve()
    assert st == rl.RLGL_OK and res[0]["status"] == rl.RLGL_OK
    bs.close()


@pytest.mark.parametrize("sched", ["threshold", "all"])
def test_batch_relabelled_layout_matches_caller_layout(sched):
    """The relabelled layout (states renumbered by decreasing out-degree
    inside the library) gives each chain's pi_hat in the caller's numbering:
    in FP64 the column sums add the same links in the same order, so the two
    layouts agree to rounding in the statistics, and both match the oracle."""
    gs = chains()
    say("case batch_relabel", sched)
    eps = 0.05 * 1e-10
    s = {"threshold": rl.SCHED_THRESHOLD, "all": rl.SCHED_ALL}[sched]
    db = rl.DeviceBatch(gs, precision=rl.FP64)
    out = {}
    for relabel in (0, 1):
        bs = rl.BatchSolver(db, sched=s, eps=eps, max_steps=20000, relabel=relabel)
        st, res, _ = bs.solve()
        assert st == rl.RLGL_OK
        out[relabel] = ([to_np(bs.chain_pi(k)).copy() for k in range(len(gs))], [r["t"] for r in res])
        bs.close()
    for k, g in enumerate(gs):
        assert l1(out[0][0][k], out[1][0][k]) <= 1e-12, k
        assert abs(out[0][1][k] - out[1][1][k]) <= 1, k
        assert l1(out[1][0][k], reference(g)) <= 1e-10, k


def test_batch_relabel_rejects_decreasing_row_pointers():
    """The relabelled layout sorts each chain's states by out-degree from its
    row pointers: a chain whose row pointers decrease is rejected at create
    (RLGL_EINVAL) before any work, and the other chains are not touched."""
    gs = [workloads.chung_lu(n, 2.3, 6.0, 0.0, 0.85, seed=n, name=f"r{n}") for n in (300, 500)]
    say("case batch_relabel_bad_rowptr")
    db = rl.DeviceBatch(gs, precision=rl.FP32C_KAHANH)
    off = int(db.node_off[1]) + 1  # chain 1's row pointers start after chain 0's n + 1
    rp = db.rowptr[off + 10:off + 12].clone()
    db.rowptr[off + 10] = rp[1] + 1  # row pointer 10 of chain 1 above row pointer 11
    with pytest.raises(rl.RlglError) as e:
        rl.BatchSolver(db, relabel=1)
    assert e.value.status == rl.RLGL_EINVAL


@pytest.mark.timeout(600)
def test_full_size_batch_certified():
    """The benchmark's batched configuration: 512 chains (n log-uniform in
    [1e3, 2e5], Chung-Lu exponent 2.3, mean degree 10, damping in
    [0.8, 0.95]), FP32 cash with compensated history, tol_l1 = 1e-6 per chain,
    the all-green schedule in the relabelled layout with the autotuned launch
    shape: every chain stops on its own target, and the oracle's FP64
    residual of its pi_hat certifies L1 <= 1e-6."""
    gs = workloads.batch_chains(512, seed=4, with_csc=True)
    say("case batch_full_size", len(gs), sum(g.n for g in gs), sum(g.nnz for g in gs))
    db = rl.DeviceBatch(gs, precision=rl.FP32C_KAHANH, tol_l1=1e-6)
    bs = rl.BatchSolver(db, sched=rl.SCHED_ALL, max_steps=100000)
    bs.autotune()
    st, res, ms = bs.solve()
    assert st == rl.RLGL_OK
    pi = to_np(bs.pi)
    bs.close()
    worst = 0.0
    for k, g in enumerate(gs):
        assert res[k]["status"] == rl.RLGL_OK and res[k]["resid"] < 1e-6 * (1 - g.c), k
        p = pi[db.node_off[k]:db.node_off[k + 1]]
        assert abs(p.sum() - 1.0) < 1e-9 and np.all(p >= 0.0), k
        worst = max(worst, oracle.residual(oracle_chain(g, explicit_val=False), p) / (1 - g.c))
    say("batch solved in", ms, "ms; worst certified L1", worst)
    assert worst <= 1e-6
