"""rlgl_validate through the C ABI: graphs that keep the contract pass (with
the measured row-sum deviation), and each kind of broken array is reported
with its own message.  The broken arrays go to rlgl_validate only, whose
reads are bounds-checked; no solver ever sees them."""
import numpy as np
import pytest

import workloads
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2008_02710_amd as rl  # noqa: E402


def graph():
    return workloads.chung_lu(5000, 2.3, 8.0, 0.1, 0.85, seed=41, name="v")


def device(g, prec=rl.FP32C_FP64H, stored=True):
    return rl.DeviceGraph.from_workload(g, precision=prec, with_csc=True, explicit_val=stored)


@pytest.mark.parametrize("prec,stored", [(rl.FP32C_FP64H, True), (rl.FP32C_FP64H, False), (rl.FP64, True)])
def test_valid_graphs_pass(prec, stored):
    say("case validate_ok", prec, stored)
    g = graph()
    assert g.n_dangling > 0
    dev = device(g, prec, stored).validate()
    if not stored:
        assert dev == 0.0
    else:
        assert 0.0 <= dev <= (1e-12 if prec == rl.FP64 else 1e-6)


def expect(dg, words, status=rl.RLGL_EINVAL):
    with pytest.raises(rl.RlglError) as e:
        dg.validate()
    assert e.value.status == status
    assert words in str(e.value), str(e.value)


def test_row_sum_off():
    say("case validate_rowsum")
    g = graph()
    dg = device(g)
    row = int(np.argmax(np.diff(g.rowptr)))
    a, b = int(g.rowptr[row]), int(g.rowptr[row + 1])
    dg.val[a:b] *= 1.5
    expect(dg, "does not sum to 1")


def test_negative_value():
    say("case validate_negative")
    g = graph()
    dg = device(g)
    dg.val[7] = -dg.val[7]
    expect(dg, "csr_val entry is negative")


def test_column_out_of_range():
    say("case validate_col")
    g = graph()
    dg = device(g, stored=False)
    dg.col[11] = g.n
    expect(dg, "csr_col entry is outside")


def test_rowptr_decreasing():
    say("case validate_rowptr")
    g = graph()
    dg = device(g, stored=False)
    deg = np.diff(g.rowptr)
    i = int(np.flatnonzero(deg > 1)[3])
    dg.rowptr[i + 1] = int(g.rowptr[i]) - 1 if g.rowptr[i] > 0 else int(g.rowptr[i + 2]) + 1
    expect(dg, "csr_rowptr")


def test_csc_links_differ_with_equal_lengths():
    """Two CSC sources swapped between columns: every column keeps its length,
    only the link hash sees it."""
    say("case validate_csc_links")
    g = graph()
    dg = device(g, stored=False)
    colptr = g.csc()[0]
    row = g.csc()[1]
    ks = np.flatnonzero(np.diff(colptr) > 0)
    k1, k2 = int(ks[5]), int(ks[-5])
    e1, e2 = int(colptr[k1]), int(colptr[k2])
    assert row[e1] != row[e2]
    dg.row[e1], dg.row[e2] = int(row[e2]), int(row[e1])
    expect(dg, "the CSC does not hold the same links as the CSR")


def test_csc_value_differs():
    say("case validate_csc_value")
    g = graph()
    dg = device(g)
    dg.cval[100] = dg.cval[100] * 0.5
    expect(dg, "same links and values")


def test_csc_length_differs():
    say("case validate_csc_length")
    g = graph()
    dg = device(g, stored=False)
    colptr = g.csc()[0]
    k = int(np.flatnonzero(np.diff(colptr) > 1)[2])
    dg.colptr[k + 1] = int(colptr[k + 1]) - 1  # one link moves to the next column
    expect(dg, "column lengths differ")


def test_scratch_and_arguments():
    say("case validate_args")
    g = graph()
    dg = device(g)
    gs = dg.struct()
    need = rl.rlgl_validate_scratch_bytes(gs)
    assert need >= 4 * g.n
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(rl.RlglError) as e:
        rl.rlgl_validate(gs, rl.FP32C_FP64H, small, need - 256)
    assert e.value.status == rl.RLGL_ENOMEM
    ok = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(rl.RlglError) as e:
        rl.rlgl_validate(gs, 7, ok, need)
    assert e.value.status == rl.RLGL_EINVAL
    assert rl.rlgl_validate(gs, rl.FP32C_FP64H, ok, need) <= 1e-6


# ------------------------------------------------ out-of-range links in the solvers
#
# A solver reads link indices only through its own range checks: a source or
# destination outside [0, n) is never followed, and the call fails with
# RLGL_EINVAL instead of returning a wrong pi_hat.


def _broken(g, which, prec=rl.FP32C_FP64H):
    dg = device(g, prec, stored=False)
    # links 7 and nnz // 2 point past the last state
    if which == "csc":
        dg.row[7] = g.n + 3
        dg.row[g.nnz // 2] = g.n
    else:
        dg.col[7] = g.n + 3
        dg.col[g.nnz // 2] = g.n
    torch.cuda.synchronize()
    return dg


@pytest.mark.parametrize("route", [rl.ROUTE_PULL, rl.ROUTE_PUSH])
@pytest.mark.parametrize("relabel", [0, 1])
def test_solver_reports_links_out_of_range(route, relabel):
    g = graph()
    which = "csc" if route == rl.ROUTE_PULL else "csr"
    say("case broken_solve", which, relabel)
    dg = _broken(g, which)
    s = rl.Solver(dg, sched=rl.SCHED_ALL, route=route, relabel=relabel)
    st, info = s.solve(1e-9, max_steps=50, raise_on_error=False)
    assert st == rl.RLGL_EINVAL
    assert "outside its range" in rl.rlgl_last_error()
    s.close()


def test_small_solver_reports_links_out_of_range():
    g = graph()
    say("case broken_small")
    for which in ("csc", "csr"):
        dg = _broken(g, which, rl.FP64)
        s = rl.SmallSolver(dg, sched=rl.SCHED_MAXC if which == "csr" else rl.SCHED_ALL)
        st, info = s.solve(1e-9, max_steps=200000, raise_on_error=False)
        assert st == rl.RLGL_EINVAL and "out of range" in rl.rlgl_last_error()


@pytest.mark.parametrize("per_cu", [0, 8])
def test_batch_reports_links_out_of_range(per_cu):
    gs = [workloads.chung_lu(n, 2.3, 6.0, 0.0, 0.85, seed=60 + k, name=f"b{k}")
          for k, n in enumerate((3000, 1200, 5000))]
    say("case broken_batch", per_cu)
    db = rl.DeviceBatch(gs, precision=rl.FP32C_KAHANH, tol_l1=1e-6)
    # one source of chain 1 points past its last state
    db.row[int(db.edge_off[1]) + 5] = gs[1].n + 2
    torch.cuda.synchronize()
    bs = rl.BatchSolver(db, max_steps=1000, wg_size=256, wg_per_cu=per_cu)
    st, res, _ = bs.solve(raise_on_error=False)
    assert res[1]["status"] == rl.RLGL_EINVAL
    assert res[0]["status"] == rl.RLGL_OK and res[2]["status"] == rl.RLGL_OK
    assert st == rl.RLGL_EINVAL
    bs.close()
