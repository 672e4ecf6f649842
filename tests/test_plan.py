"""The static pull plans (host only, no GPU): on adversarial column pointers
every link lies in exactly one item, every column in exactly one run or is a
long column, the items keep their size limits, the long-column slots name
their columns, and the plan fits the item count the device workspace is
sized for.  Malformed column pointers are rejected."""
import numpy as np
import pytest

import paper_2008_02710_amd as rl

# single chain: runs of at most 512 links and 64 columns, pieces of 512 links
# for columns above 512; batched: pieces of 4096 links for columns above
# 2048, runs of at most 2048 links and 1024 columns
LIMITS = {"pull": dict(long_above=512, piece=512, run_links=512, run_cols=64),
          "batch": dict(long_above=2048, piece=4096, run_links=2048, run_cols=1024)}


def colptrs():
    rng = np.random.default_rng(7)
    cases = {
        "one column, no links": [0],
        "one column, one link": [1],
        "one long column": [100000],
        "no links at all": [0] * 3000,
        "on the limits": [0, 511, 512, 513, 0, 1024, 1025, 2047, 2048, 2049, 4096, 4097, 0, 8193, 0],
        "64 and 65 one-link columns": [1] * 64 + [0] + [1] * 65,
        "1024 and 1025 one-link columns": [1] * 1024 + [0] + [1] * 1025,
        "alternating empty and long": [0, 600, 0, 3000, 0, 600, 0, 9000, 0],
        "power law": list(np.minimum((rng.pareto(1.1, 20000) * 3).astype(np.int64), 200000)),
        "uniform small": list(rng.integers(0, 12, 5000)),
        "dense": list(rng.integers(400, 700, 2000)),
    }
    for name, deg in cases.items():
        cp = np.zeros(len(deg) + 1, dtype=np.int64)
        cp[1:] = np.cumsum(deg)
        yield name, cp.astype(np.int32)


CASES = list(colptrs())


def check_plan(kind, cp, plan):
    lim = LIMITS[kind]
    n = cp.size - 1
    nnz = int(cp[-1])
    deg = np.diff(cp)
    items, long_cols = plan["items"], plan["long_cols"]
    assert len(items) <= plan["item_bound"]
    covered = np.zeros(nnz, dtype=np.int32)
    col_seen = np.zeros(n, dtype=np.int32)
    piece_links = np.zeros(len(long_cols), dtype=np.int64)
    is_long = deg > lim["long_above"]
    assert np.array_equal(np.sort(long_cols), np.flatnonzero(is_long))
    for x, y, p0, p1 in items:
        assert 0 <= p0 <= p1 <= nnz
        covered[p0:p1] += 1
        if x >= 0:
            # a run of whole columns [x, y)
            assert 0 <= x < y <= n and y - x <= lim["run_cols"]
            assert p0 == cp[x] and p1 == cp[y] and p1 - p0 <= lim["run_links"]
            assert not is_long[x:y].any()
            col_seen[x:y] += 1
        else:
            slot = -1 - x
            assert 0 <= slot < len(long_cols) and long_cols[slot] == y
            assert cp[y] <= p0 < p1 <= cp[y + 1] and p1 - p0 <= lim["piece"]
            piece_links[slot] += p1 - p0
    assert np.all(covered == 1), "every link in exactly one item"
    assert np.all(col_seen[~is_long] == 1) and np.all(col_seen[is_long] == 0), "every column once"
    assert np.array_equal(piece_links, deg[long_cols]), "the pieces of a long column add up to it"


@pytest.mark.parametrize("name,cp", CASES, ids=[c[0] for c in CASES])
def test_single_chain_plan(name, cp):
    check_plan("pull", cp, rl.rlgl_pull_plan(cp))


@pytest.mark.parametrize("name,cp", CASES, ids=[c[0] for c in CASES])
def test_batched_chain_plan(name, cp):
    plan = rl.rlgl_batch_chain_plan(cp)
    check_plan("batch", cp, plan)
    # the pieces come first
    items = plan["items"]
    assert plan["n_pieces"] == int((items[:, 0] < 0).sum())
    assert np.all(items[:plan["n_pieces"], 0] < 0) and np.all(items[plan["n_pieces"]:, 0] >= 0)


def test_single_chain_pieces_spread_over_the_runs():
    """The pieces of the single-chain plan sit among the first three
    quarters of its runs, not all at the start."""
    deg = [5] * 4000
    for q in range(0, 4000, 400):
        deg[q] = 1500
    cp = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    items = rl.rlgl_pull_plan(cp)["items"]
    pos = np.flatnonzero(items[:, 0] < 0)
    runs_before = np.array([int((items[:p, 0] >= 0).sum()) for p in pos])
    n_runs = int((items[:, 0] >= 0).sum())
    assert runs_before.max() <= 0.75 * n_runs + 1 and runs_before.min() > 0


@pytest.mark.parametrize("fn", [rl.rlgl_pull_plan, rl.rlgl_batch_chain_plan])
def test_malformed_column_pointers_are_rejected(fn):
    for bad in ([1, 3, 5], [0, 4, 2, 6], [0, -1, 2]):
        with pytest.raises(rl.RlglError) as e:
            fn(np.array(bad, dtype=np.int32))
        assert e.value.status == rl.RLGL_EINVAL
