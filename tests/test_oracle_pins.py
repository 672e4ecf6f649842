"""Pins of the reference oracle against what the paper and plain mathematics fix.

Every check here is independent of the oracle's own code path: closed forms
printed in the paper, exact symbolic traces, dense linear algebra, brute
force and invariants.  No GPU is used.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Example 1 (Sec. 3.1): an aperiodic irreducible 4-state chain.
P4 = np.array([[0, .5, .5, 0], [0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0]], dtype=np.float64)
PI4 = np.array([2, 1, 2, 2], dtype=np.float64) / 7.0


def chain_from_dense(P, c=1.0):
    n = P.shape[0]
    rows, cols = np.nonzero(P)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return oracle.Chain(rowptr, cols.astype(np.int32), P[rows, cols], c)


def random_chain(n, seed, c=0.85, dangling=0.0, deg=4.0):
    g = workloads.random_small(n, deg, c, seed, dangling)
    return oracle.Chain(g.rowptr, g.col, None, c), g


# ---------------------------------------------------------------- dense solves

def test_four_state_stationary_exact():
    assert np.allclose(oracle.stationary_dense(P4), PI4, atol=1e-15, rtol=0)
    assert np.allclose(oracle.stationary_gth(P4), PI4, atol=1e-15, rtol=0)


def test_dense_solvers_agree_and_fix_point():
    for seed in range(5):
        ch, _ = random_chain(40, seed, c=0.85, dangling=0.1)
        P = oracle.dense_P(ch)
        assert np.allclose(P.sum(1), 1.0, atol=1e-14)
        a = oracle.stationary_dense(P)
        b = oracle.stationary_gth(P)
        assert np.abs(a - b).sum() < 1e-13
        assert np.abs(a - a @ P).sum() < 1e-14
        w, v = np.linalg.eig(P.T)  # eigenvector of eigenvalue 1, a different library route
        k = np.argmin(np.abs(w - 1.0))
        e = np.real(v[:, k])
        e = e / e.sum()
        assert np.abs(a - e).sum() < 1e-12


def test_route_matches_dense_product():
    """route(M) is M P for the Google matrix with dangling rows uniform and
    duplicate links adding up (the chain the oracle documents)."""
    for seed in range(4):
        ch, g = random_chain(60, seed, c=0.7, dangling=0.15, deg=3.0)
        assert len(set(zip(np.repeat(np.arange(g.n), g.outdeg), g.col))) < g.nnz or seed > 0
        P = oracle.dense_P(ch)
        rng = np.random.default_rng(seed)
        M = rng.standard_normal(ch.n)
        assert np.abs(oracle.route(ch, M) - M @ P).max() < 1e-14


# ------------------------------------------------------------- Examples 1, 2

def test_example1_zero_history():
    """M_0 = e_1, G_1 = {1} gives H_2 = C_2 = 0 exactly (Example 1)."""
    ch = chain_from_dense(P4)
    s = oracle.State(ch, M0=np.array([1.0, 0, 0, 0]))
    assert np.array_equal(s.C, [-1.0, .5, .5, 0.0])
    assert np.array_equal(s.H, [1.0, 0, 0, 0])
    s.step_mask([1, 0, 0, 0])
    assert np.array_equal(s.H, np.zeros(4)) and np.array_equal(s.C, np.zeros(4))
    assert s.hsum == 0.0
    # the same start under RLGL_MaxC greens node 1 first: the solver reports it
    st, _, info = oracle.solve(ch, oracle.MAXC, eps=1e-12, M0=np.array([1.0, 0, 0, 0]))
    assert st == oracle.EZERO_HISTORY and info["t"] == 2


def _parse_trace(path):
    rows = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        t, h, c, g = [x.strip() for x in line.split("|")]
        rows.append((int(t), [x.strip() for x in h.split(",")], [x.strip() for x in c.split(",")], int(g)))
    return rows


def _eval_cells(cells, m):
    env = {"M1": m[0], "M2": m[1], "M3": m[2], "M4": m[3], "__builtins__": {}}
    return np.array([eval(x, env) for x in cells], dtype=np.float64)


@pytest.mark.parametrize("fname", ["example2_cycle_a.txt", "example2_cycle_b.txt"])
def test_example2_symbolic_traces(fname):
    """The H_t, C_t tables of Example 2, checked exactly with dyadic M_0."""
    rows = _parse_trace(os.path.join(GOLDEN, fname))
    ch = chain_from_dense(P4)
    rng = np.random.default_rng(7)
    for _ in range(5):
        m = rng.integers(1, 64, size=4).astype(np.float64) / 64.0
        s = oracle.State(ch, M0=m)
        for t, hc, cc, g in rows:
            assert s.t == t
            assert np.array_equal(s.H, _eval_cells(hc, m)), (fname, t, s.H)
            assert np.array_equal(s.C, _eval_cells(cc, m)), (fname, t, s.C)
            mask = np.zeros(4, dtype=bool)
            mask[g - 1] = True
            s.step_mask(mask)


def test_example2_first_cycle_converges_uniform():
    """With uniform M_0 the first cycle converges: C_t -> 0 and pi_hat -> pi*."""
    ch = chain_from_dense(P4)
    s = oracle.State(ch)
    cyc = [1, 0, 2, 3]
    for k in range(400):
        mask = np.zeros(4, dtype=bool)
        mask[cyc[k % 4]] = True
        s.step_mask(mask)
    assert s.l1 < 1e-15
    assert np.abs(s.pi_hat - PI4).sum() < 1e-14


def test_example2_second_cycle_never_converges():
    """Second cycle: ||C_t||_1 stays at 2|M3-M4| forever unless M3 = M4, in
    which case C_3 = 0 and pi_hat_3 = pi* exactly."""
    ch = chain_from_dense(P4)
    cyc = [0, 1, 3, 2]
    m = np.array([0.25, 0.25, 0.375, 0.125])
    s = oracle.State(ch, M0=m)
    for k in range(200):
        mask = np.zeros(4, dtype=bool)
        mask[cyc[k % 4]] = True
        s.step_mask(mask)
        if s.t >= 3:
            assert s.l1 == pytest.approx(2 * abs(m[2] - m[3]), abs=1e-15)
    m = np.full(4, 0.25)
    s = oracle.State(ch, M0=m)
    for k in range(2):
        mask = np.zeros(4, dtype=bool)
        mask[cyc[k]] = True
        s.step_mask(mask)
    assert s.t == 3 and s.l1 == 0.0
    assert np.abs(s.pi_hat - PI4).max() < 1e-15


def test_single_node_forever_stalls():
    """G_t = {1} for all t stops decreasing ||C_t||_1 after one step (Sec. 2.2)."""
    ch = chain_from_dense(P4)
    s = oracle.State(ch)
    l1 = []
    for _ in range(6):
        s.step_mask([1, 0, 0, 0])
        l1.append(s.l1)
    assert l1[0] > 0 and all(x == l1[0] for x in l1)


# ------------------------------------------------- power iteration special case

def test_all_green_equals_power_iteration():
    """G_t = [N] gives H_t = M_0 P^(t-1) and H_t 1 = 1 (Sec. 2.3.1)."""
    for seed in range(3):
        ch, _ = random_chain(50, seed, c=0.8, dangling=0.1)
        P = oracle.dense_P(ch)
        M0 = np.full(ch.n, 1.0 / ch.n)
        s = oracle.State(ch)
        for t in range(1, 25):
            ref = M0 @ np.linalg.matrix_power(P, t - 1)
            assert np.abs(s.H - ref).max() < 1e-15 * t + 1e-16
            assert abs(s.hsum - 1.0) < 1e-14
            s.step(oracle.ALL)


def test_power_iteration_reference_accuracy():
    for seed in range(3):
        ch, _ = random_chain(80, seed, c=0.85, dangling=0.05)
        pistar = oracle.stationary_dense(oracle.dense_P(ch))
        x, _ = oracle.reference_pagerank(ch, 1e-13)
        assert np.abs(x - pistar).sum() <= 1e-13


# ------------------------------------------------------------------ invariants

@pytest.mark.parametrize("sched", [oracle.ALL, oracle.THRESHOLD, oracle.TOPK, oracle.MAXC])
def test_invariants_every_step(sched):
    """sum C_t = 0 (Sec. 2.1), H_t + C_t = H_t P (eq. (7) with C_0 = 0),
    ||C_t||_1 non-increasing (proof of Theorem 2), and for G_t = [N] the
    Dobrushin bound ||C_t||_1 <= 2 c^(t-1) (Theorem 3 with m = 1)."""
    for seed in range(3):
        c = 0.85
        ch, _ = random_chain(70, seed, c=c, dangling=0.1)
        P = oracle.dense_P(ch)
        s = oracle.State(ch)
        prev = s.l1
        for _ in range(40):
            assert abs(s.C.sum()) < 1e-15
            assert np.abs(s.H + s.C - s.H @ P).max() < 1e-15
            assert s.l1 <= prev * (1 + 1e-13) + 1e-16
            if sched == oracle.ALL:
                assert s.l1 <= 2 * c ** (s.t - 1) + 1e-15
            prev = s.l1
            s.step(sched, k=5)


def test_residual_equals_cash_over_history():
    """||pi_hat - pi_hat P||_1 = ||C_t||_1 / |H_t 1| (Algorithm 1, step (7))."""
    ch, _ = random_chain(200, 3, c=0.85, dangling=0.1)
    st, pi, info, C, H = oracle.solve(ch, oracle.THRESHOLD, eps=1e-9, want_state=True)
    assert st == oracle.OK
    assert oracle.residual(ch, pi) == pytest.approx(info["resid"], rel=1e-6)


def test_pagerank_error_bound():
    """With c < 1: ||pi_hat - pi*||_1 <= resid / (1 - c) (eq. (9) with the
    contraction of Theorem 3); the stopping rule at (1-c)*tol certifies tol."""
    for seed in range(4):
        for sched in (oracle.ALL, oracle.THRESHOLD, oracle.MAXC, oracle.TOPK):
            c = 0.85
            ch, _ = random_chain(120, seed, c=c, dangling=0.1)
            pistar = oracle.stationary_dense(oracle.dense_P(ch))
            st, pi, info = oracle.solve(ch, sched, eps=(1 - c) * 1e-8, k=7)
            assert st == oracle.OK
            err = np.abs(pi - pistar).sum()
            assert err <= info["resid"] / (1 - c) + 1e-14
            assert err <= 1e-8


# ------------------------------------------------------------- closed forms

def test_two_wheels_degree_law():
    """Two-wheels graph (Sec. 6), simple random walk: pi_i = deg_i / 42."""
    edges = np.loadtxt(os.path.join(GOLDEN, "two_wheels_edges.txt"), dtype=np.int64) - 1
    assert edges.shape == (21, 2)
    src = np.concatenate([edges[:, 0], edges[:, 1]])
    dst = np.concatenate([edges[:, 1], edges[:, 0]])
    g = workloads.from_edges(12, src, dst, 1.0)
    deg = g.outdeg.astype(np.float64)
    assert list(deg) == [3, 3, 4, 3, 3, 3, 6, 4, 3, 3, 3, 4]
    pi_ref = deg / 42.0
    ch = oracle.Chain(g.rowptr, g.col, None, 1.0)
    assert np.abs(oracle.stationary_dense(oracle.dense_P(ch)) - pi_ref).max() < 1e-15
    assert np.abs(oracle.stationary_gth(oracle.dense_P(ch)) - pi_ref).max() < 1e-15
    for sched in (oracle.ALL, oracle.THRESHOLD, oracle.MAXC, oracle.TOPK):
        st, pi, info = oracle.solve(ch, sched, eps=1e-13, k=3)
        assert st == oracle.OK, sched
        assert np.abs(pi - pi_ref).sum() < 1e-11, (sched, info)


def _mf_sbm(K, n, p, q):
    N1, N2 = K * n, n
    N = N1 + N2
    A = np.full((N, N), q)
    A[:N1, :N1] = p
    A[N1:, N1:] = p
    return A / A.sum(1, keepdims=True), N1


def test_two_block_mean_field_rates():
    """Sec. 4: lambda_2 = (p^2-q^2)K/((pK+q)(qK+p)); one-block schedules
    contract ||C_t||_1 by pK/(pK+q) (G = B_1) and p/(qK+p) (G = B_2)."""
    for K, n, p, q in [(3, 4, 0.5, 0.1), (5, 3, 0.3, 0.02), (2, 6, 0.9, 0.4)]:
        P, N1 = _mf_sbm(K, n, p, q)
        lam = sorted(np.abs(np.linalg.eigvals(P)))[-2]
        assert lam == pytest.approx((p * p - q * q) * K / ((p * K + q) * (q * K + p)), rel=1e-12)
        ch = chain_from_dense(P)
        for block, factor in ((np.arange(P.shape[0]) < N1, p * K / (p * K + q)),
                              (np.arange(P.shape[0]) >= N1, p / (q * K + p))):
            s = oracle.State(ch)
            for _ in range(8):
                before = s.l1
                s.step_mask(block)
                assert s.l1 == pytest.approx(factor * before, rel=1e-10)


# ------------------------------------------------------------------ selection

def test_selection_brute_force():
    rng = np.random.default_rng(11)
    for trial in range(30):
        n = int(rng.integers(1, 300))
        C = rng.standard_normal(n) * 10.0 ** rng.integers(-12, 0)
        if n > 4:  # plant ties, including ties in |C| with opposite signs
            C[1] = -C[0]
            C[3] = C[2]
        th = oracle.theta(C, 1.0)
        assert th == pytest.approx(math.fsum(np.abs(C)) / n, rel=1e-14)
        assert np.array_equal(oracle.select(C, oracle.THRESHOLD, th), np.abs(C) >= th)
        mx = np.abs(C).max()
        assert np.array_equal(oracle.select(C, oracle.MAXC), np.abs(C) == mx)
        k = int(rng.integers(1, n + 1))
        order = sorted(range(n), key=lambda i: (-abs(C[i]), i))
        want = np.zeros(n, dtype=bool)
        want[order[:k]] = True
        assert np.array_equal(oracle.select(C, oracle.TOPK, k=k), want)
        assert oracle.select(C, oracle.ALL).all()
        r = 2.0
        assert oracle.theta(C, r) == pytest.approx(math.sqrt(math.fsum(C * C) / n), rel=1e-13)


def test_zero_cash_green_nodes_push_nothing():
    """A green node with C_i = 0 moves nothing and uses no link."""
    ch = chain_from_dense(P4)
    s = oracle.State.from_arrays(ch, C=[0.0, 0.5, -0.5, 0.0], H=[0.25] * 4, hsum=1.0)
    s.step_mask([1, 0, 0, 1])
    assert s.edges == 0 and np.array_equal(s.C, [0.0, 0.5, -0.5, 0.0])
    s.step_mask([0, 1, 0, 0])
    assert s.edges == 1


def test_largest_scc_input():
    """The undamped workload's input: the largest strongly connected component
    of a graph built by hand, renumbered in order, its internal links kept."""
    import workloads
    # a 3-cycle 0->1->2->0, a 4-cycle 3->4->5->6->3 with a self-loop on 4,
    # a one-way bridge 2->3 and a tail 6->7
    src = np.array([0, 1, 2, 3, 4, 5, 6, 4, 2, 6], dtype=np.int32)
    dst = np.array([1, 2, 0, 4, 5, 6, 3, 4, 3, 7], dtype=np.int32)
    g = workloads.from_edges(8, src, dst, 0.85, name="toy")
    h = workloads.largest_scc(g, c=1.0)
    assert h.n == 4 and h.c == 1.0 and h.nnz == 5
    edges = sorted(zip(np.repeat(np.arange(h.n), h.outdeg).tolist(), h.col.tolist()))
    assert edges == [(0, 1), (1, 1), (1, 2), (2, 3), (3, 0)]
    assert np.all(h.outdeg > 0)


def test_pc_generator_and_selection():
    """RLGL_PC drawn for all nodes at once.  The generator is splitmix64 (the
    three first outputs from state 0 are the published reference values);
    node i is green with frequency |C_i| / max |C|; the (seed, step) pair
    fixes the draw."""
    assert [oracle.splitmix64(0, i) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                           0x06C45D188009454F]
    C = np.array([0.0, -1.0, 0.5, 0.25, -0.125, 1.0, 0.75])
    steps = 4000
    counts = sum(oracle.select(C, oracle.PC, seed=11, t=t).astype(int) for t in range(1, steps + 1))
    p = np.abs(C) / np.abs(C).max()
    assert counts[0] == 0 and counts[1] == steps and counts[5] == steps
    sd = np.sqrt(steps * p * (1 - p))
    assert np.all(np.abs(counts - steps * p) <= 5 * sd + 1e-9)
    x = np.linspace(0.1, 1.0, 64)
    a = oracle.select(x, oracle.PC, seed=3, t=5)
    assert np.array_equal(a, oracle.select(x, oracle.PC, seed=3, t=5))
    assert not np.array_equal(a, oracle.select(x, oracle.PC, seed=4, t=5))
    assert not np.array_equal(a, oracle.select(x, oracle.PC, seed=3, t=6))
    # the draw of node i at step t is splitmix64 output t 2^32 + i, top 53 bits
    u = np.array([(oracle.splitmix64(3, (5 << 32) + i) >> 11) * 2.0 ** -53 for i in range(64)])
    assert np.array_equal(a, u < x / x.max())


def test_pc_solve_reaches_stationary_distribution():
    ch, _ = random_chain(60, 5, c=0.85, dangling=0.1)
    x = oracle.stationary_gth(oracle.dense_P(ch))
    st, pi, info = oracle.solve(ch, oracle.PC, eps=1e-13 * 0.15, seed=9)
    assert st == oracle.OK
    assert np.abs(pi - x).sum() <= 1e-12
    # invariants hold along a PC trajectory
    s = oracle.State(ch)
    for _ in range(50):
        s.step(oracle.PC, seed=9)
        assert abs(s.C.sum()) <= 1e-13


def test_parallel_power_iteration_baseline_agrees():
    """The all-core power iteration (a CPU baseline) takes the same iterates
    as the serial one."""
    ch, _ = random_chain(3000, 2, c=0.85, dangling=0.1, deg=6.0)
    st, x, it = oracle.power_iteration(ch, 1e-13)
    st2, y, it2, threads = oracle.power_iteration_omp(ch, 1e-13)
    assert st == st2 == oracle.OK and it == it2 and threads >= 1
    assert np.abs(x - y).sum() <= 1e-13


def test_gso_pr_error_identity():
    """Algorithm 2 keeps C_t >= 0 and H_t (I - cP) + C_t = (1-c) s, so
    pi* - H_t = C_t (I - cP)^-1 >= 0 and ||pi* - H_t||_1 = ||C_t||_1 / (1-c)
    exactly (the row sums of (I - cP)^-1 are 1/(1-c))."""
    ch, g = random_chain(80, 4, c=0.85, dangling=0.0)
    P = oracle.dense_P(ch)
    W = oracle.dense_P(oracle.Chain(g.rowptr, g.col, None, 1.0))
    pi = oracle.stationary_gth(P)
    for eps in (1e-2, 1e-5, 1e-9):
        st, H, C, steps, edges = oracle.gso_pr(ch, eps)
        assert st == oracle.OK and np.all(C >= 0.0) and C.sum() < eps
        assert np.abs(H @ (np.eye(ch.n) - 0.85 * W) + C - 0.15 / ch.n).max() < 1e-15
        assert np.all(pi - H >= -1e-16)
        assert abs(np.abs(pi - H).sum() - C.sum() / 0.15) < 1e-14


def test_gso_pr_is_rlgl_on_the_auxiliary_chain():
    """Sec. 2.4: RLGL on P^(0) from M_0 = e_0, with the green set {k} that
    Algorithm 2 picks, reproduces Algorithm 2's H_t and C_t on states 1..N;
    the first step of RLGL gives C_1 = (-(1-c), (1-c) s) and H_1 = e_0."""
    import workloads
    c = 0.85
    g = workloads.poisson_uniform(60, 3.0, c, seed=2)
    ch = oracle.Chain(g.rowptr, g.col, None, c)
    aux = workloads.auxiliary_node_chain(g, c)
    cha = oracle.Chain(aux.rowptr, aux.col, aux.val(), 1.0)
    e0 = np.zeros(aux.n)
    e0[0] = 1.0
    st0 = oracle.State(cha, M0=e0)
    assert np.allclose(st0.C, np.concatenate([[-(1 - c)], np.full(g.n, (1 - c) / g.n)]), atol=1e-16, rtol=0)
    assert np.array_equal(st0.H, e0) and st0.hsum == 1.0
    # Algorithm 2 step by step, mirrored on the auxiliary chain
    C = np.full(g.n, (1 - c) / g.n)
    for t in range(200):
        k = int(np.argmax(C))
        mask = np.zeros(aux.n, dtype=bool)
        mask[k + 1] = True
        st0.step_mask(mask)
        _, H, C, steps, _ = oracle.gso_pr(ch, 0.0, max_steps=t + 1)
        assert steps == t + 1
        assert np.abs(st0.H[1:] - H).max() < 1e-15
        assert np.abs(st0.C[1:] - C).max() < 1e-15


# ------------------------------------------------ block schedules (Sec. 5.3)

from oracle import blocks  # noqa: E402

SBM3 = ((50, 20, 10), 0.1, 0.01)


def _block_vector(c, N):
    return np.repeat(np.asarray(c, dtype=np.float64), N)


def test_block_step_equals_the_dense_step():
    """The three-number block dynamics is the RLGL step of the dense SBM chain
    with every state of the green blocks green, for all seven actions."""
    N, p, q = SBM3
    P = blocks.dense_chain(N, p, q)
    ch = chain_from_dense(P)
    blk = np.repeat(np.arange(3), N)
    rng = np.random.default_rng(5)
    for trial in range(6):
        c = rng.standard_normal(3)
        c[2] = -(N[0] * c[0] + N[1] * c[1]) / N[2]  # cash balance
        for a in blocks.ACTIONS:
            s = oracle.State.from_arrays(ch, _block_vector(c, N), np.zeros(P.shape[0]), 1.0)
            s.step_mask(np.isin(blk, a))
            want = blocks.step(c, a, N, p, q)
            scale = np.abs(c).max()  # the dense step adds up to 80 terms of this size
            assert np.abs(s.C - _block_vector(want, N)).max() < 1e-14 * scale
            assert abs(float(np.dot(N, want))) < 1e-13 * scale


def test_block_initial_cash_closed_form():
    """One power-iteration step from the uniform M_0 gives the block cash of
    the closed form of Sec. 5.3 (there written with the opposite sign of C)."""
    for N, p, q in (SBM3, ((30, 30, 5), 0.2, 0.05), ((7, 5, 3), 0.5, 0.1)):
        P = blocks.dense_chain(N, p, q)
        n = P.shape[0]
        M0 = np.full(n, 1.0 / n)
        C1 = oracle.route(chain_from_dense(P), M0) - M0
        blk = np.repeat(np.arange(3), N)
        c0 = np.array([C1[blk == j].mean() for j in range(3)])
        zeta = p / q - 1.0
        Na = np.asarray(N, dtype=np.float64)
        closed = np.array([zeta / n * sum(Na[j] * (Na[j] - Na[i]) / ((Na[i] * zeta + n) * (Na[j] * zeta + n))
                                          for j in range(3)) for i in range(3)])
        assert np.abs(c0 + closed).max() < 1e-16
        assert np.abs(C1 - _block_vector(c0, N)).max() < 1e-16


def test_block_shape_covers_the_half_space():
    """z_2 in [-2, 2] and (y_2, y_3) correspond one to one (the three cases of
    Sec. 5.3): the shape has unit L1 norm, zero balance and c_1 >= 0."""
    N = np.array(SBM3[0], dtype=np.float64)
    z2 = np.linspace(-2.0, 2.0, 401)
    c = blocks.shape_from_z2(z2, N)
    assert np.allclose((np.abs(c) * N).sum(axis=1), 1.0, atol=1e-15)
    assert np.allclose((c * N).sum(axis=1), 0.0, atol=1e-15)
    assert np.all(c[:, 0] >= -1e-18)
    back = np.array([blocks.z_of(ci, N, 1.0)[1] for ci in c])
    assert np.abs(back - z2).max() < 1e-12


def test_optimal_block_schedule():
    """Sec. 5.3 on the mean-field SBM (N = 50, 20, 10; p = 0.1, q = 0.01;
    eps = 1e-14) from the power-iteration start: the dynamic-programming
    schedule routes mostly the two small blocks, never all three (power
    iteration), needs fewer steps than power iteration at a fraction of its
    cost, is no worse than simple fixed schedules, and its value function
    predicts the cost it pays."""
    N, p, q = SBM3
    eps = 1e-14
    pol = blocks.Policy(N, p, q, eps, n1=1400, n2=81)
    assert np.all(pol.V[0] == 0.0) and np.all(pol.V >= 0.0)
    P = blocks.dense_chain(N, p, q)
    n = P.shape[0]
    C1 = oracle.route(chain_from_dense(P), np.full(n, 1.0 / n)) - 1.0 / n
    blk = np.repeat(np.arange(3), N)
    c0 = np.array([C1[blk == j].mean() for j in range(3)])
    cost, steps, acts = blocks.run(c0, pol.action, N, p, q, eps)
    pi_cost, pi_steps, _ = blocks.run(c0, lambda c: 6, N, p, q, eps)
    assert np.isfinite(cost) and cost < pi_cost / 5 and steps < pi_steps
    hist = np.bincount(acts, minlength=7)
    assert hist[6] == 0 and hist[1] + hist[2] >= 0.75 * steps
    assert abs(pol.value(c0) - cost) <= 0.1 * cost
    for cycle in ((2, 2, 2, 4), (1, 2), (0, 1, 2), (4,), (3, 4, 5)):
        it = iter(range(10 ** 9))
        fixed, _, _ = blocks.run(c0, lambda c: cycle[next(it) % len(cycle)], N, p, q, eps)
        assert cost <= fixed * 1.001, (cycle, fixed, cost)
