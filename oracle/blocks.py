"""Block schedules on the three-block mean-field SBM (Sec. 5 of Avrachenkov,
Brown, Litvak, arXiv 2008.02710).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: plain numpy in FP64,
used by ``tests/`` alone, sharing nothing with the HIP library.

The chain.  Three blocks of N_1, N_2, N_3 states; a state links to every
state of its own block with weight p and to every state of another block with
weight q; rows are normalised (the undamped chain of the SBM section).  By
symmetry every state of block j holds the same cash c_j under any block
schedule, so the process is the three numbers c = (c_1, c_2, c_3) with the
cash balance N_1 c_1 + N_2 c_2 + N_3 c_3 = 0.

A step with green blocks a (one of the seven non-empty subsets a_1..a_7 of
Sec. 5.3) moves the cash of every state of those blocks: a state of block j
sends w_ji / D_j of its cash to each state of block i, with w_jj = p,
w_ji = q (i != j) and D_j = sum_i N_i w_ji.  Its cost kappa(a) is the sum over
the green blocks of N_j D_j, the expected number of links they route.

The optimal block schedule minimises the total cost of reaching
||c||_1 = sum N_j |c_j| <= eps (the dynamic programming equation of
Sec. 5.3).  As there, the state is z = (z_1, z_2) with
z_1 = log10(||c||_1 / eps) and z_2 = y_2 - y_3, y_j = 2 N_j c_j / ||c||_1,
on the half space c_1 >= 0 (V(-c) = V(c), the symmetry theorem of Sec. 5.3),
and V is computed by backward induction along z_1, which no action
increases.  Readings where the text is silent (listed with the others in the
design notes): V between grid points is the bilinear interpolation of the
grid values; an action whose next z_1 stays inside the current grid cell
refers to the row being computed, which is then solved by repeated sweeps
until it no longer changes; ties between actions go to the lowest index.
"""
from __future__ import annotations

import numpy as np

# a_1 .. a_7 of Sec. 5.3, blocks numbered from 0
ACTIONS = ((0,), (1,), (2,), (0, 1), (1, 2), (0, 2), (0, 1, 2))


def weights(N, p: float, q: float):
    """(w, D): w[j, i] the weight of a link from block j to a state of block
    i, D[j] = sum_i N_i w[j, i]."""
    N = np.asarray(N, dtype=np.float64)
    w = np.full((3, 3), float(q))
    np.fill_diagonal(w, float(p))
    return w, w @ N


def dense_chain(N, p: float, q: float) -> np.ndarray:
    """The SBM transition matrix written out, states ordered block by block."""
    blk = np.repeat(np.arange(3), N)
    w, _ = weights(N, p, q)
    A = w[blk][:, blk]
    return A / A.sum(axis=1, keepdims=True)


def kappa(N, p: float, q: float) -> np.ndarray:
    """Cost of each action a_1..a_7 (Sec. 5.3): sum over its blocks of N_j D_j."""
    N = np.asarray(N, dtype=np.float64)
    _, D = weights(N, p, q)
    per = N * D
    return np.array([sum(per[j] for j in a) for a in ACTIONS])


def step(c, a, N, p: float, q: float) -> np.ndarray:
    """Block cash after one step with green blocks `a` (the cash recursion
    C' = C - M + M P restricted to block-constant cash)."""
    c = np.asarray(c, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    w, D = weights(N, p, q)
    out = c.copy()
    for j in a:
        out[j] -= c[j]
    for j in a:
        out += N[j] * c[j] * w[j] / D[j]
    return out


def l1(c, N) -> float:
    return float(np.sum(np.asarray(N, dtype=np.float64) * np.abs(c)))


def shape_from_z2(z2, N) -> np.ndarray:
    """Block cash of unit ||c||_1 with c_1 >= 0 and y_2 - y_3 = z2 (the three
    cases of Sec. 5.3)."""
    z2 = np.asarray(z2, dtype=np.float64)
    y2 = np.where(z2 >= 1.0, z2 - 1.0, np.where(z2 >= -1.0, (z2 - 1.0) / 2.0, -1.0))
    y3 = np.where(z2 >= 1.0, -1.0, np.where(z2 >= -1.0, -(z2 + 1.0) / 2.0, -z2 - 1.0))
    y1 = -(y2 + y3)
    y = np.stack([y1, y2, y3], axis=-1)
    return y / (2.0 * np.asarray(N, dtype=np.float64))


def z_of(c, N, eps: float):
    """(z_1, z_2, c on the half space c_1 >= 0)."""
    c = np.asarray(c, dtype=np.float64)
    if c[0] < 0.0:
        c = -c
    n1 = l1(c, N)
    y = 2.0 * np.asarray(N, dtype=np.float64) * c / n1
    return np.log10(n1 / eps), float(y[1] - y[2]), c


class Policy:
    """Value function V and optimal actions A on the grid z_1 = i h
    (i = 0..n1-1, h = z1_max / (n1 - 1)), z_2 = -2 + 4 j / (n2 - 1)."""

    def __init__(self, N, p: float, q: float, eps: float, z1_max: float = 14.0, n1: int = 14000,
                 n2: int = 321, sweeps: int = 500, tol: float = 1e-13):
        self.N = np.asarray(N, dtype=np.float64)
        self.p, self.q, self.eps = float(p), float(q), float(eps)
        self.z1 = np.linspace(0.0, z1_max, n1)
        self.z2 = np.linspace(-2.0, 2.0, n2)
        self.h = self.z1[1] - self.z1[0]
        self.kappa = kappa(self.N, p, q)
        # every action maps the unit shape at z2[j] to a shape of norm r: the
        # next state is (z_1 + log10 r, z_2') whatever z_1 is (f_a is linear)
        shapes = shape_from_z2(self.z2, self.N)
        nA = len(ACTIONS)
        self.dz = np.empty((nA, n2))
        self.z2n = np.empty((nA, n2))
        for k, a in enumerate(ACTIONS):
            for j in range(n2):
                c = step(shapes[j], a, self.N, p, q)
                r = l1(c, self.N)
                if r == 0.0:
                    self.dz[k, j] = -np.inf
                    self.z2n[k, j] = 0.0
                    continue
                _, z2n, _ = z_of(c, self.N, 1.0)
                self.dz[k, j] = np.log10(r)
                self.z2n[k, j] = z2n
        # linear interpolation along z_2 of each next state: columns j0, j0+1, weight u
        step2 = self.z2[1] - self.z2[0]
        pos = np.clip((self.z2n + 2.0) / step2, 0.0, n2 - 1.0)
        self.j0 = np.minimum(np.floor(pos).astype(np.int64), n2 - 2)
        self.u = pos - self.j0
        self.V = np.zeros((n1, n2))
        self.A = np.full((n1, n2), -1, dtype=np.int64)
        self.max_sweeps = 0
        for i in range(1, n1):
            self._row(i, sweeps, tol)

    def _at(self, rows: np.ndarray, k: int) -> np.ndarray:
        """V on grid rows `rows` (one per column j) at the next z_2 of action k."""
        j0, u = self.j0[k], self.u[k]
        return (1.0 - u) * self.V[rows, j0] + u * self.V[rows, j0 + 1]

    def _row(self, i: int, sweeps: int, tol: float):
        h = self.h
        self.V[i] = self.V[i - 1]
        # where each action lands along z_1: rows lo and lo + 1, weight t
        land = []
        for k in range(len(ACTIONS)):
            zn = np.maximum(self.z1[i] + self.dz[k], -1.0)  # at or below 0: eps reached, V = 0
            r = zn / h
            i0 = np.floor(r).astype(np.int64)
            t = r - i0
            lo = np.maximum(i0, 0)
            hi = np.minimum(lo + 1, i)
            land.append((zn <= 0.0, i0 >= 0, lo, hi, t))
        for sweep in range(sweeps):
            cand = np.empty((len(ACTIONS), len(self.z2)))
            for k in range(len(ACTIONS)):
                done, has_lo, lo, hi, t = land[k]
                v0 = np.where(has_lo, self._at(lo, k), 0.0)
                v1 = self._at(hi, k)
                cand[k] = self.kappa[k] + np.where(done, 0.0, (1.0 - t) * v0 + t * v1)
            new = cand.min(axis=0)
            self.A[i] = cand.argmin(axis=0)
            change = np.max(np.abs(new - self.V[i]))
            self.V[i] = new
            self.max_sweeps = max(self.max_sweeps, sweep + 1)
            if change <= tol * max(1.0, np.max(np.abs(new))):
                break

    def action(self, c) -> int:
        """Optimal action index at block cash c (nearest grid point)."""
        z1, z2, _ = z_of(c, self.N, self.eps)
        i = int(np.clip(np.rint(z1 / self.h), 1, len(self.z1) - 1))
        j = int(np.clip(np.rint((z2 + 2.0) / 4.0 * (len(self.z2) - 1)), 0, len(self.z2) - 1))
        return int(self.A[i, j])

    def value(self, c) -> float:
        """V at block cash c (bilinear interpolation of the grid)."""
        z1, z2, _ = z_of(c, self.N, self.eps)
        if z1 <= 0.0:
            return 0.0
        r = min(z1 / self.h, len(self.z1) - 1 - 1e-12)
        i0 = int(np.floor(r))
        t = r - i0
        v0 = np.interp(z2, self.z2, self.V[i0])
        v1 = np.interp(z2, self.z2, self.V[i0 + 1])
        return float((1 - t) * v0 + t * v1)


def run(c0, choose, N, p: float, q: float, eps: float, max_steps: int = 100000):
    """Applies choose(c) -> action index from block cash c0 until
    ||c||_1 <= eps; returns (total cost, steps, actions)."""
    kap = kappa(N, p, q)
    c = np.asarray(c0, dtype=np.float64)
    cost, acts = 0.0, []
    for _ in range(max_steps):
        if l1(c, N) <= eps:
            return cost, len(acts), acts
        k = choose(c)
        acts.append(k)
        cost += kap[k]
        c = step(c, ACTIONS[k], N, p, q)
    if l1(c, N) <= eps:
        return cost, len(acts), acts
    return np.inf, len(acts), acts
