"""Helpers shared by the GPU tests: device upload of seeded workloads and the
matching oracle chain."""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_chain(g, explicit_val=True):
    return oracle.Chain(g.rowptr, g.col, g.val() if explicit_val else None, g.c)


def solver(g, precision, explicit_val=True, with_csc=True, **opts):
    import paper_2008_02710_amd as rl
    dg = rl.DeviceGraph.from_workload(g, precision=precision, with_csc=with_csc, explicit_val=explicit_val)
    return rl.Solver(dg, **opts)


def to_np(t):
    return t.detach().cpu().numpy()


def l1(a, b):
    return float(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)).sum())
