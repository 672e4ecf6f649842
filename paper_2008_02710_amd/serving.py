"""Request loop over a serving pool: open-loop arrivals, first-come
first-served admission by slot and arena footprint, continuous batching.

The loop runs on the host.  Each pass it enqueues a few lockstep iterations
of every resident chain, and while they run it moves the requests whose
arrival time has passed into a FIFO queue and admits from the head of the
queue while the pool has a free slot and a large enough arena block (the pool
builds the plan and enqueues the upload on its own copy stream); then it
waits for the iterations and collects, copies out and releases the chains
that finished.  A request's latency runs from its arrival to the moment the host
has seen it finish.

Python's cyclic garbage collector is paused for the length of the loop: a
full collection over a large heap stops the host for tens of milliseconds,
during which no iteration is enqueued and no request admitted.  The loop
itself creates no reference cycles, so reference counting frees what it
allocates.
"""
from __future__ import annotations

import gc
import time
from collections import deque


def serve(pool, chains, arrivals, iterations: int = 4, on_result=None, clock=time.perf_counter,
          idle_sleep: float = 2e-4):
    """Runs the request stream ``chains[i]`` arriving at ``arrivals[i]``
    seconds (non-decreasing) after the start and returns one record per
    request: arrival, admission and finish times (s), latency (s) and the
    chain outcome of ``rlgl_pool_result``; ``blocked`` says whether the request
    once waited at the head of the queue because no slot or arena block was
    free.  ``on_result(i, outcome, pi)``
    is called with the device pi_hat before the slot is released."""
    if any(b < a for a, b in zip(arrivals, arrivals[1:])):
        raise ValueError("arrival times must be non-decreasing")
    collecting = gc.isenabled()
    gc.disable()
    try:
        return _serve(pool, chains, arrivals, iterations, on_result, clock, idle_sleep)
    finally:
        if collecting:
            gc.enable()


def _serve(pool, chains, arrivals, iterations, on_result, clock, idle_sleep):
    n = len(chains)
    start = clock()
    nxt = 0
    queue: deque[int] = deque()
    slot_req: dict[int, int] = {}
    admitted = [0.0] * n
    blocked = [False] * n  # the request once found no free slot or arena block at the head of the queue
    out = [None] * n
    done = 0
    while done < n:
        # the iterations of the running chains go to the GPU first, and the
        # host admits new arrivals while they run
        if slot_req:
            pool.launch(iterations)
        now = clock() - start
        while nxt < n and arrivals[nxt] <= now:
            queue.append(nxt)
            nxt += 1
        while queue:
            i = queue[0]
            slot = pool.admit(chains[i])
            if slot is None:
                blocked[i] = True
                if not slot_req:
                    raise RuntimeError(f"request {i} does not fit an empty pool "
                                       f"(footprint {pool.footprint(chains[i].n, chains[i].nnz)} bytes)")
                break
            queue.popleft()
            slot_req[slot] = i
            admitted[i] = clock() - start
        if slot_req:
            pool.wait()
            for slot in pool.poll():
                i = slot_req.pop(slot)
                t = clock() - start
                res, pi = pool.result(slot)
                if on_result is not None:
                    on_result(i, res, pi)
                out[i] = dict(arrival=arrivals[i], admitted=admitted[i], finished=t, latency=t - arrivals[i],
                              blocked=blocked[i], **res)
                pool.release(slot)
                done += 1
        elif nxt < n:
            wait = arrivals[nxt] - (clock() - start)
            if wait > 0:
                time.sleep(min(wait, idle_sleep))
    return out

