"""Continuous-batching request loop over the batch C ABI.

Requests (games) arrive over time.  The loop hands every arrived game to the
batch, which admits queued games first come first served as arena space
(the HBM-footprint budget given at creation) frees up, advances every game in
the arena by one best-response iteration per step, and reports finished
games, whose latency is completion time minus arrival time.  Games that
arrive while others are being solved join the next step that has room for
them: their work overlaps with the games already on the device.
"""
from __future__ import annotations

import time

import numpy as np

from .pg import Batch


def serve(games, arrivals, max_vertices: int, max_edges: int,
          keep_results: bool = True, clock=time.perf_counter) -> dict:
    """Solves `games` arriving at `arrivals` (seconds from the start, sorted).

    Returns {"results": {i: result dict}, "latency": [...], "arrival",
    "completion", "makespan", "steps"}.
    """
    order = np.argsort(np.asarray(arrivals), kind="stable")
    arrivals = np.asarray(arrivals, dtype=np.float64)
    n = len(games)
    completion = np.full(n, np.nan)
    results = {}
    ticket_of = {}
    nxt = 0
    steps = 0
    with Batch(max_vertices, max_edges) as b:
        t0 = clock()
        done = 0
        while done < n:
            now = clock() - t0
            # admit every request that has arrived by now
            while nxt < n and arrivals[order[nxt]] <= now:
                i = int(order[nxt])
                ticket_of[b.submit(games[i])] = i
                nxt += 1
            info_live, queued, _ = b.step()
            steps += 1
            for t in b.finished():
                r = b.poll(t)
                i = ticket_of.pop(t)
                completion[i] = clock() - t0
                if keep_results:
                    results[i] = r
                done += 1
            if info_live == 0 and queued == 0 and nxt < n and done < n:
                # idle until the next arrival
                wait = arrivals[order[nxt]] - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
        makespan = clock() - t0
    latency = completion - arrivals
    return {"results": results, "latency": latency, "arrival": arrivals,
            "completion": completion, "makespan": makespan, "steps": steps}


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process with `rate` per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
