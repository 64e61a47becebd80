"""Continuous-batching request loop over the batch C ABI.

Requests (games) arrive over time.  A submitter thread hands every game to
the batch when it arrives (validation and preprocessing run on the batch's
submission stream, pg_batch_submit), while the loop advances every game in
the arena by one best-response iteration per step (pg_batch_step, which
admits queued games first come first served as arena space -- the
HBM-footprint budget given at creation -- frees up) and collects finished
games, whose latency is completion time minus arrival time.  Games that
arrive while others are being solved join the next step that has room for
them: their preprocessing and then their work overlap with the games
already on the device.
"""
from __future__ import annotations

import threading
import time

import numpy as np

from .pg import Batch


def serve(games, arrivals, max_vertices: int, max_edges: int,
          keep_results: bool = True, clock=time.perf_counter,
          submit_thread: bool = False) -> dict:
    """Solves `games` arriving at `arrivals` (seconds from the start).

    Without `submit_thread` (default) the loop submits the games that have
    arrived between steps, all in one pg_batch_submit_many call, so each
    step sees every game that arrived before it; with it submissions run one
    by one on a thread of their own, overlapping the
    steps (lower latency below saturation, fewer games per second near it:
    the steps then hold fewer games each).
    Returns {"results": {i: result dict}, "latency": [...], "arrival",
    "completion", "makespan", "steps"}.
    """
    order = np.argsort(np.asarray(arrivals), kind="stable")
    arrivals = np.asarray(arrivals, dtype=np.float64)
    n = len(games)
    completion = np.full(n, np.nan)
    results = {}
    ticket_of = {}
    lock = threading.Lock()
    submitted = threading.Event()   # set after every submission
    state = {"count": 0, "error": None}
    steps = 0
    with Batch(max_vertices, max_edges) as b:
        t0 = clock()

        def submit(i):
            t = b.submit(games[i])
            with lock:
                ticket_of[t] = i
                state["count"] += 1
            submitted.set()

        def submitter():
            try:
                for k in range(n):
                    i = int(order[k])
                    wait = arrivals[i] - (clock() - t0)
                    if wait > 0:
                        time.sleep(wait)
                    submit(i)
            except Exception as e:   # reported by the loop
                state["error"] = e
                submitted.set()

        th = None
        nxt = 0
        if submit_thread:
            th = threading.Thread(target=submitter, daemon=True)
            th.start()
        done = 0
        try:
            while done < n:
                if state["error"] is not None:
                    raise state["error"]
                if th is None:
                    # admit every request that has arrived by now, in one
                    # call (their preprocessing runs over their union)
                    now = clock() - t0
                    arrived = []
                    while nxt < n and arrivals[order[nxt]] <= now:
                        arrived.append(int(order[nxt]))
                        nxt += 1
                    if arrived:
                        res = b.submit_many([games[i] for i in arrived])
                        for i, t in zip(arrived, res):
                            if isinstance(t, Exception):
                                raise t
                            ticket_of[t] = i
                info_live, queued, _ = b.step()
                steps += 1
                fin = b.finished()
                rs = b.poll_many(fin) if fin else []
                now = clock() - t0
                for t, r in zip(fin, rs):
                    while True:
                        with lock:
                            i = ticket_of.pop(t, None)
                        if i is not None:
                            break
                        time.sleep(1e-5)   # the submitter is storing it
                    completion[i] = now
                    if keep_results:
                        results[i] = r
                    done += 1
                if info_live == 0 and queued == 0 and done < n:
                    # idle until the next submission
                    if th is None:
                        if nxt < n:
                            wait = arrivals[order[nxt]] - (clock() - t0)
                            if wait > 0:
                                time.sleep(min(wait, 0.05))
                    else:
                        submitted.wait(0.05)
                        submitted.clear()
        finally:
            if th is not None:
                th.join()
        makespan = clock() - t0
    latency = completion - arrivals
    return {"results": results, "latency": latency, "arrival": arrivals,
            "completion": completion, "makespan": makespan, "steps": steps}


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process with `rate` per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
