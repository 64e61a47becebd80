"""Seeded synthetic parity games.

This module only draws inputs.  It holds none of the solver's arithmetic and
imports nothing from the solver or from the oracle, so both sides can take
their inputs from it.

A game is returned as a dict of numpy arrays in CSR form::

    n, m       vertex and edge counts
    offsets    int64[n+1] (or int32 with ``offsets_dtype=np.int32``)
    targets    int32[m]   successor ids, each row sorted ascending
    owner      uint8[n]   0 = Even, 1 = Odd
    pri        int32[n]   priorities (pairwise distinct except in
                          ``few_priorities_game``)

The game model is the tuple (V, V_Even, V_Odd, E, pri) of the paper's
preliminaries (section 2): every vertex has at least one outgoing edge.

Recipes (all draws from ``numpy.random.Generator(PCG64(seed))``):

* ``random_game`` -- owner ~ Bernoulli(1/2); pri = permutation(n); each row
  draws its out-degree uniformly from [dmin, dmax] (capped at n-1), then that
  many distinct successors uniformly from V minus the vertex itself (a draw t in
  [0, n-1) maps to t+1 when t >= v).  No self-loops, no duplicate edges.
* ``chain_game`` -- vertex i has the edge i -> i+1 (the last vertex wraps to
  0) and, with probability 1/2, one back edge i -> j with j uniform in [0, i)
  for i >= 1.  The wrap vertex never takes j = 0 (it would duplicate the wrap
  edge); it draws j from [1, n-1) instead.  Owners alternate in runs whose
  lengths are uniform in [1, 64], starting with a random owner; pri is a
  random permutation.
* ``few_priorities_game`` -- the graph and owners of ``random_game`` with the
  same seed; priorities drawn uniformly from [0, d) by a second, independent
  stream (``PCG64([seed, 1])``), so they repeat: the regime of the paper's
  experiments, whose games have 2 to 4 distinct priorities.
* ``odd_cycles_game`` -- structure for Odd's own cycles: about n/3
  vertices in disjoint Odd cycles of lengths uniform in [1, 6] (length 1 is
  a self-loop), each cycle of length >= 3 with probability 1/2 given one
  chord between two members that are not already joined; about n/3 Odd
  tail vertices, each with one edge to a uniformly drawn earlier vertex
  (cycle or tail) and, with probability 1/4, a second edge to a uniform
  Even vertex; the rest Even, each with 1 to 3 distinct uniform
  successors.  pri = permutation(n), or uniform in [0, d) when d > 0.  Vertex
  ids are shuffled by a uniform permutation at the end.
* ``mixed_batch`` -- the batched workload: game g uses seed base+g,
  n_g = round(exp(U(ln nmin, ln nmax))) and a random game with out-degree
  uniform in [2, 8] and int32 offsets.
"""
from __future__ import annotations

import numpy as np

__all__ = ["random_game", "chain_game", "few_priorities_game", "mixed_batch",
           "odd_cycles_game", "config_game", "CONFIG_SEED_BASE"]

CONFIG_SEED_BASE = 1000


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _rows_to_csr(deg: np.ndarray, flat: np.ndarray, offsets_dtype) -> tuple:
    offsets = np.zeros(deg.shape[0] + 1, dtype=np.int64)
    np.cumsum(deg, out=offsets[1:])
    return offsets.astype(offsets_dtype, copy=False), flat.astype(np.int32)


def random_game(n: int, dmin: int, dmax: int, seed: int,
                offsets_dtype=np.int64) -> dict:
    """Random game with distinct priorities and uniform successors."""
    if n < 2:
        raise ValueError("random_game needs n >= 2 (no self-loops allowed)")
    rng = _rng(seed)
    owner = rng.integers(0, 2, size=n, dtype=np.uint8)
    pri = rng.permutation(n).astype(np.int32)
    hi = min(dmax, n - 1)
    lo = min(dmin, hi)
    deg = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    if n <= 64:
        rows = []
        for v in range(n):
            t = rng.choice(n - 1, size=int(deg[v]), replace=False)
            t = np.where(t >= v, t + 1, t)
            rows.append(np.sort(t))
        flat = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    else:
        # draw hi candidates per row; only the first deg[v] of them are used.
        # Rows whose used prefix repeats a value are redrawn until none does.
        cand = rng.integers(0, n - 1, size=(n, hi), dtype=np.int64)
        col = np.arange(hi)[None, :]
        while True:
            used = col < deg[:, None]
            big = np.int64(n) + col  # unused slots get distinct sentinels
            work = np.where(used, cand, big)
            srt = np.sort(work, axis=1)
            dup = (srt[:, 1:] == srt[:, :-1]).any(axis=1)
            bad = np.flatnonzero(dup)
            if bad.size == 0:
                break
            cand[bad] = rng.integers(0, n - 1, size=(bad.size, hi),
                                     dtype=np.int64)
        v = np.arange(n, dtype=np.int64)[:, None]
        mapped = np.where(cand >= v, cand + 1, cand)
        mapped = np.where(col < deg[:, None], mapped, np.int64(1) << 40)
        mapped.sort(axis=1)
        flat = mapped[col < deg[:, None]]
    offsets, targets = _rows_to_csr(deg, flat, offsets_dtype)
    return {"n": n, "m": int(deg.sum()), "offsets": offsets,
            "targets": targets, "owner": owner, "pri": pri}


def chain_game(n: int, seed: int, offsets_dtype=np.int64) -> dict:
    """Long-chain stress game (one forward chain plus random back edges)."""
    if n < 3:
        raise ValueError("chain_game needs n >= 3")
    rng = _rng(seed)
    # owners in runs of uniform length [1, 64]
    first = int(rng.integers(0, 2))
    runs = []
    total = 0
    while total < n:
        r = int(rng.integers(1, 65))
        runs.append(r)
        total += r
    runs = np.array(runs, dtype=np.int64)
    run_owner = (first + np.arange(runs.size)) % 2
    owner = np.repeat(run_owner, runs)[:n].astype(np.uint8)
    pri = rng.permutation(n).astype(np.int32)
    has_back = rng.random(n) < 0.5
    has_back[0] = False
    u = rng.random(n)
    i = np.arange(n, dtype=np.int64)
    j = np.floor(u * i).astype(np.int64)  # uniform in [0, i)
    j = np.minimum(j, np.maximum(i - 1, 0))
    # the wrap vertex draws from [1, n-1) so it never repeats its edge to 0
    last = n - 1
    if has_back[last]:
        j[last] = 1 + int(np.floor(u[last] * (n - 2)))
        j[last] = min(j[last], n - 2)
    fwd = (i + 1) % n
    deg = 1 + has_back.astype(np.int64)
    a = np.where(has_back, np.minimum(fwd, j), fwd)
    b = np.where(has_back, np.maximum(fwd, j), -1)
    flat = np.stack([a, b], axis=1)[np.stack([np.ones(n, bool), has_back],
                                             axis=1)]
    offsets, targets = _rows_to_csr(deg, flat, offsets_dtype)
    return {"n": n, "m": int(deg.sum()), "offsets": offsets,
            "targets": targets, "owner": owner, "pri": pri}


def few_priorities_game(n: int, dmin: int, dmax: int, d: int, seed: int,
                        offsets_dtype=np.int64) -> dict:
    """Random game whose priorities take only d values (they repeat)."""
    g = random_game(n, dmin, dmax, seed, offsets_dtype)
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    g["pri"] = rng.integers(0, d, size=n).astype(np.int32)
    return g


def odd_cycles_game(n: int, seed: int, d: int = 0,
                    offsets_dtype=np.int64) -> dict:
    """Odd cycles (some with chords), Odd tails into them, Even rest."""
    if n < 9:
        raise ValueError("odd_cycles_game needs n >= 9")
    rng = _rng(seed)
    rows = []
    owner = []
    n_cyc = n // 3
    while len(rows) < n_cyc:
        L = int(rng.integers(1, 7))
        base = len(rows)
        mem = [[base + (i + 1) % L] for i in range(L)]
        if L >= 3 and rng.random() < 0.5:
            a, b = (int(x) for x in rng.integers(0, L, size=2))
            if b != (a + 1) % L:
                mem[a].append(base + b)
        rows.extend(mem)
        owner.extend([1] * L)
    n_cyc = len(rows)
    n_tail = min(n // 3, n - n_cyc - 1)
    n_even = n - n_cyc - n_tail
    first_even = n_cyc + n_tail
    for t in range(n_tail):
        v = n_cyc + t
        r = [int(rng.integers(0, v))]
        if rng.random() < 0.25:
            r.append(first_even + int(rng.integers(0, n_even)))
        rows.append(r)
        owner.append(1)
    for _ in range(n_even):
        k = int(rng.integers(1, 4))
        rows.append([int(x) for x in rng.choice(n, size=k, replace=False)])
        owner.append(0)
    # shuffle ids: new id of old vertex i is p[i]
    p = rng.permutation(n)
    inv = np.argsort(p)
    rows = [sorted(int(p[w]) for w in rows[int(inv[v])]) for v in range(n)]
    owner = np.asarray(owner, np.uint8)[inv]
    if d > 0:
        pri = rng.integers(0, d, size=n).astype(np.int32)
    else:
        pri = rng.permutation(n).astype(np.int32)
    deg = np.array([len(r) for r in rows], np.int64)
    flat = np.array([w for r in rows for w in r], np.int64)
    offsets, targets = _rows_to_csr(deg, flat, offsets_dtype)
    return {"n": n, "m": int(deg.sum()), "offsets": offsets,
            "targets": targets, "owner": owner, "pri": pri}


def mixed_batch(count: int, seed_base: int, nmin: int = 1000,
                nmax: int = 200000, dmin: int = 2, dmax: int = 8) -> list:
    """Games of log-uniform sizes for the batched workload."""
    games = []
    for g in range(count):
        rng = _rng(seed_base + g)
        n_g = int(round(float(np.exp(rng.uniform(np.log(nmin),
                                                 np.log(nmax))))))
        n_g = max(n_g, 2)
        sub_seed = int(rng.integers(0, 2**62))
        games.append(random_game(n_g, dmin, dmax, sub_seed,
                                 offsets_dtype=np.int32))
    return games


def config_game(config: int, k: int = 0) -> dict:
    """The workloads by index: 0 small random, 1 1M random, 2 10M random,
    3 8M long chain, 5 10M random with 4 repeated priorities (the paper's
    regime), 6 1M random with 4 priorities.  Offsets are int64 for the
    10M-vertex games and int32 for the others."""
    seed = CONFIG_SEED_BASE * config + k
    i32 = np.int32
    if config == 5:
        return few_priorities_game(10_000_000, 2, 5, 4, seed)
    if config == 6:
        return few_priorities_game(1_000_000, 2, 10, 4, seed, i32)
    if config == 0:
        return random_game(1000, 2, 5, seed, i32)
    if config == 1:
        return random_game(1_000_000, 2, 10, seed, i32)
    if config == 2:
        return random_game(10_000_000, 2, 5, seed)
    if config == 3:
        return chain_game(8_000_000, seed, i32)
    raise ValueError(f"unknown config {config}")
