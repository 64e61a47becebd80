"""Admissibility without dummy vertices (test infrastructure only).

Section 3 ("The algorithm") starts strategy improvement from sigma_init,
which sends every Even vertex to the sink; it is admissible unless Odd can
close a cycle with an odd largest priority through its own vertices only.
The paper's simple remedy inserts dummy Even vertices (oracle/orc.c,
preprocess).  This module takes the other road: remove the part of the game
that Odd wins on its own, then run Algorithm 1 on the rest unchanged.

  X  the vertices from which Odd can avoid every Even vertex forever: the
     greatest set of Odd vertices each with a successor in the set
  R  the vertices of X from which Odd, moving inside X, reaches a cycle
     whose largest priority is odd (a one-player parity game on X); found by
     peeling strongly connected components: a component (with at least one
     edge) whose largest priority is odd lies in R; one whose largest is even
     loses that vertex and is decomposed again; then everything in X that
     reaches those components inside X
  A  Odd's attractor of R in the whole game (Odd vertices with a successor
     in A, Even vertices with all successors in A)

Odd wins A.  G' = G minus A is a trap for Odd: its Odd vertices keep all
their edges and its Even vertices at least one (else they would be in A).
Every cycle of Odd vertices in G' lies in X minus R, so its largest priority
is even: sigma_init is admissible in G', and Algorithm 1 runs on G' with no
preprocessing.  W_Odd = A plus W_Odd(G'), W_Even = W_Even(G').

Parity pins: tests/test_oracle_odd_region.py (winners equal Zielonka's and
the dummy path's; R against brute-force cycle enumeration on tiny games;
the attractor's closure; G' admissible).
"""
from __future__ import annotations

import sys

import numpy as np

from . import orc


def _rows(game):
    off = np.asarray(game["offsets"], np.int64)
    tgt = np.asarray(game["targets"], np.int64)
    return off, tgt


def odd_avoid_set(game) -> np.ndarray:
    """X: greatest fixpoint of {v in V_Odd : some successor in X}."""
    off, tgt = _rows(game)
    n = int(game["n"])
    own = np.asarray(game["owner"])
    X = own == 1
    while True:
        src = np.repeat(np.arange(n), np.diff(off))
        has = np.zeros(n, bool)
        np.logical_or.at(has, src, X[tgt])
        nx = X & has
        if (nx == X).all():
            return X
        X = nx


def _sccs(vertices, succ):
    """Strongly connected components of the subgraph induced by `vertices`
    (succ(v) lists v's successors inside it); iterative Tarjan."""
    index, low = {}, {}
    on, stack, out = set(), [], []
    counter = 0
    for root in vertices:
        if root in index:
            continue
        work = [(root, iter(succ(root)))]
        index[root] = low[root] = counter
        counter += 1
        stack.append(root)
        on.add(root)
        while work:
            v, it = work[-1]
            advanced = False
            for w in it:
                if w not in index:
                    index[w] = low[w] = counter
                    counter += 1
                    stack.append(w)
                    on.add(w)
                    work.append((w, iter(succ(w))))
                    advanced = True
                    break
                if w in on:
                    low[v] = min(low[v], index[w])
            if advanced:
                continue
            work.pop()
            if work:
                u = work[-1][0]
                low[u] = min(low[u], low[v])
            if low[v] == index[v]:
                comp = []
                while True:
                    w = stack.pop()
                    on.discard(w)
                    comp.append(w)
                    if w == v:
                        break
                out.append(comp)
    return out


def odd_cycle_region(game, X) -> np.ndarray:
    """R: the vertices of X from which Odd reaches, inside X, a cycle whose
    largest priority is odd."""
    off, tgt = _rows(game)
    n = int(game["n"])
    pri = np.asarray(game["pri"], np.int64)
    seed = np.zeros(n, bool)
    work = [list(np.flatnonzero(X))]
    while work:
        V = work.pop()
        member = set(V)

        def succ(v, member=member):
            return [int(w) for w in tgt[off[v]:off[v + 1]] if int(w) in member]

        for comp in _sccs(V, succ):
            if len(comp) == 1 and comp[0] not in succ(comp[0]):
                continue   # no edge inside: on no cycle
            top = max(comp, key=lambda v: pri[v])
            if pri[top] % 2 == 1:
                seed[comp] = True
            else:
                work.append([v for v in comp if v != top])
    # everything in X that reaches the seed inside X
    R = seed.copy()
    src = np.repeat(np.arange(n), np.diff(off))
    inside = X[src] & X[tgt]
    while True:
        hit = np.zeros(n, bool)
        np.logical_or.at(hit, src[inside], R[tgt[inside]])
        nr = R | (hit & X)
        if (nr == R).all():
            return R
        R = nr


def odd_attractor(game, target) -> np.ndarray:
    """Odd's attractor of `target`: repeatedly add Odd vertices with a
    successor in it and Even vertices with every successor in it."""
    off, tgt = _rows(game)
    n = int(game["n"])
    own = np.asarray(game["owner"])
    src = np.repeat(np.arange(n), np.diff(off))
    A = np.asarray(target, bool).copy()
    deg = np.diff(off)
    while True:
        cnt = np.zeros(n, np.int64)
        np.add.at(cnt, src, A[tgt].astype(np.int64))
        na = A | ((own == 1) & (cnt > 0)) | ((own == 0) & (cnt == deg))
        if (na == A).all():
            return A
        A = na


def subgame(game, keep):
    """The game on the vertices `keep` (edges inside only, rows in their
    order), with the original id of each kept vertex."""
    off, tgt = _rows(game)
    n = int(game["n"])
    ids = np.flatnonzero(keep)
    new = np.full(n, -1, np.int64)
    new[ids] = np.arange(ids.size)
    rows, deg = [], []
    for v in ids:
        r = [int(new[w]) for w in tgt[off[v]:off[v + 1]] if keep[w]]
        rows.append(r)
        deg.append(len(r))
    o = np.zeros(ids.size + 1, np.int64)
    np.cumsum(deg, out=o[1:])
    t = np.array([x for r in rows for x in r], np.int32)
    sub = {"n": int(ids.size), "m": int(t.size), "offsets": o, "targets": t,
           "owner": np.asarray(game["owner"])[ids].astype(np.uint8),
           "pri": np.asarray(game["pri"])[ids].astype(np.int32)}
    return sub, ids


def solve(game, counts: bool = None) -> dict:
    """Algorithm 1 on the game without Odd's own winning part A: winners
    of the whole game, and sigma*, tau* of the vertices outside A (in the
    original ids; PG_SINK (-1) for the vertices of A in both), counts of
    the run on G'.  Valuations as sets of priorities (ranks) when the
    game's priorities are pairwise distinct, else as count vectors (section
    3, "Valuations"); `counts` forces the choice."""
    n = int(game["n"])
    if counts is None:
        counts = np.unique(np.asarray(game["pri"])).size < n
    X = odd_avoid_set(game)
    R = odd_cycle_region(game, X)
    A = odd_attractor(game, R)
    keep = ~A
    winner = np.ones(n, np.uint8)
    sigma = np.full(n, -1, np.int32)
    tau = np.full(n, -1, np.int32)
    out = {"X": X, "R": R, "A": A, "n_removed": int(A.sum()),
           "n_major": 0, "n_valuations": 0, "n_odd_switches": 0,
           "n_even_switches": 0, "status": 0}
    if keep.any():
        sub, ids = subgame(game, keep)
        ref = (orc.dense_solve(sub, preprocess_game=False) if counts
               else orc.solve(sub, preprocess_game=False))
        out["status"] = ref["status"]
        winner[ids] = ref["winner"]
        s, t = ref["sigma"], ref["tau"]
        sigma[ids] = np.where(s >= 0, ids[np.maximum(s, 0)], -1)
        tau[ids] = np.where(t >= 0, ids[np.maximum(t, 0)], -1)
        for k in ("n_major", "n_valuations", "n_odd_switches",
                  "n_even_switches"):
            out[k] = ref[k]
        out["sub"] = sub
        out["ids"] = ids
    out.update(winner=winner, sigma=sigma, tau=tau)
    return out


if __name__ == "__main__":
    sys.exit(0)
