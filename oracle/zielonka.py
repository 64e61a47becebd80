"""Zielonka's recursive algorithm (test infrastructure only).

An independent solver used to pin the winning regions that strategy
improvement reports.  It is the textbook recursive algorithm (the one the
paper compares against through PGSolver, section 6), written from its
definition: take the largest priority p of the subgame, the player i = p mod 2
that likes it, i's attractor A of the vertices of priority p; solve the game
without A; if the opponent wins nothing there, i wins the whole subgame,
otherwise remove the opponent's attractor to its winning part and recurse.

It works on the original game (no sink, no dummies).  Returns winner[v] =
0 for W_Even, 1 for W_Odd.
"""
from __future__ import annotations

import sys

import numpy as np


def _attractor(player, target, alive, owner, succs, preds):
    """Vertices of ``alive`` from which ``player`` forces a visit to
    ``target`` (target must be a subset of alive)."""
    attr = set(target)
    count = {}
    queue = list(target)
    while queue:
        u = queue.pop()
        for v in preds[u]:
            if v not in alive or v in attr:
                continue
            if owner[v] == player:
                attr.add(v)
                queue.append(v)
            else:
                if v not in count:
                    count[v] = sum(1 for w in succs[v] if w in alive)
                count[v] -= 1
                if count[v] == 0:
                    attr.add(v)
                    queue.append(v)
    return attr


def _solve(alive, owner, pri, succs, preds):
    if not alive:
        return set(), set()
    p = max(pri[v] for v in alive)
    i = p % 2
    top = {v for v in alive if pri[v] == p}
    a = _attractor(i, top, alive, owner, succs, preds)
    w = _solve(alive - a, owner, pri, succs, preds)
    if not w[1 - i]:
        out = [set(), set()]
        out[i] = set(alive)
        return out[0], out[1]
    b = _attractor(1 - i, w[1 - i], alive, owner, succs, preds)
    w2 = _solve(alive - b, owner, pri, succs, preds)
    out = [set(), set()]
    out[i] = set(w2[i])
    out[1 - i] = set(w2[1 - i]) | b
    return out[0], out[1]


def zielonka(game: dict) -> np.ndarray:
    n = int(game["n"])
    off = np.asarray(game["offsets"], np.int64)
    tgt = np.asarray(game["targets"], np.int64)
    owner = [int(x) for x in game["owner"]]
    pri = [int(x) for x in game["pri"]]
    succs = [tgt[off[v]:off[v + 1]].tolist() for v in range(n)]
    preds = [[] for _ in range(n)]
    for v in range(n):
        for u in succs[v]:
            preds[u].append(v)
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 4 * n + 100))
    try:
        w_even, w_odd = _solve(set(range(n)), owner, pri, succs, preds)
    finally:
        sys.setrecursionlimit(old)
    assert not (w_even & w_odd) and len(w_even) + len(w_odd) == n
    win = np.ones(n, dtype=np.uint8)
    for v in w_even:
        win[v] = 0
    return win
