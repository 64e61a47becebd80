"""Pins of oracle/odd_region.py (admissibility by removing Odd's own
winning part instead of inserting dummies): its winners equal Zielonka's and
the dummy path's; R equals a brute-force enumeration of the odd-max cycles
of X on tiny games; A is closed like an attractor; the game it leaves is
admissible (no cycle of Odd vertices with an odd largest priority)."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import odd_region, orc
from oracle.zielonka import zielonka
from paper_1705_02313_amd import synth


def _games():
    out = []
    for seed in range(40):
        n = [3, 5, 8, 12][seed % 4]
        out.append(synth.random_game(n, 1, min(4, n - 1), 6000 + seed))
    for seed in range(12):
        out.append(synth.random_game([50, 300, 2000][seed % 3], 2, 5,
                                     6100 + seed))
    out.append(synth.chain_game(500, 6200))
    out.append(synth.chain_game(64, 6201))
    # Odd cycles with and without odd maxima, chords, tails (R short of X)
    for seed in range(8):
        out.append(synth.odd_cycles_game([9, 14, 60, 400][seed % 4],
                                         6400 + seed, d=3 if seed >= 6 else 0))
    return out


def _succ(game):
    off = np.asarray(game["offsets"], np.int64)
    tgt = np.asarray(game["targets"])
    return [list(map(int, tgt[off[v]:off[v + 1]]))
            for v in range(int(game["n"]))]


@pytest.mark.parametrize("i", range(62))
def test_winners_equal_zielonka_and_the_dummy_path(i):
    g = _games()[i]
    r = odd_region.solve(g)
    assert r["status"] == 0
    z = zielonka(g)
    np.testing.assert_array_equal(r["winner"], z)
    np.testing.assert_array_equal(r["winner"], orc.solve(g)["winner"])


def _brute_region(game, X):
    """Vertices of X that reach, inside X, a simple cycle of X with an odd
    largest priority (every simple cycle enumerated)."""
    succ = _succ(game)
    pri = np.asarray(game["pri"])
    xs = [v for v in range(int(game["n"])) if X[v]]
    on_odd = set()
    # simple cycles: start at their least vertex, extend by larger ones
    for s in xs:
        stack = [(s, [s])]
        while stack:
            v, path = stack.pop()
            for w in succ[v]:
                if not X[w]:
                    continue
                if w == s:
                    if max(pri[u] for u in path) % 2 == 1:
                        on_odd.update(path)
                elif w > s and w not in path:
                    stack.append((w, path + [w]))
    R = set(on_odd)
    changed = True
    while changed:
        changed = False
        for v in xs:
            if v not in R and any(X[w] and w in R for w in succ[v]):
                R.add(v)
                changed = True
    return R


@pytest.mark.parametrize("seed", range(60))
def test_region_against_cycle_enumeration(seed):
    n = [4, 6, 8, 10, 12][seed % 5]
    g = synth.random_game(n, 1, min(4, n - 1), 6300 + seed)
    # more Odd vertices: more of X
    g["owner"] = (np.random.Generator(np.random.PCG64(seed)).random(n)
                  < 0.8).astype(np.uint8)
    X = odd_region.odd_avoid_set(g)
    R = odd_region.odd_cycle_region(g, X)
    assert set(np.flatnonzero(R)) == _brute_region(g, X)
    np.testing.assert_array_equal(odd_region.solve(g)["winner"], zielonka(g))


@pytest.mark.parametrize("seed", range(24))
def test_region_against_cycle_enumeration_on_cycle_soups(seed):
    g = synth.odd_cycles_game([9, 12, 15][seed % 3], 6500 + seed,
                              d=4 if seed % 2 else 0)
    X = odd_region.odd_avoid_set(g)
    R = odd_region.odd_cycle_region(g, X)
    assert set(np.flatnonzero(R)) == _brute_region(g, X)
    np.testing.assert_array_equal(odd_region.solve(g)["winner"], zielonka(g))


def test_self_loops_and_even_cycles():
    # 0 (Odd, pri 3) -> 0 self loop: Odd wins alone
    # 1 (Odd, pri 2) <-> 2 (Odd, pri 0): an even cycle of Odd vertices only
    # 3 (Even, pri 1) -> 1 or 0: Even avoids 0
    g = {"n": 4, "m": 5, "offsets": np.array([0, 1, 2, 3, 5]),
         "targets": np.array([0, 2, 1, 0, 1], np.int32),
         "owner": np.array([1, 1, 1, 0], np.uint8),
         "pri": np.array([3, 2, 0, 1], np.int32)}
    X = odd_region.odd_avoid_set(g)
    assert X.tolist() == [True, True, True, False]
    R = odd_region.odd_cycle_region(g, X)
    assert R.tolist() == [True, False, False, False]
    A = odd_region.odd_attractor(g, R)
    assert A.tolist() == [True, False, False, False]
    r = odd_region.solve(g)
    assert r["winner"].tolist() == zielonka(g).tolist() == [1, 0, 0, 0]
    assert r["sigma"][3] == 1 and r["sigma"][0] == -1 and r["tau"][0] == -1


@pytest.mark.parametrize("i", range(62))
def test_attractor_closure_and_admissible_rest(i):
    g = _games()[i]
    r = odd_region.solve(g)
    A = r["A"]
    succ = _succ(g)
    own = np.asarray(g["owner"])
    for v in range(int(g["n"])):
        if A[v]:
            continue
        if own[v] == 1:   # an Odd vertex outside A has no edge into A
            assert not any(A[w] for w in succ[v])
        else:             # an Even vertex outside A keeps an edge outside
            assert any(not A[w] for w in succ[v])
    if "sub" in r:
        sub = r["sub"]
        Xs = odd_region.odd_avoid_set(sub)
        assert not odd_region.odd_cycle_region(sub, Xs).any()


def test_nothing_removed_without_odd_cycles():
    g = synth.random_game(400, 2, 5, 6400)
    g["owner"] = np.zeros(400, np.uint8)   # Even only: X is empty
    r = odd_region.solve(g)
    assert r["n_removed"] == 0
    ref = orc.solve(g, preprocess_game=False)
    np.testing.assert_array_equal(r["sigma"], ref["sigma"])
    assert r["n_valuations"] == ref["n_valuations"]
