"""Pins of the count-valuation oracle (oracle/orc_dense.c) for games whose
priorities repeat.  Nothing here touches the GPU.  Each test names what it
pins:
  * the Maxdiff order on hand-made count vectors (section 3, "Valuations");
  * valuations and cycle parity against the literal oracle's backward tree
    (section 3; section 5's sequential algorithm);
  * whole runs of Algorithm 1 against the literal oracle, valuation counts
    and strategies included (section 4);
  * winners against Zielonka's algorithm (positional determinacy, Theorem 1);
  * best responses against brute force over every tau (section 3, "Best
    responses");
  * with distinct priorities, the count path against the rank path of the
    C oracle on the same modified game (the two representations order the
    vertices alike);
  * the preprocessing reading of this path: the same X, X' and redirected
    edges as the rank path, dummies at priority 0, originals raised by 2,
    winners kept;
  * the best-response variants of section 6: Bellman-Ford labels and round
    counts against the literal oracle's Bellman-Ford and against SI's best
    responses; SI-Reset and Bellman-Ford leave the outer loop unchanged.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import literal as L
from oracle import orc
from oracle.zielonka import zielonka
from paper_1705_02313_amd import synth


def _few(seed, nmin=4, nmax=40, dmax=4):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(nmin, nmax + 1))
    d = int(rng.integers(2, dmax + 1))
    return synth.few_priorities_game(n, 1, int(rng.integers(2, 5)), d,
                                     5000 + seed)


# ---------------------------------------------------------------------------
# the order (section 3)
# ---------------------------------------------------------------------------
def test_dense_maxdiff_hand_cases():
    # columns: priorities 1 and 2 (values); rows: vertices 0..3, row 4 = sink
    values = np.array([1, 2], np.int32)
    counts = np.array([[0, 1],     # v0: one 2
                       [1, 1],     # v1: one 1, one 2
                       [0, 2],     # v2: two 2s
                       [0, 1],     # v3: same as v0
                       [0, 0]],    # sink
                      np.int32)
    top = np.array([0, 0, 0, 0], np.uint8)
    c = lambda a, b: orc.dense_compare(counts, top, values, a, b)
    # Maxdiff(v0, v1) = 1 (odd): fewer 1s is the larger valuation
    assert c(0, 1) == 1 and c(1, 0) == -1
    # Maxdiff(v2, v0) = 2 (even): more 2s is the larger valuation
    assert c(2, 0) == 1 and c(0, 2) == -1
    # Maxdiff(v2, v1) = 2 decides before priority 1 is looked at
    assert c(2, 1) == 1
    # equal vectors of different vertices, and the sink's zero vector
    assert c(0, 3) == 0 and c(4, 4) == 0
    assert c(0, 4) == 1          # one even 2 beats the empty path
    top2 = np.array([1, 0, 0, 1], np.uint8)
    c2 = lambda a, b: orc.dense_compare(counts, top2, values, a, b)
    assert c2(0, 2) == 1 and c2(2, 0) == -1 and c2(0, 3) == 0
    assert c2(0, 4) == 1 and c2(4, 3) == -1


@pytest.mark.parametrize("seed", range(10))
def test_dense_compare_is_a_total_preorder(seed):
    rng = np.random.default_rng(seed)
    n, d = 30, 4
    values = np.sort(rng.choice(10, size=d, replace=False)).astype(np.int32)
    counts = rng.integers(0, 3, size=(n + 1, d)).astype(np.int32)
    counts[n] = 0
    top = (rng.random(n) < 0.2).astype(np.uint8)
    counts[:n][top == 1] = 0
    cmp = np.array([[orc.dense_compare(counts, top, values, a, b)
                     for b in range(n + 1)] for a in range(n + 1)])
    np.testing.assert_array_equal(cmp, -cmp.T)
    for a in range(n + 1):
        for b in range(n + 1):
            if cmp[a, b] <= 0:
                # transitivity through every c
                assert not np.any((cmp[b, :] <= 0) & (cmp[a, :] > 0))
    # the literal comparator agrees pair by pair
    vals = [L.TOP if v < n and top[v] else counts[v] for v in range(n + 1)]
    for a in range(n + 1):
        for b in range(n + 1):
            le = L.val_le(vals[a], vals[b], values)
            assert le == (cmp[a, b] <= 0)


# ---------------------------------------------------------------------------
# valuations (section 3) against the literal backward-tree oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(30))
def test_dense_valuation_matches_literal(seed):
    g = _few(seed)
    rng = np.random.default_rng(100 + seed)
    rows = L.rows_of(g)
    n = g["n"]
    sigma = [L.SINK if g["owner"][v] == 1 or rng.random() < 0.3
             else int(rng.choice(rows[v])) for v in range(n)]
    tau = [int(rng.choice(rows[v])) if g["owner"][v] == 1 else L.SINK
           for v in range(n)]
    succ = np.array([tau[v] if g["owner"][v] else sigma[v]
                     for v in range(n)], np.int32)
    counts, top, values, rc = orc.dense_valuation(succ, g["pri"])
    vals = L.Vals(g["pri"])
    lv, cycles = L.valuation(g, vals, sigma, tau)
    np.testing.assert_array_equal(values, vals.dom)
    for v in range(n):
        if lv[v] is L.TOP:
            assert top[v] == 1
            assert not counts[v].any()
        else:
            assert top[v] == 0
            np.testing.assert_array_equal(counts[v], lv[v])
    assert not counts[n].any()
    odd_cycle = any(not L.cycle_is_even(g, c) for c in cycles)
    assert rc == (orc.EINADMISSIBLE if odd_cycle else orc.OK)


# ---------------------------------------------------------------------------
# whole runs (section 4)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(40))
def test_dense_solve_matches_literal(seed):
    g = _few(seed)
    aug = orc.dense_preprocess(g)
    r = orc.dense_solve(g, trace=True)
    assert r["status"] == orc.OK
    lit = L.solve(aug, preprocess_game=False)
    np.testing.assert_array_equal(lit["winner"][:g["n"]], r["winner"])
    np.testing.assert_array_equal(lit["sigma"], r["sigma"])
    np.testing.assert_array_equal(lit["tau"], r["tau"])
    assert lit["n_major"] == r["n_major"]
    assert lit["n_valuations"] == r["n_valuations"]
    assert r["trace"].shape == (r["n_valuations"], 2)
    for v in range(aug["n"]):
        if lit["val"][v] is L.TOP:
            assert r["top"][v] == 1
        else:
            np.testing.assert_array_equal(r["counts"][v], lit["val"][v])


@pytest.mark.parametrize("seed", range(30))
def test_dense_winners_zielonka(seed):
    g = _few(seed, nmin=20, nmax=300, dmax=6)
    np.testing.assert_array_equal(orc.dense_solve(g)["winner"], zielonka(g))


def test_dense_winners_zielonka_larger():
    for seed, n, d in [(1, 3000, 2), (2, 3000, 3), (3, 2500, 4), (4, 2000, 8)]:
        g = synth.few_priorities_game(n, 2, 5, d, seed)
        np.testing.assert_array_equal(orc.dense_solve(g)["winner"],
                                      zielonka(g))


@pytest.mark.parametrize("seed", range(15))
def test_dense_best_response_is_pointwise_minimum(seed):
    """Brute force over every positional tau on modified games of at most
    12 vertices with repeated priorities."""
    rng = np.random.default_rng(700 + seed)
    g = synth.few_priorities_game(int(rng.integers(3, 8)), 1, 3,
                                  int(rng.integers(2, 4)), 800 + seed)
    aug = orc.dense_preprocess(g)
    if aug["n"] > 12:
        pytest.skip("modified game too large for brute force")
    r = L.solve(aug, preprocess_game=False)
    rows = L.rows_of(aug)
    dom = r["vals"].dom
    for sigma, tau, val in r["majors"]:
        best = L.brute_force_tau_min(aug, r["vals"], rows, sigma)
        for v in range(aug["n"]):
            assert L.val_le(val[v], best[v], dom) and \
                L.val_le(best[v], val[v], dom)


@pytest.mark.parametrize("seed", range(12))
def test_dense_equals_rank_path_on_distinct_priorities(seed):
    """With distinct priorities the count order is the rank order: on the
    same modified game both oracles take the same switches."""
    g = synth.random_game(30 + 20 * seed, 1 + seed % 3, 5, 2000 + seed) \
        if seed % 4 else synth.chain_game(30 + 20 * seed, 2000 + seed)
    aug = orc.preprocess(g)
    rk = orc.solve(g)
    dn = orc.dense_solve(g, aug=aug)
    assert rk["status"] == dn["status"] == orc.OK
    for k in ("winner", "sigma", "tau"):
        np.testing.assert_array_equal(rk[k], dn[k])
    for k in ("n_major", "n_valuations", "n_odd_switches", "n_even_switches"):
        assert rk[k] == dn[k]
    # the last valuation: ranks and counts order every pair alike
    n = aug["n"]
    key = rk["key"].astype(np.int64)
    rng = np.random.default_rng(seed)
    for a, b in rng.integers(0, n + 1, size=(300, 2)):
        want = int(np.sign(key[a] - key[b]))
        assert orc.dense_compare(dn["counts"], dn["top"], dn["values"],
                                 int(a), int(b)) == want


def test_dense_inadmissible_without_preprocessing():
    # two Odd vertices in a cycle whose largest priority (3) is odd
    g = {"n": 2, "m": 2, "offsets": np.array([0, 1, 2]),
         "targets": np.array([1, 0], np.int32),
         "owner": np.array([1, 1], np.uint8),
         "pri": np.array([3, 3], np.int32)}
    assert orc.dense_solve(g, preprocess_game=False)["status"] == \
        orc.EINADMISSIBLE
    r = orc.dense_solve(g)
    assert r["status"] == orc.OK
    np.testing.assert_array_equal(r["winner"], [1, 1])


# ---------------------------------------------------------------------------
# preprocessing of this path (section 3, "The algorithm")
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(20))
def test_dense_preprocess_reading(seed):
    rng = np.random.default_rng(seed)
    g = synth.few_priorities_game(int(rng.integers(10, 200)), 1, 4,
                                  int(rng.integers(2, 5)), 3000 + seed)
    g["owner"] = (rng.random(g["n"]) < 0.8).astype(np.uint8)  # many X sets
    dn = orc.dense_preprocess(g)
    rk = orc.preprocess(g)
    for k in ("offsets", "targets", "owner", "dummy_of"):
        np.testing.assert_array_equal(dn[k], rk[k])
    n, k = g["n"], dn["n"] - g["n"]
    shift = 2 if k > 0 else 0
    np.testing.assert_array_equal(dn["pri"][:n], g["pri"] + shift)
    assert not dn["pri"][n:].any()
    lit = L.identity_augment(dn)
    from tests.test_oracle_pins import _odd_subgraph_acyclic
    assert _odd_subgraph_acyclic(lit)
    np.testing.assert_array_equal(zielonka(dn)[:n], zielonka(g))


# ---------------------------------------------------------------------------
# best-response variants (section 4; section 6, Table 2's SI / SI-Reset /
# Bellman-Ford comparison)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(20))
def test_dense_bellman_ford_matches_literal_and_si(seed):
    """At every major iteration of the SI run: the C oracle's Bellman-Ford
    labels and round count equal the literal oracle's, the labels equal SI's
    best-response valuations, and its tau realises them."""
    g = _few(seed, nmin=5, nmax=60)
    aug = orc.dense_preprocess(g)
    lit = L.solve(aug, preprocess_game=False)
    rows = L.rows_of(aug)
    for sigma, tau, val in lit["majors"]:
        bf = orc.dense_bellman_ford(aug, sigma)
        lab, rounds = L.bellman_ford(aug, lit["vals"], rows, sigma)
        assert bf["rounds"] == rounds
        for v in range(aug["n"]):
            for ref in (lab[v], val[v]):
                if ref is L.TOP:
                    assert bf["top"][v] == 1
                else:
                    assert bf["top"][v] == 0
                    np.testing.assert_array_equal(bf["counts"][v], ref)
        succ = np.where(aug["owner"] == 1, bf["tau"], sigma).astype(np.int32)
        c2, t2, _, rc = orc.dense_valuation(succ, aug["pri"])
        assert rc == orc.OK
        np.testing.assert_array_equal(t2, bf["top"])
        np.testing.assert_array_equal(c2, bf["counts"])


@pytest.mark.parametrize("seed", range(15))
def test_dense_best_response_variants_same_outer_run(seed):
    """The outer loop sees only valuations, which every best response gives
    alike: the same sigma at the end, winners and major iterations."""
    g = _few(seed, nmin=20, nmax=400)
    si = orc.dense_solve(g)
    for br in (orc.BR_SI_RESET, orc.BR_BELLMAN_FORD):
        r = orc.dense_solve(g, br=br)
        assert r["status"] == orc.OK
        np.testing.assert_array_equal(r["winner"], si["winner"])
        np.testing.assert_array_equal(r["sigma"], si["sigma"])
        assert r["n_major"] == si["n_major"]
        np.testing.assert_array_equal(r["top"], si["top"])
        np.testing.assert_array_equal(r["counts"], si["counts"])


@pytest.mark.parametrize("seed", range(10))
def test_si_reset_rank_oracle(seed):
    g = synth.random_game(50 + 30 * seed, 1 + seed % 3, 5, 4000 + seed)
    si = orc.solve(g)
    rs = orc.solve(g, reset=True)
    assert rs["status"] == orc.OK
    for k in ("winner", "sigma", "key"):
        np.testing.assert_array_equal(rs[k], si[k])
    assert rs["n_major"] == si["n_major"]
    assert rs["n_valuations"] >= rs["n_major"]
