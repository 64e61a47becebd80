"""Monotonicity of the valuations along Algorithm 1, on the literal layer's
dense valuations (no rank keys involved):

* an Odd switch lowers no valuation (section 4: each All_Odd step of the
  one-player improvement for Odd switches to strictly better edges for Odd,
  which can only lower the valuations): inside an inner loop the
  valuations are pointwise non-increasing, strictly somewhere while Odd
  still switches;
* an Even switch of switchable edges raises the best response's valuation
  pointwise, strictly somewhere (section 3, Theorem 1, second item), and the
  next best response is the pointwise least valuation over Odd's strategies
  (section 3, "Best responses"): so every valuation after a best response is
  at least that best response, pointwise.

The device relies on the two consequences: a vertex top in a best response
stays top in every later valuation (it marks such vertices and its walks
stop at them), and a vertex finite in one valuation of an inner loop stays
finite for the rest of that loop (its fate is kept).  Planted mistakes in
the oracle's switching rules are caught by these pins too.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import literal
from oracle.literal import TOP
from paper_1705_02313_amd import synth


def _le_all(a, b, dom):
    return all(literal.val_le(x, y, dom) for x, y in zip(a, b))


def _lt_some(a, b, dom):
    return any(literal.val_lt(x, y, dom) for x, y in zip(a, b))


def _run(game, odd_rule=None, even_rule=None):
    """Algorithm 1 on the literal layer; returns, per major iteration, the
    list of its inner loop's valuations (the last one the best response)."""
    g = literal.preprocess(game)
    rows = literal.rows_of(g)
    vals = literal.Vals(g["pri"])
    odd_rule = odd_rule or literal.odd_switches
    even_rule = even_rule or literal.even_switches
    sigma, tau = literal.initial_strategies(g, rows)
    majors = []
    for _ in range(10000):
        inner = []
        for _ in range(10000):
            val, cycles = literal.valuation(g, vals, sigma, tau)
            assert all(literal.cycle_is_even(g, c) for c in cycles)
            inner.append(val)
            tau2, c = odd_rule(g, vals, rows, sigma, tau, val)
            if c == 0:
                break
            tau = tau2
        majors.append(inner)
        sigma2, c = even_rule(g, vals, rows, sigma, inner[-1])
        if c == 0:
            return majors, vals.dom
        sigma = sigma2
    raise AssertionError("no termination")


def _check(majors, dom):
    prev_br = None
    for inner in majors:
        # Odd's switches: non-increasing, strictly while it switches
        for a, b in zip(inner, inner[1:]):
            assert _le_all(b, a, dom)
            assert _lt_some(b, a, dom)
            # a finite vertex stays finite inside the loop
            assert all(y is not TOP for x, y in zip(a, b) if x is not TOP)
        if prev_br is not None:
            br = inner[-1]
            # Theorem 1: the best responses improve, strictly somewhere
            assert _le_all(prev_br, br, dom)
            assert _lt_some(prev_br, br, dom)
            # every valuation after a best response is at least it; a top
            # vertex stays top
            for val in inner:
                assert _le_all(prev_br, val, dom)
                assert all(y is TOP for x, y in zip(prev_br, val) if x is TOP)
        prev_br = inner[-1]


@pytest.mark.parametrize("seed", range(30))
def test_valuations_are_monotone_along_the_run(seed):
    rng = np.random.Generator(np.random.PCG64(9100 + seed))
    n = int(rng.integers(8, 160))
    if seed % 3 == 2:
        game = synth.few_priorities_game(n, 1, 4, 3, 9100 + seed)
    else:
        game = synth.random_game(n, 1, 4, 9100 + seed)
    majors, dom = _run(game)
    _check(majors, dom)


def test_long_runs_are_monotone():
    """Games with several outer iterations and long inner loops."""
    seen = 0
    for seed in range(40):
        game = synth.random_game(120, 2, 3, 9200 + seed)
        majors, dom = _run(game)
        _check(majors, dom)
        seen += sum(len(inner) for inner in majors) >= 8
    assert seen >= 10


def _first_best(g, vals, rows, v, val, better):
    best = rows[v][0]
    for u in rows[v][1:]:
        if better(val[u], val[best]):
            best = u
    return best


def test_planted_wrong_odd_direction_is_caught():
    """An Odd rule that switches to the largest successor (a sign mistake)
    raises valuations inside the inner loop: the pins fail."""
    def bad_odd(g, vals, rows, sigma, tau, val):
        dom = vals.dom
        new_tau, count = list(tau), 0
        for v in range(int(g["n"])):
            if g["owner"][v] != 1:
                continue
            b = _first_best(g, vals, rows, v, val,
                            lambda x, y: literal.val_lt(y, x, dom))
            if literal.val_lt(val[tau[v]], val[b], dom):
                new_tau[v] = b
                count += 1
        return new_tau, count

    caught = 0
    for seed in range(20):
        game = synth.random_game(60, 2, 4, 9300 + seed)
        try:
            majors, dom = _run(game, odd_rule=bad_odd)
            _check(majors, dom)
        except AssertionError:
            caught += 1
        except RuntimeError:
            caught += 1
    assert caught >= 10


def test_planted_non_improving_even_switch_is_caught():
    """An Even rule that also moves to equal-or-worse successors breaks the
    strict improvement of Theorem 1."""
    def bad_even(g, vals, rows, sigma, val):
        dom = vals.dom
        zero = vals.zero()

        def vv(u):
            return zero if u == literal.SINK else val[u]

        new_sigma, count = list(sigma), 0
        for v in range(int(g["n"])):
            if g["owner"][v] != 0:
                continue
            worst = literal.SINK
            for u in rows[v]:
                if literal.val_lt(vv(u), vv(worst), dom):
                    worst = u
            if literal.val_lt(vv(worst), vv(sigma[v]), dom):
                new_sigma[v] = worst
                count += 1
        return new_sigma, count

    caught = 0
    for seed in range(20):
        game = synth.random_game(60, 2, 4, 9400 + seed)
        try:
            majors, dom = _run(game, even_rule=bad_even)
            _check(majors, dom)
        except (AssertionError, literal.Inadmissible):
            caught += 1
    assert caught >= 10
