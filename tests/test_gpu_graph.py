"""The captured best-response iteration (a HIP graph per ng/cand pair,
replayed on the caller's stream) against eager launches and the oracle:
several solves on one game (every replay after the first two captures), and
best responses interleaved with eager valuations and host synchronisations
between the replays."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import Game
from tests.helpers import oracle_trajectory, to_np

pytestmark = pytest.mark.gpu


def _same(a, b):
    for k in ("winner", "sigma", "tau"):
        np.testing.assert_array_equal(to_np(a[k]), to_np(b[k]))
    for k in ("n_major", "n_valuations", "n_odd_switches", "n_even_switches"):
        assert a["stats"][k] == b["stats"][k]


@pytest.mark.parametrize("kind", ["random", "chain", "counts"])
def test_graph_solves_match_eager_and_oracle(kind):
    if kind == "random":
        g = synth.random_game(40000, 2, 6, 61)
        ref = orc.solve(g)
    elif kind == "chain":
        g = synth.chain_game(50000, 62)
        ref = orc.solve(g)
    else:
        g = synth.few_priorities_game(40000, 2, 6, 4, 63)
        ref = orc.dense_solve(g)
    with Game.from_dict(g, graph=False) as d0:
        eager = d0.solve()
    with Game.from_dict(g) as d1:
        runs = [d1.solve() for _ in range(3)]
    for r in runs:
        _same(r, eager)
    np.testing.assert_array_equal(to_np(eager["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(eager["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(eager["tau"]), ref["tau_orig"])
    assert eager["stats"]["n_valuations"] == ref["n_valuations"]


def test_graph_best_responses_between_eager_work():
    g = synth.random_game(30000, 2, 6, 64)
    aug = orc.preprocess(g)
    sigmas = []
    last = None
    for sigma, tau, key in oracle_trajectory(aug):
        if last is None or not np.array_equal(sigma, last):
            sigmas.append(sigma)
            last = sigma
    assert len(sigmas) >= 3
    with Game.from_dict(g) as dg, Game.from_dict(g, graph=False) as de:
        s0, t0 = dg.initial_strategies()
        t0 = to_np(t0)
        for sigma in sigmas:
            tg, kg, ng = dg.best_response(sigma, t0)
            te, ke, ne = de.best_response(sigma, t0)
            np.testing.assert_array_equal(to_np(tg), to_np(te))
            np.testing.assert_array_equal(to_np(kg), to_np(ke))
            assert ng == ne
            # eager work on the graph game between replays
            kv, nf = dg.valuation(sigma, to_np(tg))
            np.testing.assert_array_equal(to_np(kv), to_np(ke))
