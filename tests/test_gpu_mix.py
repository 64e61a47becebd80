"""The batched/served mix at its stated size against oracle-written values.

1,024 random games (seeds 4000 + g, n log-uniform in [1e3, 2e5], out-degree
uniform in [2, 8]) go through the serving loop twice: all present at the
start, and as a Poisson stream under an arena budget of a quarter of the
mix's modified vertices and edges (games queue, join and leave the arena
between steps).  Every game's winners, sigma*, tau*, iteration and switch
counts must equal what the CPU oracle computed for it alone
(tests/golden/golden_c4.json, written by tests/golden/make_golden_mix.py,
which calls only oracle/).
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from paper_1705_02313_amd import synth
from paper_1705_02313_amd.serve import poisson_arrivals, serve
from tests.helpers import np_hash

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def mix():
    path = os.path.join(HERE, "golden", "golden_c4.json")
    with open(path) as f:
        gold = json.load(f)
    games = synth.mixed_batch(gold["games"], gold["seed_base"])
    return games, gold["data"]


def _assert_game(i, r, gd):
    st = r["stats"]
    assert (st["n"], st["n_aug"], st["m_aug"]) == \
        (gd["n"], gd["n_aug"], gd["m_aug"]), i
    assert st["n_major"] == gd["n_major"], i
    assert st["n_valuations"] == gd["n_valuations"], i
    assert st["n_odd_switches"] == gd["n_odd_switches"], i
    assert st["n_even_switches"] == gd["n_even_switches"], i
    assert np_hash(np.asarray(r["winner"]).astype(np.int32)) == \
        gd["winner_hash"], i
    assert np_hash(r["sigma"]) == gd["sigma_hash"], i
    assert np_hash(r["tau"]) == gd["tau_hash"], i


def _budget(gold, frac):
    nv = sum(g["n_aug"] for g in gold)
    ne = sum(g["m_aug"] for g in gold)
    return (max(int(nv * frac), max(g["n_aug"] for g in gold) + 1),
            max(int(ne * frac), max(g["m_aug"] for g in gold) + 1))


def test_mix_all_present_at_start(mix):
    games, gold = mix
    print("1024-game mix, all at t=0", flush=True)
    bv, be = _budget(gold, 1.0)
    r = serve(games, np.zeros(len(games)), bv, be)
    assert len(r["results"]) == len(games)
    for i, gd in enumerate(gold):
        _assert_game(i, r["results"][i], gd)


def test_mix_served_poisson_quarter_arena(mix):
    games, gold = mix
    print("1024-game mix, Poisson arrivals, quarter arena", flush=True)
    bv, be = _budget(gold, 0.25)
    # about the batched rate of the mix on one MI355X, so that requests
    # arrive while others run and the arena fills and drains
    arr = poisson_arrivals(len(games), 1500.0, 4242)
    r = serve(games, arr, bv, be)
    assert len(r["results"]) == len(games)
    lat = r["latency"]
    assert np.isfinite(lat).all() and (lat >= 0).all()
    for i, gd in enumerate(gold):
        _assert_game(i, r["results"][i], gd)
