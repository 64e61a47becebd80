"""Full-size workloads on the device against stored oracle results.

The expected values in tests/golden/ were written by
tests/golden/make_golden.py, which runs only the CPU oracle.  The device runs
in the configuration bench.py times (game arrays handed over as device
tensors).  Besides the stored values, properties that hold at any size are
checked: at the end no edge is switchable and both winning sets are closed.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import Game
from tests.helpers import (KEY_TOP, is_original_edge, np_hash, tau_to_aug,
                           to_np)

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    path = os.path.join(HERE, "golden", f"golden_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)["data"]


def _final_checks(dev: Game, out, tau):
    """No switchable edge at the end; closure of the winning sets (tau in
    the modified game's ids)."""
    sigma = to_np(out["sigma"])
    key, _ = dev.valuation(sigma, tau)
    key = to_np(key).astype(np.int64)
    ex = dev.export()
    off, tgt, own = ex["offsets"], ex["targets"], ex["owner"]
    N = ex["n"]
    src = np.repeat(np.arange(N), np.diff(off))
    kt = key[tgt]
    # best option per row
    row_min = np.full(N, np.iinfo(np.int64).max)
    np.minimum.at(row_min, src, kt)
    row_max = np.full(N, key[N])          # Even may always take the sink
    np.maximum.at(row_max, src, kt)
    cur = np.where(own == 0, np.where(sigma < 0, N, sigma), tau)
    kc = key[cur]
    odd = own == 1
    assert not (odd & (row_min < kc)).any(), "an Odd edge is switchable"
    assert not (~odd & (row_max > kc)).any(), "an Even edge is switchable"
    w_even = key[:N] == KEY_TOP
    # Even keeps its winning vertices inside W_Even; Odd cannot leave it
    assert w_even[cur[~odd & w_even]].all()
    edge_from_weven_odd = w_even[src] & odd[src]
    assert w_even[tgt[edge_from_weven_odd]].all()
    # Odd keeps its vertices in W_Odd; Even cannot leave W_Odd
    assert (~w_even[cur[odd & ~w_even]]).all()
    edge_from_wodd_even = (~w_even[src]) & (~odd[src])
    assert (~w_even[tgt[edge_from_wodd_even]]).all()
    np.testing.assert_array_equal(to_np(out["winner"]),
                                  (~w_even[:dev.n]).astype(np.uint8))


def _run(game, gold, device=True):
    with Game.from_dict(game, device=device) as dev:
        assert dev.n_aug == gold["n_aug"] and dev.m_aug == gold["m_aug"]
        s0, t0 = dev.initial_strategies()
        k0, _ = dev.valuation(s0, t0)
        assert np_hash(to_np(k0)) == gold["trace"][0]
        out = dev.solve(trace=len(gold["trace"]) + 8)
        st = out["stats"]
        assert st["n_major"] == gold["n_major"]
        assert st["n_valuations"] == gold["n_valuations"]
        assert st["n_odd_switches"] == gold["n_odd_switches"]
        assert st["n_even_switches"] == gold["n_even_switches"]
        # every valuation of the run, bit for bit (hash of all n_aug + 1
        # keys in the caller's ids), and the last one
        tr = out["trace"]
        assert st["n_traced"] == len(gold["trace"])
        got = [int(x) for x in tr["key_hash"]]
        bad = [i for i, (a, b) in enumerate(zip(got, gold["trace"]))
               if a != b]
        assert not bad, f"valuations {bad[:10]} differ from the oracle's"
        assert got[-1] == gold["key_hash"]
        assert (tr["switches"][:-1] >= 0).all() and tr["switches"][-1] == 0
        assert int(tr["switches"].sum()) == gold["n_odd_switches"]
        assert np_hash(to_np(out["winner"]).astype(np.int32)) == \
            gold["winner_hash"]
        assert np_hash(to_np(out["sigma"])) == gold["sigma_hash"]
        # the reported tau names original vertices for the original ones;
        # back in the modified game's ids it is the stored one
        tau = to_np(out["tau"])
        assert is_original_edge(game, tau, dev.n)
        ex = dev.export()
        tau = tau_to_aug(ex["offsets"], ex["targets"], ex["owner"], tau,
                         dev.n)
        assert np_hash(tau) == gold["tau_hash"]
        _final_checks(dev, out, tau)


def _offsets(game, dtype):
    g = dict(game)
    g["offsets"] = np.asarray(game["offsets"]).astype(dtype)
    return g


@pytest.mark.parametrize("offsets", ["int64", "int32"])
def test_config0_twenty_seeds(offsets):
    gold = _golden("c0s")
    for seed, gd in gold.items():
        print("c0 seed", seed, offsets, flush=True)
        g = _offsets(synth.random_game(1000, 2, 5, int(seed)), offsets)
        assert np.asarray(g["offsets"]).dtype == np.dtype(offsets)
        _run(g, gd, device=(offsets == "int32"))


# the workloads' own offset widths: int32 for configs 1 and 3, int64 for
# config 2; the other width as well where it can address the edges
@pytest.mark.parametrize("cfg,offsets", [(1, "int32"), (1, "int64"),
                                         (2, "int64"), (3, "int32"),
                                         (3, "int64")])
def test_full_size_config(cfg, offsets):
    gold = _golden(f"c{cfg}")
    print("config", cfg, offsets, flush=True)
    g = _offsets(synth.config_game(cfg), offsets)
    _run(g, gold)
