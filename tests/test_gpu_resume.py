"""Warm start and checkpoints of pg_solve, the per-valuation trace, and
calls from two threads at once.

* A run stopped by a cap (outer or inner) hands back its strategies; a run
  started from them takes exactly the remaining iterations of the
  uninterrupted run: the same winners and strategies, counts that add up,
  and its traced valuations are the tail of the uninterrupted trace.  All of
  it against the CPU oracle's run of the same game (Algorithm 1).
* Two threads load and solve different games on two streams at the same
  time (their loads share the per-device memory cache): each result equals
  the oracle's.
* Games handed to a batch as device arrays give the oracle's results.
"""
from __future__ import annotations

import threading

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import (PG_EINVAL, Batch, Game, PgError,
                                     write_trace_jsonl)
from tests.helpers import np_hash, to_np

pytestmark = pytest.mark.gpu


def _assert_final(out, ref):
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])


@pytest.mark.parametrize("device", [False, True])
def test_trace_matches_oracle_trace(device):
    g = synth.random_game(4000, 2, 6, 31)
    ref = orc.solve(g, trace=True)
    with Game.from_dict(g, device=device) as d:
        out = d.solve(trace=4096)
    _assert_final(out, ref)
    tr = out["trace"]
    assert out["stats"]["n_traced"] == ref["n_valuations"]
    assert [int(x) for x in tr["key_hash"]] == [int(x) for x in ref["trace"]]
    assert int(tr["switches"].sum()) == ref["n_odd_switches"]
    assert (tr["finite"] >= 1).all() and (tr["ms"] > 0).all()
    assert out["stats"]["iteration_ms"] > 0
    # a short trace stops at its capacity
    with Game.from_dict(g, device=device) as d:
        out2 = d.solve(trace=3)
    assert out2["stats"]["n_traced"] == 3
    assert [int(x) for x in out2["trace"]["key_hash"]] == \
        [int(x) for x in ref["trace"][:3]]


def test_trace_jsonl(tmp_path):
    g = synth.random_game(1500, 2, 5, 32)
    with Game.from_dict(g) as d:
        out = d.solve(trace=512)
    path = tmp_path / "trace.jsonl"
    write_trace_jsonl(str(path), out, {"workload": "test"})
    import json
    rows = [json.loads(x) for x in path.read_text().splitlines()]
    assert len(rows) == out["stats"]["n_valuations"]
    assert rows[-1]["odd_switches"] == 0
    assert all(r["workload"] == "test" for r in rows)


@pytest.mark.parametrize("device", [False, True])
def test_resume_after_outer_cap(device):
    g = synth.random_game(6000, 2, 5, 33)
    ref = orc.solve(g, trace=True)
    assert ref["n_major"] >= 4
    with Game.from_dict(g, device=device) as d:
        full = d.solve(trace=8192)
        _assert_final(full, ref)
        for k in (1, 2, ref["n_major"] - 2):
            cp = d.solve(max_major=k, keep_dummies=True, checkpoint=True,
                         trace=8192)
            assert cp["stopped"] and cp["stats"]["n_major"] == k
            rest = d.solve(init_sigma=cp["sigma"], init_tau=cp["tau"],
                           trace=8192)
            _assert_final(rest, ref)
            a, b = cp["stats"], rest["stats"]
            assert a["n_major"] + b["n_major"] == ref["n_major"]
            assert a["n_valuations"] + b["n_valuations"] == \
                ref["n_valuations"]
            assert a["n_odd_switches"] + b["n_odd_switches"] == \
                ref["n_odd_switches"]
            assert a["n_even_switches"] + b["n_even_switches"] == \
                ref["n_even_switches"]
            joined = list(cp["trace"]["key_hash"]) + \
                list(rest["trace"]["key_hash"])
            assert [int(x) for x in joined] == [int(x) for x in ref["trace"]]


def test_resume_inside_a_best_response():
    g = synth.random_game(6000, 2, 5, 34)
    ref = orc.solve(g)
    with Game.from_dict(g) as d:
        cp = d.solve(max_inner=2, keep_dummies=True, checkpoint=True)
        assert cp["stopped"] and cp["stats"]["n_valuations"] == 2
        rest = d.solve(init_sigma=cp["sigma"], init_tau=cp["tau"])
    _assert_final(rest, ref)
    assert rest["stats"]["n_major"] == ref["n_major"]
    assert 2 + rest["stats"]["n_valuations"] == ref["n_valuations"]


def test_warm_start_one_side_only():
    """init_tau alone keeps sigma_init; init_sigma alone keeps the first
    row entries for Odd."""
    g = synth.random_game(2000, 2, 5, 35)
    ref = orc.solve(g)
    aug = orc.preprocess(g)
    sigma0, tau0 = orc.initial_strategies(aug)
    with Game.from_dict(g) as d:
        _assert_final(d.solve(init_tau=tau0), ref)
        _assert_final(d.solve(init_sigma=sigma0), ref)
        with pytest.raises(PgError) as e:
            # an Even vertex's entry (Odd entries of sigma are ignored)
            bad = sigma0.copy()
            bad[int(np.flatnonzero(aug["owner"] == 0)[0])] = d.n_aug + 5
            d.solve(init_sigma=bad)
        assert e.value.status == PG_EINVAL


def test_two_threads_two_streams():
    """Loads and solves on two threads with their own streams at once; the
    loads' temporaries go through the shared device memory cache."""
    import torch
    games = [[synth.random_game(n, 2, 6, 40 + 10 * t + k)
              for k, n in enumerate((30000, 5000, 60000, 12000))]
             for t in range(2)]
    refs = [[orc.solve(g) for g in gs] for gs in games]
    errors = []

    def worker(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for rep in range(3):
                    for g, ref in zip(games[t], refs[t]):
                        with Game.from_dict(g, device=True) as d:
                            out = d.solve()
                        s.synchronize()
                        _assert_final(out, ref)
                        assert out["stats"]["n_valuations"] == \
                            ref["n_valuations"]
        except Exception as e:  # reported by the main thread
            errors.append(e)

    ths = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert not errors, errors[0]


def test_batch_submit_device_arrays():
    games = [synth.random_game(n, 2, 7, 50 + n) for n in (800, 5000, 20000)]
    with Batch(200000, 2000000) as b:
        tickets = [b.submit(g, device=True) for g in games]
        out = {}
        for _ in range(100000):
            b.step()
            for t in b.finished():
                out[t] = b.poll(t)
            if len(out) == len(games):
                break
    for g, t in zip(games, tickets):
        ref = orc.solve(g)
        _assert_final(out[t], ref)
        assert out[t]["stats"]["n_valuations"] == ref["n_valuations"]
        assert np_hash(out[t]["sigma"]) == np_hash(ref["sigma"])
