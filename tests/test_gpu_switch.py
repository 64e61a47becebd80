"""All_Odd over the bucketed edge layout (PG_SWITCH_BUCKETS) against the CPU
oracle and against the row form (PG_SWITCH_ROWS), through the C ABI: whole
solves, best responses from a given strategy (also one naming vertices
outside their rows), sizes with one and with many chunks and buckets and
ragged tails, games with no Odd vertex, and the flags' error path."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import PG_EINVAL, Game
from tests.helpers import off_row_tau, oracle_trajectory, to_np

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check(g, switch):
    ref = orc.solve(g)
    assert ref["status"] == 0
    with Game.from_dict(g, switch=switch) as d:
        out = d.solve()
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
    st = out["stats"]
    assert st["n_major"] == ref["n_major"]
    assert st["n_valuations"] == ref["n_valuations"]
    assert st["n_odd_switches"] == ref["n_odd_switches"]
    assert st["n_even_switches"] == ref["n_even_switches"]


# n chosen so that the Odd vertices fill one bucket (2,048) or several with a
# ragged last one, and the Odd rows one chunk (32,768 edges) or many
@pytest.mark.parametrize("n,kind,seed", [
    (3, "rnd", 1), (40, "rnd", 2), (3000, "rnd", 3), (4095, "rnd", 4),
    (4097, "rnd", 5), (20011, "rnd", 6), (60000, "rnd", 7),
    (30007, "chain", 8), (12, "chain", 9)])
def test_bucketed_solves_match_oracle(n, kind, seed):
    g = synth.random_game(n, 2, 10, seed) if kind == "rnd" else \
        synth.chain_game(n, seed)
    _say("bucketed solve", kind, n, seed)
    _check(g, "buckets")


def _oracle_best_response(aug, sigma, tau):
    by_pri = orc.order_by_pri(aug["pri"])
    t = tau.copy()
    nval = 0
    while True:
        succ = np.where(aug["owner"] == 1, t, sigma).astype(np.int32)
        key, _, rc = orc.valuation(succ, aug["pri"], by_pri=by_pri)
        assert rc == 0
        nval += 1
        t, c = orc.odd_switch(aug, key, t)
        if c == 0:
            return t, key, nval


def test_bucketed_and_row_forms_agree_along_a_solve():
    """Best responses from Even strategies taken along the oracle's solve:
    both forms give the oracle's tau, keys and valuation count."""
    g = synth.random_game(40000, 2, 5, 17)
    aug = orc.preprocess(g)
    traj = list(oracle_trajectory(aug))
    with Game.from_dict(g, switch="buckets") as a, \
            Game.from_dict(g, switch="rows") as b:
        for k in (0, len(traj) // 3, len(traj) - 1):
            sigma, tau, _ = traj[k]
            _say("trajectory point", k, "of", len(traj))
            t, key, nval = _oracle_best_response(aug, sigma, tau)
            for dev in (a, b):
                dtau, dkey, dn = dev.best_response(sigma, tau)
                np.testing.assert_array_equal(to_np(dtau), t)
                np.testing.assert_array_equal(to_np(dkey), key)
                assert dn == nval


def test_bucketed_best_response_from_strategy_outside_rows():
    """A current choice outside the row (allowed at the C ABI) has its key
    read on its own, as the oracle does."""
    g = synth.random_game(6000, 2, 5, 6)
    aug = orc.preprocess(g)
    sigma, tau = orc.initial_strategies(aug)
    tau = off_row_tau(aug, tau, 400, 1)
    t, key, nval = _oracle_best_response(aug, sigma, tau)
    with Game.from_dict(g, switch="buckets") as dev:
        dtau, dkey, dn = dev.best_response(sigma, tau)
    np.testing.assert_array_equal(to_np(dtau), t)
    np.testing.assert_array_equal(to_np(dkey), key)
    assert dn == nval


def test_bucketed_without_odd_vertices_and_all_odd():
    g = synth.random_game(5000, 2, 5, 3)
    for own in (0, 1):
        h = dict(g)
        h["owner"] = np.full(g["n"], own, np.uint8)
        _say("owner", own)
        _check(h, "buckets")


def test_bucketed_repeated_edges_and_large_priorities():
    rng = np.random.default_rng(11)
    g = synth.random_game(9000, 3, 8, 12)
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v)
         for k, v in g.items()}
    # every third row repeats its first target
    off = g["offsets"]
    rows = np.flatnonzero(np.diff(off) >= 2)[::3]
    g["targets"][off[rows] + 1] = g["targets"][off[rows]]
    g["pri"] = (rng.choice(2**29, size=g["n"], replace=False) + 2**30
                ).astype(np.int32)
    _check(g, "buckets")


def test_switch_flags_exclude_each_other():
    from paper_1705_02313_amd.pg import (PG_SWITCH_BUCKETS, PG_SWITCH_ROWS,
                                         lib)
    import ctypes
    g = synth.random_game(50, 2, 3, 1)
    h = ctypes.c_void_p()
    off = np.ascontiguousarray(g["offsets"], np.int64)
    tgt = np.ascontiguousarray(g["targets"], np.int32)
    own = np.ascontiguousarray(g["owner"], np.uint8)
    pri = np.ascontiguousarray(g["pri"], np.int32)
    rc = lib().pg_load_csr(g["n"], g["m"], off.ctypes.data_as(ctypes.c_void_p),
                           tgt.ctypes.data_as(ctypes.c_void_p),
                           own.ctypes.data_as(ctypes.c_void_p),
                           pri.ctypes.data_as(ctypes.c_void_p),
                           PG_SWITCH_ROWS | PG_SWITCH_BUCKETS, None,
                           ctypes.byref(h))
    assert rc == PG_EINVAL
    with pytest.raises(ValueError):
        Game.from_dict(g, switch="both")  # rejected before the C ABI


@pytest.mark.parametrize("n_odd", [2048, 4096, 8192])
def test_bucketed_exact_bucket_and_chunk_boundaries(n_odd):
    """Odd vertices filling whole buckets (2,048 each) and Odd rows (8 edges
    each) filling half a chunk, one chunk or two (32,768 edges each)."""
    rng = np.random.default_rng(n_odd)
    n = 2 * n_odd
    deg = np.where(np.arange(n) < n_odd, 8, rng.integers(2, 6, n))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(deg)
    g = {"n": n, "m": int(off[-1]), "offsets": off,
         "targets": rng.integers(0, n, int(off[-1])).astype(np.int32),
         "owner": (np.arange(n) < n_odd).astype(np.uint8),
         "pri": rng.permutation(n).astype(np.int32)}
    aug = orc.preprocess(g)
    own = aug["owner"]
    assert int((own == 1).sum()) == n_odd
    assert int(np.diff(aug["offsets"])[own == 1].sum()) == 8 * n_odd
    _check(g, "buckets")


def test_bucketed_flag_ignored_by_count_valuations():
    """Count valuations read rows whatever the flag says: same solve as the
    oracle's."""
    g = synth.few_priorities_game(5000, 2, 5, 4, 3)
    ref = orc.dense_solve(g)
    with Game.from_dict(g, switch="buckets") as d:
        assert d.d == ref["values"].size
        out = d.solve()
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
    assert out["stats"]["n_valuations"] == ref["n_valuations"]


@pytest.mark.parametrize("opts", [{"careful_walks": True}, {"graph": False},
                                  {"host_reduced_list": True}],
                         ids=["careful", "eager", "host_list"])
@pytest.mark.parametrize("kind", ["rnd", "chain"])
def test_bucketed_with_other_load_flags(opts, kind):
    """The bucketed step under host-driven walk rounds (and the rerun after
    bounded rounds leave work), eager launches, and the host-ranked reduced
    list: the oracle's solve each time."""
    g = synth.random_game(30000, 2, 6, 51) if kind == "rnd" else \
        synth.chain_game(40000, 52)
    ref = orc.solve(g)
    assert ref["status"] == 0
    _say("bucketed with", opts, kind)
    with Game.from_dict(g, switch="buckets", **opts) as d:
        out = d.solve()
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
    assert out["stats"]["n_valuations"] == ref["n_valuations"]
    assert out["stats"]["n_odd_switches"] == ref["n_odd_switches"]
