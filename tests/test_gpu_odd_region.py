"""PG_ODD_REGION on the device: the game without Odd's own winning region
(no dummies) against the oracle's odd_region.solve (winners, sigma*, tau*,
counts, the reduced game itself) and against the dummy path's winners."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import odd_region, orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import PG_EINVAL, PG_SINK, Game, PgError, lib

pytestmark = pytest.mark.gpu


def _cases():
    return [
        ("random1k", synth.random_game(1000, 2, 5, 8100)),
        ("random20k", synth.random_game(20000, 2, 5, 8101, np.int32)),
        ("random20k_deg10", synth.random_game(20000, 2, 10, 8102)),
        ("few20k", synth.few_priorities_game(20000, 2, 5, 4, 8103)),
        ("chain20k", synth.chain_game(20000, 8104)),
        ("cycles60", synth.odd_cycles_game(60, 8105)),
        ("cycles3k", synth.odd_cycles_game(3000, 8106)),
        ("cycles3k_few", synth.odd_cycles_game(3000, 8107, d=4)),
        ("cycles30k", synth.odd_cycles_game(30000, 8108)),
        ("random200k", synth.random_game(200000, 2, 5, 8109, np.int32)),
    ]


def _check(game, out, ref):
    np.testing.assert_array_equal(out["winner"], ref["winner"])
    np.testing.assert_array_equal(out["sigma"], ref["sigma"])
    np.testing.assert_array_equal(out["tau"], ref["tau"])
    st = out["stats"]
    for k in ("n_major", "n_valuations", "n_odd_switches", "n_even_switches"):
        assert st[k] == ref[k], k
    assert st["n_aug"] == game["n"] - ref["n_removed"]


@pytest.mark.parametrize("case", range(10))
def test_solve_matches_the_oracle(case):
    name, g = _cases()[case]
    print(f"odd-region solve {name} n={g['n']}", flush=True)
    ref = odd_region.solve(g)
    assert ref["status"] == 0
    game = Game.from_dict(g, odd_region=True)
    try:
        out = game.solve()
        # the stored game is the oracle's subgame
        if ref["n_removed"] < g["n"]:
            sub = game.export()
            for k in ("offsets", "targets", "owner", "pri"):
                np.testing.assert_array_equal(sub[k], ref["sub"][k], k)
    finally:
        game.free()
    _check(g, out, ref)
    # Odd's own region does not change who wins
    np.testing.assert_array_equal(out["winner"], orc.solve(g)["winner"])


def test_device_pointers():
    import torch
    g = synth.odd_cycles_game(3000, 8110)
    ref = odd_region.solve(g)
    game = Game.from_dict(g, device=True, odd_region=True)
    try:
        out = game.solve()
    finally:
        game.free()
    out = {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v)
           for k, v in out.items()}
    _check(g, out, ref)


def test_odd_wins_everything():
    # every vertex Odd's, one cycle through all with an odd largest priority
    n = 7
    g = {"n": n, "m": n,
         "offsets": np.arange(n + 1, dtype=np.int64),
         "targets": ((np.arange(n) + 1) % n).astype(np.int32),
         "owner": np.ones(n, np.uint8),
         "pri": np.array([4, 0, 2, 9, 6, 1, 8], np.int32)}
    ref = odd_region.solve(g)
    assert ref["n_removed"] == n
    game = Game.from_dict(g, odd_region=True)
    try:
        assert game.n_aug == 0 and game.m_aug == 0
        empty = game.export()
        assert empty["n"] == 0 and list(empty["offsets"]) == [0]
        out = game.solve()
        with pytest.raises(PgError) as e:
            game.set_tuning(stride0=16)
        assert e.value.status == PG_EINVAL
    finally:
        game.free()
    assert (out["winner"] == 1).all()
    assert (out["sigma"] == PG_SINK).all() and (out["tau"] == PG_SINK).all()
    assert out["stats"]["n_major"] == 0


def test_nothing_removed_equals_no_preprocessing():
    """Without an all-Odd cycle of odd largest priority nothing is removed
    and the run is the one on the game itself."""
    g = synth.odd_cycles_game(3000, 8111)
    g["pri"] = (2 * np.argsort(np.asarray(g["pri"]))).astype(np.int32)
    # every priority even: every all-Odd cycle is even
    ref = odd_region.solve(g)
    assert ref["n_removed"] == 0
    a = Game.from_dict(g, odd_region=True)
    b = Game.from_dict(g, preprocess=False)
    try:
        assert a.n_aug == g["n"] and a.m_aug == g["m"]
        oa, ob = a.solve(), b.solve()
    finally:
        a.free()
        b.free()
    for k in ("winner", "sigma", "tau"):
        np.testing.assert_array_equal(oa[k], ob[k], k)
    _check(g, oa, ref)


def test_checkpoint_and_warm_start_in_original_ids():
    g = synth.random_game(20000, 2, 5, 8112)
    ref = odd_region.solve(g)
    assert ref["n_major"] >= 3
    game = Game.from_dict(g, odd_region=True)
    try:
        part = game.solve(max_major=2, checkpoint=True)
        assert part["stopped"]
        assert part["sigma"].shape == (g["n"],)
        rest = game.solve(init_sigma=part["sigma"], init_tau=part["tau"])
    finally:
        game.free()
    np.testing.assert_array_equal(rest["winner"], ref["winner"])
    np.testing.assert_array_equal(rest["sigma"], ref["sigma"])
    np.testing.assert_array_equal(rest["tau"], ref["tau"])
    assert part["stats"]["n_major"] == 2
    assert part["stats"]["n_major"] + rest["stats"]["n_major"] \
        == ref["n_major"]


def test_start_strategy_into_the_region_is_rejected():
    g = synth.random_game(2000, 2, 5, 8113)
    ref = odd_region.solve(g)
    A = np.flatnonzero(ref["A"])
    keep = np.flatnonzero(~ref["A"])
    even = keep[np.asarray(g["owner"])[keep] == 0]
    assert A.size and even.size
    sigma = np.full(g["n"], PG_SINK, np.int32)
    sigma[even[0]] = A[0]
    game = Game.from_dict(g, odd_region=True)
    try:
        with pytest.raises(PgError) as e:
            game.solve(init_sigma=sigma)
        assert e.value.status == PG_EINVAL
        # the per-vertex calls are refused
        with pytest.raises(PgError) as e:
            z = np.full(game.n_aug, PG_SINK, np.int32)
            game.best_response(z, z)
        assert e.value.status == PG_EINVAL
        # and the game still solves
        _check(g, game.solve(), ref)
    finally:
        game.free()


def test_flag_conflicts():
    g = synth.random_game(100, 2, 4, 8114)
    with pytest.raises(PgError) as e:
        Game.from_dict(g, odd_region=True, preprocess=False)
    assert e.value.status == PG_EINVAL
    assert lib() is not None


@pytest.mark.parametrize("case", ["cycles", "random", "all_odd"])
def test_without_allocation(case):
    """pg_solve_noalloc with PG_ODD_REGION: the same outputs as a loaded
    game, n entries in the original ids."""
    from paper_1705_02313_amd.pg import solve_noalloc
    if case == "cycles":
        g = synth.odd_cycles_game(3000, 8120)
    elif case == "random":
        g = synth.random_game(20000, 2, 6, 8121, np.int32)
    else:
        n = 5
        g = {"n": n, "m": n, "offsets": np.arange(n + 1, dtype=np.int64),
             "targets": ((np.arange(n) + 1) % n).astype(np.int32),
             "owner": np.ones(n, np.uint8),
             "pri": np.array([0, 2, 7, 4, 6], np.int32)}
    ref = odd_region.solve(g)
    out = solve_noalloc(g, odd_region=True)
    _check(g, out, ref)


@pytest.mark.parametrize("seed", range(6))
def test_small_and_degenerate_games(seed):
    """Self-loops, repeated edges, one-vertex games and games whose every
    vertex is one player's, against the oracle."""
    rng = np.random.Generator(np.random.PCG64(8200 + seed))
    n = [1, 2, 3, 7, 40, 300][seed]
    deg = rng.integers(1, 4, size=n)
    rows = [np.sort(rng.integers(0, n, size=d)) for d in deg]   # loops, repeats
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(deg)
    own = (rng.random(n) < [0.5, 1.0, 0.0, 0.7, 0.9, 0.6][seed]).astype(
        np.uint8)
    g = {"n": n, "m": int(off[-1]), "offsets": off,
         "targets": np.concatenate(rows).astype(np.int32), "owner": own,
         "pri": rng.permutation(n).astype(np.int32)}
    ref = odd_region.solve(g)
    game = Game.from_dict(g, odd_region=True)
    try:
        out = game.solve()
    finally:
        game.free()
    _check(g, out, ref)


@pytest.mark.parametrize("config", [1, 6])
def test_full_size(config):
    """The 1M-vertex workloads (distinct priorities; 4 repeated priorities,
    count valuations) with PG_ODD_REGION against the oracle, and the same
    winners as the dummy path."""
    g = synth.config_game(config)
    print(f"odd-region full size config {config} n={g['n']}", flush=True)
    ref = odd_region.solve(g)
    with Game.from_dict(g, odd_region=True) as game:
        out = game.solve()
    _check(g, out, ref)
    with Game.from_dict(g) as game:
        np.testing.assert_array_equal(game.solve()["winner"], ref["winner"])
