"""Device path vs the CPU oracle, element by element (bit-exact: all outputs
are integers).  Every call goes through the C ABI of the HIP library."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import Game
from tests.helpers import off_row_tau, oracle_trajectory, to_np

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _tiny_games():
    out = []
    for n in range(3, 13):
        for seed in range(6):
            out.append(("rnd", n, seed, synth.random_game(n, 2, 5, 100 * n + seed)))
    for n in (3, 5, 9, 12):
        out.append(("chain", n, 0, synth.chain_game(n, 7 + n)))
    return out


def _compare_aug(dev: Game, aug: dict):
    ex = dev.export()
    assert ex["n"] == aug["n"] and ex["m"] == aug["m"]
    np.testing.assert_array_equal(ex["offsets"], aug["offsets"])
    np.testing.assert_array_equal(ex["targets"], aug["targets"])
    np.testing.assert_array_equal(ex["owner"], aug["owner"])
    np.testing.assert_array_equal(ex["pri"], aug["pri"])


def test_preprocess_matches_oracle(pglib):
    cases = [("c0", 1000, s, synth.random_game(1000, 2, 5, s)) for s in range(4)]
    cases += [("chain", 3000, 1, synth.chain_game(3000, 11))]
    cases += _tiny_games()[::7]
    for name, n, seed, g in cases:
        _say("preprocess", name, n, seed)
        with Game.from_dict(g) as dev:
            _compare_aug(dev, orc.preprocess(g))


def test_valuations_along_trajectory(pglib):
    """Every valuation of the oracle's Algorithm 1 run, recomputed on the
    device from the same (sigma, tau)."""
    for n, seed, kind in [(1000, 0, "rnd"), (1000, 1, "rnd"), (2000, 2, "chain"),
                          (20000, 3, "rnd")]:
        g = synth.random_game(n, 2, 5, seed) if kind == "rnd" else \
            synth.chain_game(n, seed)
        aug = orc.preprocess(g)
        _say("trajectory", kind, n, seed)
        with Game.from_dict(g) as dev:
            for k, (sigma, tau, key) in enumerate(oracle_trajectory(aug)):
                dkey, nf = dev.valuation(sigma, tau)
                np.testing.assert_array_equal(to_np(dkey), key,
                                              err_msg=f"valuation {k}")
                assert nf == int((key != orc.KEY_TOP).sum())


def test_best_response_matches_oracle(pglib):
    g = synth.random_game(3000, 2, 5, 5)
    aug = orc.preprocess(g)
    sigma, tau = orc.initial_strategies(aug)
    with Game.from_dict(g) as dev:
        for major in range(4):
            # oracle inner loop
            t = tau.copy()
            nval = 0
            by_pri = orc.order_by_pri(aug["pri"])
            while True:
                succ = np.where(aug["owner"] == 1, t, sigma).astype(np.int32)
                key, _, rc = orc.valuation(succ, aug["pri"], by_pri=by_pri)
                nval += 1
                t, c = orc.odd_switch(aug, key, t)
                if c == 0:
                    break
            dtau, dkey, dn = dev.best_response(sigma, tau)
            np.testing.assert_array_equal(to_np(dtau), t)
            np.testing.assert_array_equal(to_np(dkey), key)
            assert dn == nval
            tau = t
            sigma, c = orc.even_switch(aug, key, sigma)
            if c == 0:
                break


def _solve_both(g, **kw):
    ref = orc.solve(g)
    assert ref["status"] == 0
    with Game.from_dict(g, **kw) as dev:
        out = dev.solve()
    return ref, out


def _assert_solve_equal(ref, out):
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
    assert out["stats"]["n_major"] == ref["n_major"]
    assert out["stats"]["n_valuations"] == ref["n_valuations"]


def test_solve_tiny_games(pglib):
    for name, n, seed, g in _tiny_games():
        _say("solve tiny", name, n, seed)
        ref, out = _solve_both(g)
        _assert_solve_equal(ref, out)


def test_solve_config0_seeds(pglib):
    for seed in range(12):
        g = synth.random_game(1000, 2, 5, seed)
        _say("solve c0 seed", seed)
        ref, out = _solve_both(g)
        _assert_solve_equal(ref, out)


def test_solve_midsize_ragged(pglib):
    """Sizes spanning many tiles with ragged tails."""
    for n, kind in [(4099, "rnd"), (50_001, "rnd"), (30_007, "chain")]:
        g = synth.random_game(n, 2, 10, n) if kind == "rnd" else \
            synth.chain_game(n, n)
        _say("solve midsize", kind, n)
        ref, out = _solve_both(g)
        _assert_solve_equal(ref, out)


def test_device_pointers_same_as_host(pglib):
    import torch
    g = synth.random_game(5000, 2, 8, 77)
    with Game.from_dict(g) as h:
        a = h.solve()
    with Game.from_dict(g, device=True) as d:
        b = d.solve()
        assert isinstance(b["winner"], torch.Tensor) and b["winner"].is_cuda
    np.testing.assert_array_equal(to_np(a["winner"]), to_np(b["winner"]))
    np.testing.assert_array_equal(to_np(a["sigma"]), to_np(b["sigma"]))
    np.testing.assert_array_equal(to_np(a["tau"]), to_np(b["tau"]))
    assert a["stats"]["n_valuations"] == b["stats"]["n_valuations"]


def test_device_pointers_boundary_calls(pglib):
    """Initial strategies, valuations and best responses with device arrays:
    vertex ids in and out are the caller's (the library stores a rank game
    in signed-priority order and translates at the C ABI)."""
    g = synth.random_game(7000, 2, 6, 78)
    aug = orc.preprocess(g)
    sigma, tau = orc.initial_strategies(aug)
    with Game.from_dict(g, device=True) as d:
        ds, dt = d.initial_strategies()
        np.testing.assert_array_equal(to_np(ds), sigma)
        np.testing.assert_array_equal(to_np(dt), tau)
        traj = list(oracle_trajectory(aug))
        for k in (0, len(traj) // 2, len(traj) - 1):
            s_k, t_k, key = traj[k]
            dkey, nf = d.valuation(s_k, t_k)
            np.testing.assert_array_equal(to_np(dkey), key,
                                          err_msg=f"valuation {k}")
        ref = orc.solve(g)
        out = d.solve()
        _assert_solve_equal(ref, out)
        dtau, dkey, _ = d.best_response(ref["sigma"], ref["tau"])
        np.testing.assert_array_equal(to_np(dtau), ref["tau"])


def test_best_response_from_strategy_outside_rows(pglib):
    """Odd strategies may name vertices outside their rows at the C ABI:
    the current choice's key is then read on its own, as the oracle does."""
    g = synth.random_game(3000, 2, 5, 6)
    aug = orc.preprocess(g)
    sigma, tau = orc.initial_strategies(aug)
    tau = off_row_tau(aug, tau, 200, 1)
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
            break
    with Game.from_dict(g) as dev:
        dtau, dkey, dn = dev.best_response(sigma, tau)
    np.testing.assert_array_equal(to_np(dtau), t)
    np.testing.assert_array_equal(to_np(dkey), key)
    assert dn == nval


def test_host_reduced_list_split(pglib):
    """PG_HOST_REDUCED_LIST (the host ranks the reduced list, the paper's
    GPU-LR split): the same keys along a trajectory and the same solve."""
    for n, seed, kind in [(3000, 21, "rnd"), (4000, 22, "chain")]:
        g = synth.random_game(n, 2, 5, seed) if kind == "rnd" else \
            synth.chain_game(n, seed)
        aug = orc.preprocess(g)
        _say("host reduced list", kind, n, seed)
        with Game.from_dict(g, host_reduced_list=True) as dev:
            traj = list(oracle_trajectory(aug))
            for k in (0, len(traj) // 2, len(traj) - 1):
                sigma, tau, key = traj[k]
                dkey, nf = dev.valuation(sigma, tau)
                np.testing.assert_array_equal(to_np(dkey), key,
                                              err_msg=f"valuation {k}")
        ref, out = _solve_both(g, host_reduced_list=True)
        _assert_solve_equal(ref, out)


def test_memory_cache_reuse_and_release(pglib):
    """Freed games leave their memory to a per-device cache that later
    loads reuse: games of changing sizes, one after another, each equal to
    the oracle; after pg_release_cache loads still work."""
    from paper_1705_02313_amd import pg
    for i, n in enumerate([5000, 800, 12000, 800, 5000]):
        g = synth.random_game(n, 2, 6, 300 + i)
        _say("cache reuse", n)
        ref, out = _solve_both(g)
        _assert_solve_equal(ref, out)
        if i == 2:
            pg.release_cache()
    pg.release_cache()
    g = synth.chain_game(3000, 9)
    ref, out = _solve_both(g)
    _assert_solve_equal(ref, out)


def test_cache_release_with_a_game_still_loaded(pglib):
    """pg_release_cache while a game is loaded keeps the slabs that game's
    blocks live in; both games still solve like the oracle, and once every
    game is freed and the cache released the device memory is back."""
    import torch
    from paper_1705_02313_amd import pg
    pg.release_cache()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    g1 = synth.random_game(20000, 2, 6, 401)
    g2 = synth.random_game(9000, 2, 6, 402)
    d1 = Game.from_dict(g1)
    with Game.from_dict(g2):
        pass                      # its blocks go back to the cache
    pg.release_cache()            # d1's slabs stay, with their free blocks
    out1 = d1.solve()
    _assert_solve_equal(orc.solve(g1), out1)
    ref2, out2 = _solve_both(g2)  # reuses the cached blocks
    _assert_solve_equal(ref2, out2)
    d1.free()
    pg.release_cache()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (64 << 20), (free0, free1)
