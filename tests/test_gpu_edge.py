"""Edge cases and error paths of the device path, through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import (PG_EINADMISSIBLE, PG_EINVAL,
                                     PG_EITERLIMIT, Game, PgError)
from tests.helpers import to_np

pytestmark = pytest.mark.gpu


def _game(rows, owner, pri, off_dtype=np.int64):
    off = np.zeros(len(rows) + 1, off_dtype)
    off[1:] = np.cumsum([len(r) for r in rows])
    return {"n": len(rows), "m": int(off[-1]), "offsets": off,
            "targets": np.array([t for r in rows for t in r], np.int32),
            "owner": np.array(owner, np.uint8),
            "pri": np.array(pri, np.int32)}


def _check_solve(g, **kw):
    ref = orc.solve(g, **kw)
    assert ref["status"] == 0
    with Game.from_dict(g, preprocess=kw.get("preprocess_game", True)) as d:
        out = d.solve()
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
    assert out["stats"]["n_major"] == ref["n_major"]
    assert out["stats"]["n_valuations"] == ref["n_valuations"]
    return out


@pytest.mark.parametrize("owner,pri", [(0, 0), (0, 1), (1, 2), (1, 3)])
def test_single_vertex_self_loop(owner, pri):
    out = _check_solve(_game([[0]], [owner], [pri]))
    assert to_np(out["winner"])[0] == pri % 2


def test_two_vertices_and_repeated_edges():
    _check_solve(_game([[1, 1, 0], [0, 0]], [0, 1], [3, 4]))
    _check_solve(_game([[1, 1, 0], [0, 0]], [1, 1], [3, 4]))
    _check_solve(_game([[0, 1], [1, 0, 1]], [1, 0], [0, 5]))


def test_all_even_all_odd_all_top():
    g = synth.random_game(500, 2, 5, 3)
    for own in (0, 1):
        h = dict(g)
        h["owner"] = np.full(g["n"], own, np.uint8)
        _check_solve(h)
    # every vertex Even with an even self-loop: Even wins everywhere
    n = 300
    rows = [[v, (v + 1) % n] for v in range(n)]
    pri = 2 * np.random.default_rng(1).permutation(n)
    out = _check_solve(_game(rows, [0] * n, pri))
    assert (to_np(out["winner"]) == 0).all()


def test_int32_offsets_same_as_int64():
    g = synth.random_game(4000, 2, 6, 21)
    h = dict(g)
    h["offsets"] = g["offsets"].astype(np.int32)
    with Game.from_dict(g) as a, Game.from_dict(h) as b:
        ra, rb = a.solve(), b.solve()
    for k in ("winner", "sigma", "tau"):
        np.testing.assert_array_equal(ra[k], rb[k])


def test_large_priorities():
    rng = np.random.default_rng(4)
    g = synth.random_game(2000, 2, 5, 4)
    g["pri"] = (rng.choice(2**30, size=2000, replace=False) + 2**30 - 5000
                ).astype(np.int32)
    _check_solve(g)


def test_priority_overflow_after_shift_rejected():
    g = synth.random_game(200, 2, 5, 8)
    g["pri"] = g["pri"].copy()
    g["pri"][0] = 2**31 - 2          # the preprocessing shift overflows int32
    with pytest.raises(PgError) as e:
        Game.from_dict(g)
    assert e.value.status == PG_EINVAL


@pytest.mark.parametrize("fault", ["decreasing", "terminal", "target",
                                   "owner", "negative", "duplicate",
                                   "last_offset"])
def test_invalid_games_rejected(fault):
    g = synth.random_game(100, 2, 5, 9)
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v)
         for k, v in g.items()}
    if fault == "decreasing":
        g["offsets"][5] = g["offsets"][7]
    elif fault == "terminal":
        g["offsets"][6] = g["offsets"][5]
    elif fault == "target":
        g["targets"][3] = 100
    elif fault == "owner":
        g["owner"][2] = 2
    elif fault == "negative":
        g["pri"][1] = -1
    elif fault == "duplicate":
        g["pri"][1] = g["pri"][2]
    elif fault == "last_offset":
        g["offsets"][-1] -= 1
    with pytest.raises(PgError) as e:
        Game.from_dict(g)
    assert e.value.status == PG_EINVAL


def test_iteration_caps():
    g = synth.random_game(3000, 2, 5, 2)
    with Game.from_dict(g) as d:
        with pytest.raises(PgError) as e:
            d.solve(max_inner=1)
        assert e.value.status == PG_EITERLIMIT
        with pytest.raises(PgError) as e:
            d.solve(max_major=1)
        assert e.value.status == PG_EITERLIMIT
        # the game is still usable afterwards
        ref = orc.solve(g)
        np.testing.assert_array_equal(d.solve()["winner"], ref["winner"])


def test_inadmissible_without_preprocessing():
    # two Odd vertices on an odd cycle (largest priority 3)
    g = _game([[1], [0]], [1, 1], [3, 0])
    with Game.from_dict(g, preprocess=False) as d:
        with pytest.raises(PgError) as e:
            d.solve()
        assert e.value.status == PG_EINADMISSIBLE
        sigma, tau = d.initial_strategies()
        with pytest.raises(PgError) as e:
            d.valuation(sigma, tau)
        assert e.value.status == PG_EINADMISSIBLE
    # with preprocessing the same game solves, Odd wins both
    out = _check_solve(g)
    assert (to_np(out["winner"]) == 1).all()


def test_bad_strategy_entries_rejected():
    g = synth.random_game(50, 2, 3, 1)
    with Game.from_dict(g) as d:
        sigma, tau = d.initial_strategies()
        odd = np.flatnonzero(d.export()["owner"] == 1)
        tau = tau.copy()
        tau[odd[0]] = -1                      # Odd cannot choose the sink
        with pytest.raises(PgError) as e:
            d.valuation(sigma, tau)
        assert e.value.status == PG_EINVAL
        sigma = sigma.copy()
        sigma[0 if d.export()["owner"][0] == 0 else odd[0]] = d.n_aug
        tau[odd[0]] = d.n_aug                 # out of range
        with pytest.raises(PgError):
            d.valuation(sigma, tau)


def test_deterministic_repeats():
    g = synth.random_game(30000, 2, 8, 31)
    with Game.from_dict(g) as d:
        a = d.solve()
        b = d.solve()
    for k in ("winner", "sigma", "tau"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("n,careful", [(1000, False), (200_000, False),
                                       (2_000_000, False), (200_000, True)])
def test_deep_list_valuation(n, careful):
    """One play through every vertex (the chain i -> i+1, each dummy to its
    w, one Even vertex to the sink): an Euler list as long as the game."""
    g = synth.chain_game(n, 77)
    aug = orc.preprocess(g)
    N = aug["n"]
    off, tgt, own = aug["offsets"], aug["targets"], aug["owner"]
    nxt = np.empty(N, np.int32)
    for_chain = (np.arange(g["n"]) + 1) % g["n"]
    # the successor along the chain (through the dummy when there is one)
    # is the first or the second entry of each row
    first = tgt[off[:-1]]
    second = np.where(np.diff(off) > 1, tgt[np.minimum(off[:-1] + 1,
                                                       len(tgt) - 1)], -1)
    n0 = g["n"]
    dummy_of = aug["dummy_of"]
    target_of = np.arange(N)
    target_of[n0:] = dummy_of           # what each vertex stands for
    want = np.concatenate([for_chain, dummy_of]).astype(np.int64)
    pick_first = target_of[first] == want
    nxt[:] = np.where(pick_first, first, second)
    assert (target_of[nxt] == want).all()
    sigma = np.where(own == 0, nxt, -1).astype(np.int32)
    tau = np.where(own == 1, nxt, -1).astype(np.int32)
    even = np.flatnonzero(own[:n0] == 0)
    sigma[even[len(even) // 2]] = -1     # one Even vertex ends the play
    succ = np.where(own == 1, tau, sigma).astype(np.int32)
    key, nf, rc = orc.valuation(succ, aug["pri"])
    assert rc == 0
    with Game.from_dict(g, careful_walks=careful) as d:
        dkey, dnf = d.valuation(sigma, tau)
    assert dnf == nf
    np.testing.assert_array_equal(to_np(dkey), key)


@pytest.mark.parametrize("g", [synth.random_game(20000, 2, 6, 41),
                               synth.chain_game(30000, 42)],
                         ids=["random", "chain"])
def test_careful_walks_same_results(g):
    """The host-driven walk rounds (the fallback of the fixed device rounds)
    give the oracle's results on whole solves."""
    ref = orc.solve(g)
    assert ref["status"] == 0
    with Game.from_dict(g, careful_walks=True) as d:
        out = d.solve()
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
    assert out["stats"]["n_valuations"] == ref["n_valuations"]
