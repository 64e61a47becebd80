"""Count valuations on the device (games whose priorities repeat) against
the count-valuation oracle, through the C ABI: valuations along the
oracle's trajectory (counts and top flags, element by element), whole
solves (strategies, winners, iteration and switch counts) for every count
row width, the forced mode on distinct priorities, the host-driven walk
path, deep lists and the error paths."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import (PG_BR_BELLMAN_FORD, PG_BR_SI_RESET,
                                     PG_EINVAL, Game, PgError)
from tests.helpers import dense_oracle_trajectory, off_row_tau, to_np

pytestmark = pytest.mark.gpu


def _check_solve(g, **kw):
    ref = orc.dense_solve(g)
    assert ref["status"] == orc.OK
    with Game.from_dict(g, **kw) as d:
        assert d.d == ref["values"].size
        np.testing.assert_array_equal(d.values, ref["values"])
        out = d.solve()
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
    st = out["stats"]
    assert st["n_major"] == ref["n_major"]
    assert st["n_valuations"] == ref["n_valuations"]
    assert st["n_odd_switches"] == ref["n_odd_switches"]
    assert st["n_even_switches"] == ref["n_even_switches"]
    return out


@pytest.mark.parametrize("n,d,seed", [(300, 2, 1), (5000, 3, 2),
                                      (20000, 4, 3), (3000, 7, 4)])
def test_count_valuations_along_trajectory(n, d, seed):
    g = synth.few_priorities_game(n, 2, 5, d, seed)
    aug = orc.dense_preprocess(g)
    with Game.from_dict(g) as dev:
        assert dev.n_aug == aug["n"]
        for i, (sigma, tau, counts, top) in enumerate(
                dense_oracle_trajectory(aug, max_vals=12)):
            c, t, nf = dev.valuation_counts(sigma, tau)
            np.testing.assert_array_equal(to_np(t), top, err_msg=f"val {i}")
            np.testing.assert_array_equal(to_np(c), counts,
                                          err_msg=f"val {i}")
            assert nf == int((top == 0).sum()) + 1


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8, 9, 16, 17, 31])
def test_count_solve_every_row_width(d):
    g = synth.few_priorities_game(4000, 1, 6, d, 100 + d)
    _check_solve(g)


@pytest.mark.parametrize("seed", range(6))
def test_count_solve_small_ragged(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    g = synth.few_priorities_game(n, 1, 4, int(rng.integers(2, 5)),
                                  200 + seed)
    _check_solve(g)


def test_count_solve_midsize():
    g = synth.few_priorities_game(300_000, 2, 8, 4, 77)
    _check_solve(g)


def test_count_solve_deep_chain():
    """A chain game with few priorities: Euler lists as deep as the game."""
    g = synth.chain_game(200_000, 91)
    g["pri"] = np.random.default_rng(91).integers(0, 3, g["n"]).astype(
        np.int32)
    _check_solve(g)


def test_count_forced_on_distinct_priorities():
    g = synth.random_game(24, 1, 3, 5)
    _check_solve(g, count_valuation=True)


def test_count_careful_walks():
    g = synth.few_priorities_game(30000, 2, 6, 4, 8)
    _check_solve(g, careful_walks=True)


def test_count_device_pointers():
    g = synth.few_priorities_game(10000, 2, 5, 3, 9)
    ref = orc.dense_solve(g)
    with Game.from_dict(g, device=True) as d:
        out = d.solve()
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])


def test_count_errors():
    g = synth.few_priorities_game(2000, 2, 4, 40, 10)
    with pytest.raises(PgError) as e:
        Game.from_dict(g)
    assert e.value.status == PG_EINVAL
    h = synth.few_priorities_game(500, 2, 4, 3, 11)
    with Game.from_dict(h) as d:
        sigma, tau = d.initial_strategies()
        with pytest.raises(PgError) as e:
            d.valuation(sigma, tau)
        assert e.value.status == PG_EINVAL
        t2, key, nv = d.best_response(sigma, tau)
        assert key is None and nv >= 1
    # rank games reject the count entry point
    r = synth.random_game(500, 2, 4, 12)
    with Game.from_dict(r) as d:
        assert d.d == 0
        sigma, tau = d.initial_strategies()
        with pytest.raises(PgError) as e:
            d.valuation_counts(sigma, tau)
        assert e.value.status == PG_EINVAL


def test_count_all_top_and_single_vertices():
    # every play infinite: Even vertices on even self-loops
    g = {"n": 3, "m": 3, "offsets": np.array([0, 1, 2, 3]),
         "targets": np.array([0, 1, 2], np.int32),
         "owner": np.array([0, 0, 1], np.uint8),
         "pri": np.array([2, 2, 2], np.int32)}
    out = _check_solve(g)
    np.testing.assert_array_equal(to_np(out["winner"]), [0, 0, 0])
    for owner, pri in [(0, 0), (0, 1), (1, 2), (1, 3)]:
        one = {"n": 1, "m": 1, "offsets": np.array([0, 1]),
               "targets": np.array([0], np.int32),
               "owner": np.array([owner], np.uint8),
               "pri": np.array([pri], np.int32)}
        _check_solve(one, count_valuation=True)


def test_count_sparse_huge_priorities():
    """Repeated priorities far above 32 n take the sorting repeat check."""
    g = synth.few_priorities_game(3000, 1, 5, 3, 13)
    g["pri"] = np.array([0, 1 << 29, (1 << 29) + 1], np.int32)[g["pri"]]
    out = _check_solve(g)
    with Game.from_dict(g) as d:
        assert d.d >= 3 and d.values[-1] >= (1 << 29)
    assert out["stats"]["n_valuations"] >= 1


@pytest.mark.parametrize("br", [PG_BR_SI_RESET, PG_BR_BELLMAN_FORD])
@pytest.mark.parametrize("n,d,seed", [(500, 2, 21), (20000, 4, 22),
                                      (5000, 9, 23)])
def test_count_best_response_variants(br, n, d, seed):
    """SI-Reset and Bellman-Ford (section 6's best-response comparison)
    against the oracle: strategies, winners, outer iterations, and the
    number of valuations (SI-Reset) or Bellman-Ford rounds."""
    g = synth.few_priorities_game(n, 2, 5, d, seed)
    ref = orc.dense_solve(g, br=br)
    assert ref["status"] == orc.OK
    with Game.from_dict(g) as dev:
        out = dev.solve(best_response=br)
    np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
    np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
    np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
    assert out["stats"]["n_major"] == ref["n_major"]
    assert out["stats"]["n_valuations"] == ref["n_valuations"]


def test_rank_si_reset_and_bellman_ford_errors():
    g = synth.random_game(3000, 2, 5, 24)
    ref = orc.solve(g, reset=True)
    with Game.from_dict(g) as dev:
        out = dev.solve(best_response=PG_BR_SI_RESET)
        np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
        np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
        np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
        assert out["stats"]["n_valuations"] == ref["n_valuations"]
        with pytest.raises(PgError) as e:
            dev.solve(best_response=PG_BR_BELLMAN_FORD)
        assert e.value.status == PG_EINVAL
        with pytest.raises(PgError) as e:
            dev.solve(best_response=7)
        assert e.value.status == PG_EINVAL


def test_count_best_response_from_strategy_outside_rows():
    """As the rank test: Odd choices outside their rows are compared by
    their own count rows, as the oracle does."""
    g = synth.few_priorities_game(3000, 2, 5, 4, 21)
    aug = orc.dense_preprocess(g)
    sigma, tau = orc.initial_strategies(aug)
    tau = off_row_tau(aug, tau, 200, 2)
    t = tau.copy()
    nval = 0
    while True:
        succ = np.where(aug["owner"] == 1, t, sigma).astype(np.int32)
        counts, top, values, rc = orc.dense_valuation(succ, aug["pri"])
        assert rc == 0
        nval += 1
        t, c = orc.dense_odd_switch(aug, counts, top, values, t)
        if c == 0:
            break
    with Game.from_dict(g) as dev:
        assert dev.d == values.size
        dtau, key, dn = dev.best_response(sigma, tau)
    assert key is None
    np.testing.assert_array_equal(to_np(dtau), t)
    assert dn == nval
