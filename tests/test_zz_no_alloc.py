"""pg_solve_noalloc (load, solve and release from the library's static
scratch, no allocation) against pg_load_csr + pg_solve on the same games:
two calls in a row, the second with a smaller game, so that the second runs
on scratch the first left behind; host and device arrays; the largest game
the limits allow; a game with repeated priorities; the size limits."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import (PG_EINVAL, PG_NOALLOC_MAX_EDGES,
                                     PG_NOALLOC_MAX_VERTICES, Game, PgError,
                                     solve_noalloc)
from tests.helpers import to_np

pytestmark = pytest.mark.gpu


def _same(a, b):
    for k in ("winner", "sigma", "tau"):
        np.testing.assert_array_equal(to_np(a[k]), to_np(b[k]), err_msg=k)
    for k in ("n_aug", "m_aug", "n_major", "n_valuations", "n_odd_switches",
              "n_even_switches"):
        assert a["stats"][k] == b["stats"][k], k


@pytest.mark.parametrize("device", [False, True])
def test_two_calls_in_a_row_match_load_and_solve(device):
    import torch
    big = synth.random_game(50000, 2, 8, 71)
    small = synth.random_game(3000, 2, 5, 72)
    for g in (big, small):
        print("noalloc n =", g["n"], "device =", device, flush=True)
        got = solve_noalloc(g, device=device)
        torch.cuda.synchronize()
        with Game.from_dict(g, device=device) as d:
            ref = d.solve()
        torch.cuda.synchronize()
        _same(got, ref)
        np.testing.assert_array_equal(to_np(got["winner"]),
                                      orc.solve(g)["winner"])


def test_largest_game_within_the_limits():
    n = PG_NOALLOC_MAX_VERTICES
    g = synth.random_game(n, 13, 17, 73)
    assert g["m"] <= PG_NOALLOC_MAX_EDGES
    print("noalloc largest: n =", n, "m =", g["m"], flush=True)
    got = solve_noalloc(g)
    with Game.from_dict(g) as d:
        ref = d.solve()
    _same(got, ref)
    # then a smaller one on what the large one left
    g2 = synth.chain_game(5000, 74)
    got2 = solve_noalloc(g2, keep_dummies=True)
    with Game.from_dict(g2) as d:
        ref2 = d.solve(keep_dummies=True)
    _same(got2, ref2)


def test_repeated_priorities():
    g = synth.few_priorities_game(20000, 2, 6, 4, 75)
    got = solve_noalloc(g)
    with Game.from_dict(g) as d:
        ref = d.solve()
    _same(got, ref)
    ref_o = orc.dense_solve(g)
    np.testing.assert_array_equal(to_np(got["winner"]), ref_o["winner"])


def test_limits_are_checked_on_the_host():
    g = synth.random_game(PG_NOALLOC_MAX_VERTICES + 1, 2, 3, 76)
    with pytest.raises(PgError) as e:
        solve_noalloc(g)
    assert e.value.status == PG_EINVAL
    g = synth.random_game(1000, 2, 3, 77)
    g["m"] = PG_NOALLOC_MAX_EDGES + 1   # only the count is looked at first
    with pytest.raises(PgError) as e:
        solve_noalloc({**g, "targets": np.zeros(PG_NOALLOC_MAX_EDGES + 1,
                                                np.int32)})
    assert e.value.status == PG_EINVAL
