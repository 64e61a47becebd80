"""The tuning table and pg_set_tuning change how a valuation's work is split
and scheduled, never its result: every table entry and the extreme values
of every parameter give the same valuations (per-valuation key hashes),
strategies, winners and counts as the oracle on the same games."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import (PG_EINVAL, Game, PgError, tuning_table)
from tests.helpers import np_hash, to_np

pytestmark = pytest.mark.gpu

EXTREMES = [dict(stride0=8), dict(stride0=64), dict(per_thread=8),
            dict(walk_full=2), dict(walk_round=8, walk_rounds=1),
            dict(walk_block=64), dict(walk_full=64, walk_round=256,
                                      walk_rounds=8),
            dict(stride0=8, per_thread=1, walk_full=3, walk_round=8,
                 walk_rounds=2, walk_block=128)]


def _trace_keys(g):
    """Per-valuation key hashes of a solve from the initial strategies."""
    out = g.solve(trace=512)
    return out, [int(x) for x in out["trace"]["key_hash"]]


@pytest.mark.parametrize("kind", ["random", "chain"])
def test_every_tuning_gives_the_same_solve(kind):
    game = (synth.random_game(20000, 2, 6, 81) if kind == "random"
            else synth.chain_game(8000, 82))
    ref = orc.solve(game)
    with Game.from_dict(game) as g:
        tunings = [t for _, t in tuning_table()]
        tunings += [dict(tunings[0], **e) for e in EXTREMES]
        base = None
        for t in tunings:
            print(kind, t, flush=True)
            g.set_tuning(**t)
            assert g.tuning() == t
            out, keys = _trace_keys(g)
            np.testing.assert_array_equal(to_np(out["winner"]), ref["winner"])
            np.testing.assert_array_equal(to_np(out["sigma"]), ref["sigma"])
            np.testing.assert_array_equal(to_np(out["tau"]), ref["tau_orig"])
            assert out["stats"]["n_valuations"] == ref["n_valuations"]
            if base is None:
                base = keys
            assert keys == base


def test_table_applies_by_size_and_rejects_bad_values():
    table = tuning_table()
    game = synth.random_game(3000, 2, 5, 83)
    with Game.from_dict(game) as g:
        want = [t for lo, t in table if lo <= g.n_aug][-1]
        assert g.tuning() == want
        for bad in (dict(stride0=4), dict(stride0=48), dict(per_thread=3),
                    dict(walk_full=1), dict(walk_round=300),
                    dict(walk_rounds=0), dict(walk_block=512)):
            with pytest.raises(PgError) as e:
                g.set_tuning(**bad)
            assert e.value.status == PG_EINVAL
        assert g.tuning() == want
    dense = synth.few_priorities_game(2000, 2, 5, 4, 84)
    with Game.from_dict(dense) as g:
        with pytest.raises(PgError) as e:
            g.set_tuning(stride0=16)
        assert e.value.status == PG_EINVAL
