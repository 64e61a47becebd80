"""The multi-core CPU-LR baseline (baselines/cpu_lr.c) against the oracle:
the same keys along whole oracle trajectories, the same Odd switches."""
from __future__ import annotations

import numpy as np
import pytest

from baselines import cpu_lr
from oracle import orc
from paper_1705_02313_amd import synth
from tests.helpers import oracle_trajectory


@pytest.mark.parametrize("kind,n,seed", [("rnd", 12, 1), ("rnd", 1000, 2),
                                         ("rnd", 20000, 3), ("chain", 3000, 4),
                                         ("chain", 17, 5)])
def test_cpu_lr_keys_match_oracle(kind, n, seed):
    g = synth.random_game(n, 2, 5, seed) if kind == "rnd" else \
        synth.chain_game(n, seed)
    aug = orc.preprocess(g)
    own = np.asarray(aug["owner"])
    by_pri, by_signed = cpu_lr.orders(aug["pri"])
    for k, (sigma, tau, key) in enumerate(oracle_trajectory(aug)):
        succ = np.where(own == 1, tau, sigma).astype(np.int32)
        for threads in (1, 4):
            ckey, nf, rc = cpu_lr.valuation(succ, aug["pri"], by_pri,
                                            by_signed, threads)
            assert rc == 0
            np.testing.assert_array_equal(ckey, key, err_msg=f"val {k}")
            assert nf == int((key != orc.KEY_TOP).sum())
        t1, c1 = orc.odd_switch(aug, key, tau)
        t2, c2 = cpu_lr.odd_switch(aug, key, tau, 4)
        np.testing.assert_array_equal(t1, t2)
        assert c1 == c2


def test_cpu_lr_reports_an_odd_cycle():
    # two Odd vertices in a cycle whose largest priority is odd
    succ = np.array([1, 0], np.int32)
    pri = np.array([3, 2], np.int32)
    _, _, rc = cpu_lr.valuation(succ, pri)
    assert rc == 2
