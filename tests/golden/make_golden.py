"""Writes the stored expected values for the full-size workloads.

Calls only the CPU oracle (oracle/orc.py) on inputs from the seeded
generators; nothing here touches the GPU path.  Each file golden_<name>.json
holds sizes, iteration counts, the hash (tests/helpers.np_hash, identical to
orc_hash) of the final winner/sigma/tau/key arrays and the hash of every
valuation's key array in order.

    python tests/golden/make_golden.py c1 c2 c3 c0s
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import orc  # noqa: E402
from paper_1705_02313_amd import synth  # noqa: E402


def record(game: dict) -> dict:
    t0 = time.perf_counter()
    r = orc.solve(game, trace=True)
    dt = time.perf_counter() - t0
    assert r["status"] == 0
    aug = r["aug"]
    return {
        "n": int(game["n"]), "m": int(game["m"]),
        "n_aug": int(aug["n"]), "m_aug": int(aug["m"]),
        "n_major": r["n_major"], "n_valuations": r["n_valuations"],
        "n_odd_switches": r["n_odd_switches"],
        "n_even_switches": r["n_even_switches"],
        "w_even": int((r["winner"] == 0).sum()),
        "winner_hash": orc.key_hash(r["winner"].astype(np.int32)),
        "sigma_hash": orc.key_hash(r["sigma"]),
        "tau_hash": orc.key_hash(r["tau"]),
        "key_hash": orc.key_hash(r["key"]),
        "trace": [int(x) for x in r["trace"]],
        "oracle_seconds": round(dt, 2),
    }


def main(names):
    for name in names:
        if name == "c0s":
            out = {str(s): record(synth.random_game(1000, 2, 5, s))
                   for s in range(20)}
        else:
            cfg = int(name[1:])
            out = record(synth.config_game(cfg))
        path = os.path.join(HERE, f"golden_{name}.json")
        with open(path, "w") as f:
            json.dump({"workload": name, "source": "oracle/orc.c via "
                       "tests/golden/make_golden.py", "data": out}, f)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c0s", "c1", "c2", "c3"])
