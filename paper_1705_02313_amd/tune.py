"""Measures the tuning table of the rank valuation on this GPU.

    python -m paper_1705_02313_amd.tune --out tune.json [--classes ...]
    python -m paper_1705_02313_amd.tune --apply tune.json

For each size class a random game (out-degree uniform in [2, 5], seeded) of
about the class's size is loaded and solved under candidate parameters:
starting from the library's current entry, one parameter at a time takes
each of its candidate values and keeps the fastest (median wall time of the
solve over `--reps` runs); two sweeps over the parameters.  Every candidate
must reproduce the first solve's winners, strategies and counts, which the
script checks (the parameters only change how the work is split).
--apply rewrites the table between the BEGIN/END TABLE markers of
csrc/pg_tune.hip; rebuild the library afterwards.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_SRC = os.path.join(HERE, "csrc", "pg_tune.hip")

CANDIDATES = {
    "stride0": [8, 16, 32, 64],
    "per_thread": [1, 2, 4, 8],
    "walk_full": [8, 12, 16, 24, 32],
    "walk_round": [32, 64, 128],
    "walk_rounds": [2, 3, 4],
    "walk_block": [64, 128, 256],
}
# (lower bound of n_aug, vertices of the measured game); a game of n
# vertices has about 1.33 n after the admissibility preprocessing
CLASSES = [(0, 1000), (4096, 6000), (32768, 40000), (262144, 300000),
           (1048576, 1000000), (4194304, 4000000), (8388608, 10000000)]


def _solve(g, reps):
    import torch
    ts = []
    out = g.solve()   # untimed: captures the iteration graphs again
    torch.cuda.synchronize()
    for _ in range(reps):
        out = g.solve()
        torch.cuda.synchronize()
        ts.append(out["stats"]["seconds"])
    return statistics.median(ts), out


def _same(a, b) -> bool:
    return (all(np.array_equal(np.asarray(a[k]), np.asarray(b[k]))
                for k in ("winner", "sigma", "tau")) and
            all(a["stats"][k] == b["stats"][k]
                for k in ("n_major", "n_valuations", "n_odd_switches",
                          "n_even_switches")))


def tune_class(n: int, reps: int, sweeps: int, log) -> dict:
    import torch
    from . import synth
    from .pg import Game
    game = synth.random_game(n, 2, 5, 9000 + n % 997)
    arrs = {k: torch.from_numpy(np.ascontiguousarray(game[k])).cuda()
            for k in ("offsets", "targets", "owner", "pri")}
    g = Game(arrs["offsets"], arrs["targets"], arrs["owner"], arrs["pri"],
             n=n)
    try:
        best = g.tuning()
        t_best, ref = _solve(g, reps)
        ref = {"winner": ref["winner"].cpu().numpy(),
               "sigma": ref["sigma"].cpu().numpy(),
               "tau": ref["tau"].cpu().numpy(), "stats": ref["stats"]}
        t0 = t_best
        tried = []
        for _ in range(sweeps):
            for name, values in CANDIDATES.items():
                for v in values:
                    if v == best[name]:
                        continue
                    cand = dict(best, **{name: v})
                    g.set_tuning(**cand)
                    t, out = _solve(g, reps)
                    got = {"winner": out["winner"].cpu().numpy(),
                           "sigma": out["sigma"].cpu().numpy(),
                           "tau": out["tau"].cpu().numpy(),
                           "stats": out["stats"]}
                    if not _same(got, ref):
                        raise RuntimeError(f"tuning {cand} changed the result")
                    tried.append((cand, t))
                    if t < t_best:
                        t_best, best = t, cand
                g.set_tuning(**best)
            log(f"n={n} n_aug={g.n_aug}: {t0 * 1e3:.2f} -> "
                f"{t_best * 1e3:.2f} ms  {best}")
        return {"n": n, "n_aug": g.n_aug, "start_ms": t0 * 1e3,
                "best_ms": t_best * 1e3, "best": best,
                "candidates": len(tried),
                "valuations": int(ref["stats"]["n_valuations"])}
    finally:
        g.free()


def apply(path: str):
    with open(path) as f:
        res = json.load(f)
    rows = []
    for lo, r in sorted(res["classes"].items(), key=lambda kv: int(kv[0])):
        b = r["best"]
        rows.append(f"    {{{int(lo)}, {{{b['stride0']}, {b['per_thread']}, "
                    f"{b['walk_full']}, {b['walk_round']}, "
                    f"{b['walk_rounds']}, {b['walk_block']}}}}},")
    src = open(TABLE_SRC).read()
    a = src.index("// BEGIN TABLE")
    z = src.index("// END TABLE")
    head = src[:a] + "// BEGIN TABLE (tune.py)\nconst TuneEntry kTuneTable[] = {\n"
    src = head + "\n".join(rows) + "\n};\n" + src[z:]
    with open(TABLE_SRC, "w") as f:
        f.write(src)
    print(f"wrote {len(rows)} entries to {TABLE_SRC}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--apply", default=None)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--sweeps", type=int, default=2)
    ap.add_argument("--classes", type=int, nargs="*", default=None,
                    help="indices into the class list (default: all)")
    args = ap.parse_args()
    if args.apply:
        apply(args.apply)
        return
    import torch
    torch.cuda.set_device(0)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    picks = args.classes if args.classes is not None else range(len(CLASSES))
    res = {"gpu": torch.cuda.get_device_name(0), "reps": args.reps,
           "sweeps": args.sweeps, "classes": {}}
    for i in picks:
        lo, n = CLASSES[i]
        res["classes"][str(lo)] = tune_class(n, args.reps, args.sweeps, log)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
