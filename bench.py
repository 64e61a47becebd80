"""Benchmark: greedy all-switches strategy improvement on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

A step is one whole job on the workload's game, whose arrays already sit in
HBM when the timed region starts: pg_load_csr (validation, the admissibility
preprocessing, the signed-priority order) + pg_solve (every best-response
iteration and every Even switch until no switch) + pg_free.  The headline
value is edges per second per best-response iteration,
    m * n_valuations / (seconds per step),
m being the original game's edge count.

Workloads (seeded, synthetic; see paper_1705_02313_amd/synth.py):
  c2  random game, n = 10,000,000, out-degree U[2,5], int64 offsets (default)
  c1  random game, n = 1,000,000, out-degree U[2,10]
  c3  long-chain game, n = 8,000,000
  c0  random game, n = 1,000, out-degree U[2,5]
  d4  random game, n = 10,000,000, out-degree U[2,5], priorities drawn from
      4 values: count valuations, the paper's regime (2 to 4 priorities)
  d4s the same with n = 1,000,000, out-degree U[2,10]
  c4  batched/served mix: 1,024 random games, n log-uniform in [1e3, 2e5],
      out-degree U[2,8]; games/s one at a time (pg_load_csr + pg_solve each),
      batched with every game present at the start (the calibration rate mu),
      and served as a Poisson stream at 1.5 mu under an arena budget of a
      quarter of the mix's modified vertices (latency p50/p99)

Printed: one JSON line with the driver's fields plus
  "roofline"   the best-response iteration (one replay of its HIP graph:
               walks, valuation, All_Odd) as the unit: the method's least
               bytes per iteration (CSR offsets and targets, one key gather
               per edge, 25 B per vertex, 12 B per element of a 2n'-element
               Euler list) over the iteration's average device time, taken
               with HIP events on the solve's stream around every iteration
               of the timed steps, against 8 TB/s; "traffic" is the
               rocprofv3 counter bytes per iteration (FETCH_SIZE +
               WRITE_SIZE scaled on a plain copy: bytes through the L2's
               fabric port, Infinity Cache hits included, so an upper bound
               on HBM bytes) when they were taken on the current sources
  "dominant_kernel"  the kernel with the largest summed time in up to two
               profiled steps after the timed steps, its own algorithmic
               bytes over its event-timed duration
  "iteration_bytes"  every kernel's algorithmic bytes per iteration, the
               counter bytes, a measured 1 GiB copy rate
  "mix"        (c2 runs, unless --no-mix) the 1,024-game batched/served
               workload: games/s one at a time, batched and served, p50/p99
               latency, identical results, a roofline fraction and the CPU
               oracle on a sample of the mix
  "cpu_baseline"  the CPU oracle timed on this host, pinned to one core, on
               a bounded sample of the same workload, with
               "cpu_lr_baseline" beside it for rank valuations (the
               multi-core CPU-LR baseline on the same sample)
and on c3 "deep_list_valuation" (one valuation of a play through every
vertex).  --best-response picks the best responses
(section 6's comparison: SI, SI-Reset, Bellman-Ford on count games).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c0": ("random parity game n=1000 deg U[2,5]", 0),
    "c1": ("random parity game n=1000000 deg U[2,10]", 1),
    "c2": ("random parity game n=10000000 deg U[2,5] int64 offsets", 2),
    "c3": ("long-chain parity game n=8000000", 3),
    "c4": ("1024 random parity games, n log-uniform [1e3, 2e5], deg U[2,8]",
           4),
    "d4": ("random parity game n=10000000 deg U[2,5], 4 repeated priorities "
           "(count valuations)", 5),
    "d4s": ("random parity game n=1000000 deg U[2,10], 4 repeated priorities "
            "(count valuations)", 6),
}


TRAFFIC_FILES = {"c2": "traffic_random10M.json"}


# the sources of everything a single rank-valuation game's load and solve
# launch (batches, count valuations and PG_ODD_REGION live in other files)
SINGLE_GAME_SOURCES = ["pg_api.hip", "pg_common.h", "pg_prims.hip",
                       "pg_switch.hip", "pg_tune.hip", "pg_val.hip"]


def sources_sha256() -> str:
    """Hash of the kernel sources a single rank-valuation game runs and of
    the header (file names and contents), to tie stored counter readings to
    the code they measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_02313_amd", "csrc")
    files = [os.path.join(csrc, f) for f in SINGLE_GAME_SOURCES]
    files.append(os.path.join(ROOT, "include", "pg.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(workload: str, kind: str):
    """HBM bytes per launch of `kind` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by its reading on a plain
    copy), or None when there is none or the kernels changed since."""
    name = TRAFFIC_FILES.get(workload)
    if not name:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("sources_sha256") != sources_sha256():
        return None
    return t["bytes_per_launch"].get(kind)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Device-to-device copy rate on this GPU in GB/s (bytes read plus bytes
    written), the practical ceiling beside the 8 TB/s specification."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / statistics.median(ts) / 1e9


def random_gather_rate(n_words: int = 1 << 28, n_idx: int = 1 << 26,
                       reps: int = 5) -> dict:
    """Random 4-byte gathers per second from a 1 GiB array (each index
    almost surely on a line of its own), with the index reads and output
    writes (12 B per gather, coalesced) that the gather also pays: the rate
    at which a pass that touches one random line per step can run."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(12345)
    src = torch.arange(n_words, dtype=torch.int32, device="cuda")
    idx = torch.randint(0, n_words, (n_idx,), device="cuda", generator=g)
    out = src[idx]
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        torch.index_select(src, 0, idx, out=out)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    del src, idx, out
    torch.cuda.empty_cache()
    t = statistics.median(ts)
    return {"gathers_per_s": n_idx / t, "array_bytes": 4 * n_words,
            "gathers": n_idx, "seconds": t}


def traffic_summary(pmc_dir: str, workload: str = "c2") -> dict:
    """Reads four rocprofv3 --pmc runs under pmc_dir (<workload>_FETCH_SIZE,
    <workload>_WRITE_SIZE, copy_FETCH_SIZE, copy_WRITE_SIZE, each holding a
    *counter_collection.csv) and returns the counter bytes per launch by the
    library's kernel kind, each counter scaled by its reading on the plain
    copy (--copy-calibration 1024: 1 GiB read and 1 GiB written)."""
    import csv
    import glob

    def per_kernel(sub):
        files = glob.glob(os.path.join(pmc_dir, sub, "**",
                                       "*counter_collection.csv"),
                          recursive=True)
        if not files:
            raise FileNotFoundError(f"no counter CSV under {sub}")
        acc = {}
        for f in files:
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    name = row["Kernel_Name"].split("(")[0]
                    name = name.replace("void ", "").strip()
                    name = name.split("<")[0].split("::")[-1]
                    a = acc.setdefault(name, [0.0, 0])
                    a[0] += float(row["Counter_Value"])
                    a[1] += 1
        return acc

    copy_f = per_kernel("copy_FETCH_SIZE")
    copy_w = per_kernel("copy_WRITE_SIZE")
    ck = max(copy_f, key=lambda k: copy_f[k][0])
    gib = float(1 << 30)
    f_scale = gib / (copy_f[ck][0] / copy_f[ck][1] * 1024.0)
    w_scale = gib / (copy_w[ck][0] / copy_w[ck][1] * 1024.0)
    fetch = per_kernel(f"{workload}_FETCH_SIZE")
    write = per_kernel(f"{workload}_WRITE_SIZE")
    by_kind = {}
    for name, (kib, calls) in fetch.items():
        kind = KERNEL_KINDS.get(name, "other")
        wk = write.get(name, [0.0, calls])[0]
        b = by_kind.setdefault(kind, [0.0, 0, 0.0, 0.0])
        b[0] += 1024.0 * (kib * f_scale + wk * w_scale)
        b[1] += calls
        b[2] += 1024.0 * kib * f_scale
        b[3] += 1024.0 * wk * w_scale
    return {"workload": workload, "sources_sha256": sources_sha256(),
            "scale": {"FETCH_SIZE": round(f_scale, 4),
                      "WRITE_SIZE": round(w_scale, 4)},
            "bytes_per_launch": {k: round(v[0] / v[1]) for k, v in
                                 sorted(by_kind.items(),
                                        key=lambda kv: -kv[1][0])},
            "fetched_per_launch": {k: round(v[2] / v[1]) for k, v in
                                   by_kind.items()},
            "written_per_launch": {k: round(v[3] / v[1]) for k, v in
                                   by_kind.items()},
            "launches": {k: v[1] for k, v in by_kind.items()}}


# the library's kernel kinds (pg_profile_read names) of each kernel a
# rank-valuation solve launches
KERNEL_KINDS = {
    "k_ng_full": "ng_walk", "k_ng_round": "ng_round",
    "k_ng_round_list": "ng_round",
    "k_root_full": "root_walk", "k_root_round": "root_round",
    "k_root_round_list": "root_round",
    "k_ps_split": "sort_split",
    "k_1s_pass": "sort_pass", "k_scan_reduce": "scan", "k_scan_down": "scan",
    "k_scan_top": "scan", "k_link_info": "link_info",
    "k_link_build": "link_build", "k_lr_sum1": "lr_sum1",
    "k_lr_sumk": "lr_sumk", "k_lr_top": "lr_top", "k_lr_distk": "lr_distk",
    "k_lr_emit1": "lr_emit1", "k_tsw_stage": "odd_stage",
    "k_tsw_min": "odd_switch", "k_odd_switch": "odd_switch",
    "k_even_switch": "even_switch", "k_fill_i32": "fill",
    "k_fill_u8": "fill", "k_zero3": "fill", "k_1s_base": "scan",
    "k_sum_dist": "other", "k_rs_upsweep": "sort_hist",
    "k_rs_downsweep": "sort_pass",
}


def method_min_bytes(n_aug: int, m_aug: int, offset_bytes: int) -> int:
    """The method's own least I/O per best-response iteration: the CSR
    offsets and targets, one key gather per edge, per vertex its owner, its
    strategy read and written and its current choice's key (13 B) and its
    successor and priority reads and key write (12 B), and 12 B per element
    of an Euler list of 2 n' elements."""
    return (offset_bytes * (n_aug + 1) + 8 * m_aug + 25 * n_aug +
            12 * 2 * n_aug)


def deep_list_valuation(arrs, n: int, reps: int = 5) -> dict:
    """One valuation of a play through every vertex: each original vertex i
    takes the row entry standing for i + 1 (mod n; a dummy d_w stands for
    w), each dummy its only entry, and one Even vertex the sink, so the
    finite part is one list about as deep as the modified game.  Wall time
    of pg_valuation on device arrays (median of `reps`)."""
    import torch
    from paper_1705_02313_amd.pg import Game
    with Game(arrs["offsets"], arrs["targets"], arrs["owner"], arrs["pri"],
              n=n) as g:
        ex = g.export()
        off, tgt, own = ex["offsets"], ex["targets"], ex["owner"]
        N = ex["n"]
        sf = np.arange(N, dtype=np.int64)
        sf[n:] = tgt[off[n:N]]
        want = np.concatenate([(np.arange(n) + 1) % n, sf[n:]])
        src = np.repeat(np.arange(N), np.diff(off))
        hit = sf[tgt] == want[src]
        e = np.flatnonzero(hit)
        first = np.full(N, -1, np.int64)
        first[src[e][::-1]] = e[::-1]
        assert (first >= 0).all()
        nxt = tgt[first].astype(np.int32)
        sigma = np.where(own == 0, nxt, -1).astype(np.int32)
        tau = np.where(own == 1, nxt, -1).astype(np.int32)
        even = np.flatnonzero(own[:n] == 0)
        sigma[even[len(even) // 2]] = -1
        ds = torch.from_numpy(sigma).cuda()
        dt = torch.from_numpy(tau).cuda()
        _, nf = g.valuation(ds, dt)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            g.valuation(ds, dt)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
    return {"ms_median": 1e3 * statistics.median(ts), "finite": nf,
            "n_aug": int(N), "reps": reps}


class one_core:
    """Pins this process to one CPU (the first it may use) inside the block,
    so that the oracle's timing uses exactly one core; the previous
    affinity comes back at the end (no re-exec, no child process)."""

    def __enter__(self):
        self.prev = None
        try:
            self.prev = os.sched_getaffinity(0)
            self.core = min(self.prev)
            os.sched_setaffinity(0, {self.core})
        except (AttributeError, OSError):
            self.core = None
        return self

    def __exit__(self, *exc):
        if self.prev is not None:
            os.sched_setaffinity(0, self.prev)


def host_info() -> dict:
    """The host's CPU model, its logical CPU count and the CPUs this process
    may use."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu": _host_cpu(), "nproc": os.cpu_count(),
            "usable_cpus": usable}


def cpu_baseline(game: dict, iters: int = 3, counts: bool = False):
    """The CPU oracle on this host: its preprocessing, then the first `iters`
    best-response iterations (valuation + All_Odd) of Algorithm 1 (with the
    count-valuation oracle when `counts`).  For rank valuations the
    multi-core CPU-LR baseline (baselines/cpu_lr.c, the paper's CPU-LR) is
    timed on the same iterations; returns (oracle, cpu_lr or None)."""
    from oracle import orc
    with one_core() as pin:
        t0 = time.perf_counter()
        aug = orc.dense_preprocess(game) if counts else orc.preprocess(game)
        t_pre = time.perf_counter() - t0
        sigma, tau = orc.initial_strategies(aug)
        sigma0, tau0 = sigma.copy(), tau.copy()
        by_pri = None if counts else orc.order_by_pri(aug["pri"])
        times = []
        for _ in range(iters):
            t1 = time.perf_counter()
            succ = np.where(aug["owner"] == 1, tau, sigma).astype(np.int32)
            if counts:
                cnt, top, values, rc = orc.dense_valuation(succ, aug["pri"])
                tau, c = orc.dense_odd_switch(aug, cnt, top, values, tau)
            else:
                key, _, rc = orc.valuation(succ, aug["pri"], by_pri=by_pri)
                tau, c = orc.odd_switch(aug, key, tau)
            times.append(time.perf_counter() - t1)
            if c == 0:
                break
    t_iter = statistics.median(times)
    oracle = {"value": game["m"] / t_iter, "unit": "edges/s per "
              "best-response iteration", "cores": 1, "kind": "oracle",
              "sample": f"oracle preprocessing ({t_pre:.2f} s, not in value) "
                        f"then {len(times)} best-response iterations "
                        "(valuation + All_Odd) from the initial strategies, "
                        f"median {t_iter:.3f} s each, single thread pinned "
                        f"to CPU {pin.core}",
              "host": host_info()}
    lr = None
    if not counts:
        from baselines import cpu_lr
        r = cpu_lr.time_iterations(aug, sigma0, tau0, iters=len(times))
        lr = {"value": game["m"] / r["seconds_median"],
              "unit": "edges/s per best-response iteration",
              "cores": r["threads"], "kind": "cpu-lr",
              "sample": f"the same {len(times)} iterations on the same "
                        "modified game, multi-core list ranking (OpenMP), "
                        f"median {r['seconds_median']:.3f} s each"}
    return oracle, lr


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_mix(n_games: int, oracle_budget_s: float = 10.0) -> dict:
    """The batched/served workload: one-at-a-time solves, every game present
    at t = 0 (the calibration rate mu), then a Poisson stream at 1.5 mu
    under an arena budget of a quarter of the mix; the CPU oracle on the
    first games of the mix, pinned to one core, for about
    `oracle_budget_s`."""
    import torch
    from paper_1705_02313_amd import synth
    from paper_1705_02313_amd.pg import Game
    from paper_1705_02313_amd.serve import poisson_arrivals, serve

    t0 = time.perf_counter()
    games = synth.mixed_batch(n_games, 4000)
    log(f"generated {len(games)} games in {time.perf_counter() - t0:.1f}s, "
        f"sum n = {sum(g['n'] for g in games)}")
    torch.cuda.set_device(0)
    # one game at a time
    solo = []
    t0 = time.perf_counter()
    n_aug_total = m_aug_total = 0
    for g in games:
        with Game.from_dict(g) as d:
            r = d.solve()
            n_aug_total += d.n_aug
            m_aug_total += d.m_aug
        solo.append(r)
    t_solo = time.perf_counter() - t0
    log(f"one at a time: {t_solo:.2f}s, {len(games) / t_solo:.1f} games/s")

    def same(res) -> bool:
        for i, r in res["results"].items():
            a = solo[i]
            if not (np.array_equal(a["winner"], r["winner"]) and
                    np.array_equal(a["sigma"], r["sigma"]) and
                    np.array_equal(a["tau"], r["tau"]) and
                    a["stats"]["n_valuations"] == r["stats"]["n_valuations"]
                    and a["stats"]["n_major"] == r["stats"]["n_major"]):
                return False
        return len(res["results"]) == len(games)

    cap_v, cap_e = n_aug_total + 1, m_aug_total + 1
    # calibration: every game present at t = 0 (submitted before the first
    # step, so that every step holds every unfinished game)
    zeros = np.zeros(len(games))
    rb = serve(games, zeros, cap_v, cap_e, submit_thread=False)
    mu = len(games) / rb["makespan"]
    log(f"batched (all at t=0): {rb['makespan']:.2f}s, {mu:.1f} games/s, "
        f"{rb['steps']} steps")
    # served: Poisson stream at 1.5 mu, arena budget a quarter of the mix
    arr = poisson_arrivals(len(games), 1.5 * mu, 4242)
    budget_v = max(cap_v // 4, max(int(r["stats"]["n_aug"]) for r in solo) + 1)
    budget_e = max(cap_e // 4, max(int(r["stats"]["m_aug"]) for r in solo) + 1)
    # submissions between steps (a submitter thread of its own lowers the
    # latency only below the calibration rate and costs throughput above it)
    rs = serve(games, arr, budget_v, budget_e, submit_thread=False)
    lat = rs["latency"]
    served = len(games) / rs["makespan"]
    log(f"served (Poisson 1.5 mu, quarter arena): {rs['makespan']:.2f}s, "
        f"{served:.1f} games/s, p50 {np.percentile(lat, 50) * 1e3:.1f} ms, "
        f"p99 {np.percentile(lat, 99) * 1e3:.1f} ms")
    # the same stream at the calibration rate: latency below saturation
    arr1 = poisson_arrivals(len(games), mu, 4243)
    r1 = serve(games, arr1, budget_v, budget_e, submit_thread=False)
    lat1 = r1["latency"]
    log(f"served (Poisson 1.0 mu): {len(games) / r1['makespan']:.1f} "
        f"games/s, p50 {np.percentile(lat1, 50) * 1e3:.1f} ms, "
        f"p99 {np.percentile(lat1, 99) * 1e3:.1f} ms")
    ident = same(rb) and same(rs) and same(r1)
    # the method's least bytes over every iteration of every game
    mix_bytes = sum(
        method_min_bytes(int(r["stats"]["n_aug"]), int(r["stats"]["m_aug"]),
                         np.asarray(g["offsets"]).itemsize) *
        int(r["stats"]["n_valuations"]) for g, r in zip(games, solo))

    def frac(seconds):
        return round(mix_bytes / seconds / 1e9 / HBM_PEAK_GBS, 4)

    # the oracle, one game after another, on one core
    from oracle import orc
    done = 0
    with one_core() as pin:
        t0 = time.perf_counter()
        while done < len(games) and time.perf_counter() - t0 < oracle_budget_s:
            orc.solve(games[done])
            done += 1
        t_orc = time.perf_counter() - t0
    edges_done = sum(g["m"] for g in games[:done])
    edges_all = sum(g["m"] for g in games)
    return {
        "workload": WORKLOADS["c4"][0],
        "games": len(games),
        "sum_n": int(sum(g["n"] for g in games)),
        "sum_n_aug": int(n_aug_total),
        "sum_valuations": int(sum(r["stats"]["n_valuations"] for r in solo)),
        "arena_budget_vertices": int(budget_v),
        "arrivals": "Poisson, rate 1.5 x batched calibration rate",
        "served_games_per_s": served,
        "served_makespan_s": rs["makespan"],
        "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
        "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
        "batched_all_at_once_games_per_s": mu,
        "one_at_a_time_games_per_s": len(games) / t_solo,
        "speedup_served_vs_one_at_a_time": served * t_solo / len(games),
        "speedup_batched_vs_one_at_a_time": mu * t_solo / len(games),
        "identical_to_one_at_a_time": bool(ident),
        "served_steps": rs["steps"],
        "at_calibration_rate": {
            "arrivals": "Poisson, rate 1.0 x batched calibration rate",
            "served_games_per_s": len(games) / r1["makespan"],
            "latency_p50_ms": float(np.percentile(lat1, 50) * 1e3),
            "latency_p99_ms": float(np.percentile(lat1, 99) * 1e3)},
        "roofline": {"bound": "hbm", "unit": "fraction of 8 TB/s",
                     "method_min_bytes_all_games": int(mix_bytes),
                     "served_frac": frac(rs["makespan"]),
                     "batched_frac": frac(rb["makespan"]),
                     "one_at_a_time_frac": frac(t_solo)},
        "cpu_baseline": {
            "value": done / t_orc, "unit": "games/s", "cores": 1,
            "kind": "oracle",
            "sample": f"the first {done} games of the mix solved one after "
                      f"another by the oracle ({t_orc:.1f} s, pinned to CPU "
                      f"{pin.core}); {edges_done} of the mix's {edges_all} "
                      "edges",
            "host": host_info()},
    }


def bench_mix(args) -> dict:
    """The batched/served workload as the headline line."""
    mix = run_mix(args.mix_games)
    return {
        "metric": "batched games/s",
        "value": mix["served_games_per_s"],
        "unit": "games/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": mix["served_makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": mix["workload"], "games": mix["games"],
                   "sum_n": mix["sum_n"], "sum_n_aug": mix["sum_n_aug"],
                   "arena_budget_vertices": mix["arena_budget_vertices"],
                   "arrivals": mix["arrivals"]},
        **{k: v for k, v in mix.items()
           if k not in ("workload", "games", "sum_n", "sum_n_aug",
                        "arena_budget_vertices", "arrivals")},
    }


def odd_region_run(arrs, game: dict, winner_dummies, reps: int = 2) -> dict:
    """The same game loaded with PG_ODD_REGION (Odd's own winning region
    removed, no dummies): the reduced game's size and the per-iteration time
    beside the dummy path's, after one untimed run.  The winners must be
    those of the dummy path."""
    import torch
    from paper_1705_02313_amd.pg import Game
    runs = []
    for i in range(reps + 1):
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        g = Game(arrs["offsets"], arrs["targets"], arrs["owner"], arrs["pri"],
                 n=game["n"], odd_region=True)
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        out = g.solve()
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        g.free()
        if i:
            runs.append((t_b - t_a, t_c - t_b, out["stats"]))
    win = out["winner"].cpu().numpy()
    if not np.array_equal(win, winner_dummies):
        raise RuntimeError("PG_ODD_REGION winners differ from the dummy "
                           "path's")
    st = runs[0][2]
    nval = int(st["n_valuations"])
    solve_s = statistics.median(r[1] for r in runs)
    it_ev = statistics.median(r[2]["iteration_ms"] for r in runs) / max(nval,
                                                                        1)
    return {"n_aug": int(st["n_aug"]), "m_aug": int(st["m_aug"]),
            "removed": int(game["n"] - st["n_aug"]),
            "n_major": int(st["n_major"]), "n_valuations": nval,
            "load_seconds_median": statistics.median(r[0] for r in runs),
            "solve_seconds_median": solve_s,
            "ms_per_iteration": 1e3 * solve_s / max(nval, 1),
            "event_ms_per_iteration": it_ev,
            "winners_equal_dummy_path": True, "reps": reps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-kernel event profiler")
    ap.add_argument("--best-response", default="si",
                    choices=["si", "reset", "bf"],
                    help="best responses: one-player SI (Algorithm 1), "
                         "SI-Reset, or Bellman-Ford (count games)")
    ap.add_argument("--host-reduced-list", action="store_true",
                    help="rank the reduced list on the host (the paper's "
                         "GPU-LR split), to measure it against the device")
    ap.add_argument("--no-mix", action="store_true",
                    help="leave the batched/served mix out of a c2 run")
    ap.add_argument("--no-odd-region", action="store_true",
                    help="leave out the run that removes Odd's own region "
                         "instead of inserting dummies (PG_ODD_REGION)")
    ap.add_argument("--mix-games", type=int, default=1024,
                    help="games in the batched/served workload")
    ap.add_argument("--traffic-summary", metavar="PMC_DIR",
                    help="only write profiles/traffic_random10M.json from "
                         "four rocprofv3 --pmc runs under PMC_DIR (c2 and "
                         "copy runs of FETCH_SIZE and WRITE_SIZE)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 3 times (a plain "
                         "copy kernel of known size, to scale HBM counters)")
    args = ap.parse_args()
    if args.traffic_summary:
        t = traffic_summary(args.traffic_summary, "c2")
        path = os.path.join(ROOT, "profiles", TRAFFIC_FILES["c2"])
        with open(path, "w") as f:
            json.dump(t, f, indent=1)
            f.write("\n")
        print(json.dumps(t))
        return
    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not "
              "supported (the solver keeps a whole game on one device)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        print(json.dumps(bench_mix(args)), flush=True)
        return

    import torch
    from paper_1705_02313_amd import synth
    from paper_1705_02313_amd.pg import Game

    br = {"si": 0, "reset": 1, "bf": 2}[args.best_response]
    desc, cfg = WORKLOADS[args.workload]
    log(f"generating {args.workload}: {desc}")
    t0 = time.perf_counter()
    game = synth.config_game(cfg)
    log(f"generated n={game['n']} m={game['m']} in "
        f"{time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    arrs = {k: torch.from_numpy(np.ascontiguousarray(game[k])).to(dev)
            for k in ("offsets", "targets", "owner", "pri")}
    torch.cuda.synchronize()

    def step(profile: bool):
        t_a = time.perf_counter()
        g = Game(arrs["offsets"], arrs["targets"], arrs["owner"], arrs["pri"],
                 n=game["n"], host_reduced_list=args.host_reduced_list)
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        if profile:
            g.profile(True)
        out = g.solve(best_response=br)
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        prof = g.profile_read() if profile else {}
        info = (g.n_aug, g.m_aug, g.d)
        g.free()
        torch.cuda.synchronize()
        t_d = time.perf_counter()
        return {"load": t_b - t_a, "solve": t_c - t_b, "free": t_d - t_c,
                "total": t_d - t_a, "stats": out["stats"], "prof": prof,
                "aug": info, "winner": out["winner"]}

    for i in range(args.warmup):
        r = step(False)
        log(f"warmup {i}: {r['total'] * 1e3:.1f} ms "
            f"(solve {r['solve'] * 1e3:.1f} ms)")

    torch.cuda.synchronize()
    runs = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_start = time.perf_counter()
    ev0.record()
    for i in range(args.steps):
        r = step(False)
        runs.append(r)
        log(f"step {i}: {r['total'] * 1e3:.1f} ms (load {r['load'] * 1e3:.1f}, "
            f"solve {r['solve'] * 1e3:.1f}, valuations "
            f"{r['stats']['n_valuations']})")
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps

    nval = runs[0]["stats"]["n_valuations"]
    assert all(r["stats"]["n_valuations"] == nval for r in runs)
    win = runs[0]["winner"].cpu().numpy()
    m = game["m"]
    value = m * nval / (ms_per_step / 1e3)
    solve_s = [r["solve"] for r in runs]
    load_s = [r["load"] for r in runs]

    # Roofline of the best-response iteration (one replay of its HIP graph)
    # from the timed steps: the library records HIP events on the solve's
    # stream around every iteration (pg_stats.iteration_ms, summed).
    n_aug, m_aug = runs[0]["aug"][0], runs[0]["aug"][1]
    b_min = method_min_bytes(n_aug, m_aug,
                             np.asarray(game["offsets"]).itemsize)
    it_ev_s = statistics.median(r["stats"]["iteration_ms"] for r in runs) \
        / 1e3 / nval
    it_wall_s = statistics.median(r["solve"] for r in runs) / nval
    roof = None
    if it_ev_s > 0:
        roof = {"bound": "hbm",
                "kernel": "best-response iteration (one HIP-graph replay: "
                          "ng and root walks, parent sort, Euler list, list "
                          "ranking, All_Odd)",
                "achieved": round(b_min / it_ev_s / 1e9, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(b_min / it_ev_s / 1e9 / HBM_PEAK_GBS, 4),
                "avg_launch_us": round(it_ev_s * 1e6, 2),
                "bytes_per_launch": b_min,
                "launches": nval * args.steps,
                "traffic": None,
                "traffic_kind": "rocprofv3 FETCH_SIZE + WRITE_SIZE per "
                                "iteration, each scaled by its reading on a "
                                "plain copy: bytes through the L2's fabric "
                                "port (Infinity Cache hits included)",
                "wall_us_per_iteration": round(it_wall_s * 1e6, 2),
                "wall_frac": round(b_min / it_wall_s / 1e9 / HBM_PEAK_GBS,
                                   4),
                "measured_over": f"HIP events around each of the "
                                 f"{nval * args.steps} iterations of the "
                                 "timed steps"}

    # Per-kernel figures: the library's event profiler records a pair of
    # HIP events around every kernel on its stream; those events drain the
    # stream between kernels, so they come from profiled steps of the same
    # job after the timed ones.
    dominant = None
    iteration_bytes = None
    kernels = {}
    prof_steps = 0
    if not args.no_profile:
        prof_steps = max(1, min(args.steps, 2))
        pruns = [step(True) for _ in range(prof_steps)]
        agg = {}
        for r in pruns:
            for k, d in r["prof"].items():
                a = agg.setdefault(k, {"ms": 0.0, "calls": 0, "bytes": 0.0})
                a["ms"] += d["ms"]
                a["calls"] += d["calls"]
                a["bytes"] += d["bytes"]
        for k, a in agg.items():
            kernels[k] = {"ms_total": round(a["ms"], 3), "calls": a["calls"],
                          "avg_us": round(1e3 * a["ms"] / a["calls"], 2),
                          "alg_GBps": round(a["bytes"] / (a["ms"] / 1e3) / 1e9,
                                            1) if a["ms"] > 0 else None}
        dom = max(agg, key=lambda k: agg[k]["ms"])
        a = agg[dom]
        achieved = a["bytes"] / (a["ms"] / 1e3) / 1e9
        dominant = {"kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "avg_launch_us": round(1e3 * a["ms"] / a["calls"], 2),
                    "bytes_per_launch": round(a["bytes"] / a["calls"]),
                    "traffic": counter_traffic(args.workload, dom),
                    "measured_over": f"{prof_steps} profiled steps of the "
                                     "same job after the timed steps"}
        it_bytes = sum(a["bytes"] for a in agg.values()) / (prof_steps * nval)
        traffic = {k: counter_traffic(args.workload, k) for k in agg}
        it_traffic = None
        if all(v is not None for v in traffic.values()):
            it_traffic = sum(traffic[k] * agg[k]["calls"] for k in agg) / (
                prof_steps * nval)
        if roof is not None and it_traffic:
            roof["traffic"] = round(it_traffic)
        iteration_bytes = {
            "kernel_alg_bytes": round(it_bytes),
            "kernel_alg_frac": (round(it_bytes / it_ev_s / 1e9 /
                                      HBM_PEAK_GBS, 4) if it_ev_s else None),
            "method_min_bytes": b_min,
            "counter_bytes": round(it_traffic) if it_traffic else None,
            "counter_GBps": (round(it_traffic / it_ev_s / 1e9, 1)
                             if it_traffic and it_ev_s else None),
            "copy_GBps": round(copy_bandwidth(), 1)}
        # the random-line view: counter bytes are whole 128-byte lines (or
        # 64-byte halves), so lines per iteration over the rate of random
        # gathers measured here is the time a pass touching each of those
        # lines at random would take
        rg = random_gather_rate()
        iteration_bytes["random_gather_G_per_s"] = round(
            rg["gathers_per_s"] / 1e9, 2)
        if it_traffic and it_ev_s:
            lines = it_traffic / 128.0
            floor_s = lines / rg["gathers_per_s"]
            iteration_bytes["counter_lines_per_iteration"] = round(lines)
            iteration_bytes["line_floor_us"] = round(floor_s * 1e6, 1)
            iteration_bytes["line_floor_frac"] = round(floor_s / it_ev_s, 3)

    line = {
        "metric": "edges/s per best-response iteration",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": game["n"], "m": m,
                   "n_aug": runs[0]["aug"][0], "m_aug": runs[0]["aug"][1],
                   "valuation": (f"counts, d={runs[0]['aug'][2]}"
                                 if runs[0]["aug"][2] else "ranks"),
                   "step": "pg_load_csr + pg_solve + pg_free, inputs resident "
                           "in HBM"},
        "solve_seconds_median": statistics.median(solve_s),
        "load_seconds_median": statistics.median(load_s),
        "n_major": runs[0]["stats"]["n_major"],
        "n_valuations": nval,
        "best_response": args.best_response,
        "host_reduced_list": args.host_reduced_list,
        "ms_per_iteration": 1e3 * statistics.median(solve_s) / nval,
        "aug_edges_per_s": runs[0]["aug"][1] * nval /
        statistics.median(solve_s),
        "w_even": int((win == 0).sum()),
        "event_ms_total": ev0.elapsed_time(ev1),
        "roofline": roof,
        "dominant_kernel": dominant,
        "iteration_bytes": iteration_bytes,
        "kernels": kernels,
    }
    if not args.no_odd_region and args.best_response == "si":
        log("admissibility without dummies (PG_ODD_REGION)")
        line["odd_region"] = odd_region_run(arrs, game, win)
    if args.workload == "c3":
        log("deep-list valuation")
        line["deep_list_valuation"] = deep_list_valuation(arrs, game["n"])
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample of the same workload")
        line["cpu_baseline"], line["cpu_lr_baseline"] = cpu_baseline(
            game, counts=runs[0]["aug"][2] > 0)
    else:
        line["cpu_baseline"] = None
    if args.workload == "c2" and not args.no_mix:
        log("batched/served mix")
        line["mix"] = run_mix(args.mix_games)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
