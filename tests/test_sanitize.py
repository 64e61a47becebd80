"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize_main.c drives the C oracle (oracle/orc.c, oracle/orc_dense.c)
and the CPU-LR baseline (baselines/cpu_lr.c) on small games: preprocessing,
whole solves with both rank constructions, CPU-LR best-response iterations,
and count-valuation solves with the three best responses.  Built with gcc
-fsanitize=address,undefined (host code; no GPU involved), it must exit
cleanly with no sanitizer report, and its results must equal the regular
builds' (the ctypes oracle and baseline the other tests use).
"""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    out = tmp_path_factory.mktemp("san") / "sanitize_main"
    srcs = [os.path.join(ROOT, "tests", "sanitize_main.c"),
            os.path.join(ROOT, "oracle", "orc.c"),
            os.path.join(ROOT, "oracle", "orc_dense.c"),
            os.path.join(ROOT, "baselines", "cpu_lr.c")]
    subprocess.run(["gcc", "-std=gnu99", "-O1", "-g", "-fopenmp",
                    "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", *srcs, "-o", str(out)],
                   check=True)
    return str(out)


def _write(game, few, path):
    with open(path, "wb") as f:
        np.array([game["n"], game["m"]], np.int64).tofile(f)
        np.asarray(game["offsets"], np.int64).tofile(f)
        np.asarray(game["targets"], np.int32).tofile(f)
        np.asarray(game["owner"], np.uint8).tofile(f)
        np.asarray(game["pri"], np.int32).tofile(f)
        np.asarray(few, np.int32).tofile(f)


def _parse(text):
    out = {}
    for ln in text.splitlines():
        parts = ln.split()
        if parts:
            out[parts[0]] = parts[1:]
    return out


@pytest.mark.parametrize("kind,n,seed", [("random", 40, 1),
                                         ("random", 700, 2),
                                         ("random", 3000, 3),
                                         ("chain", 2000, 4)])
def test_cpu_code_clean_under_sanitizers(driver, tmp_path, kind, n, seed):
    g = synth.random_game(n, 2, 5, seed) if kind == "random" else \
        synth.chain_game(n, seed)
    few = np.random.Generator(np.random.PCG64([seed, 7])).integers(
        0, 4, size=n).astype(np.int32)
    path = tmp_path / "game.bin"
    _write(g, few, path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([driver, str(path)], capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
    res = _parse(r.stdout)
    ref = orc.solve(g, trace=True)
    aug = ref["aug"]
    assert [int(x) for x in res["n_aug"]] == [aug["n"], aug["m"]]
    for method in (0, 1):
        rc, nmaj, nval, nodd, neven, hs, ht, hk = \
            [int(x) for x in res[f"solve{method}"]]
        assert rc == 0
        assert (nmaj, nval, nodd, neven) == (
            ref["n_major"], ref["n_valuations"], ref["n_odd_switches"],
            ref["n_even_switches"])
        assert hs == orc.key_hash(ref["sigma"])
        assert ht == orc.key_hash(ref["tau"])
        assert hk == orc.key_hash(ref["key"])
        assert [int(x) for x in res[f"trace{method}"]] == \
            [int(x) for x in ref["trace"]]
    # CPU-LR's first best response follows the oracle's first valuations
    lr = [int(x) for x in res["cpulr"]]
    assert lr == [int(x) for x in ref["trace"][:len(lr)]]
    gf = dict(g, pri=few)
    for br in (0, 1, 2):
        d = orc.dense_solve(gf, br=br)
        rc, nmaj, nval, hs, hc = [int(x) for x in res[f"dense{br}"]]
        assert rc == 0
        assert (nmaj, nval) == (d["n_major"], d["n_valuations"])
        assert hs == orc.key_hash(d["sigma"])
        assert hc == orc.key_hash(np.ascontiguousarray(d["counts"]).ravel())
