"""Batched / served solving: every game's result in the mix equals the CPU
oracle's result for that game alone (strategies, winners, iteration and
switch counts), also when the arena is too small for all games at once and
games join and leave it between steps."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import orc
from paper_1705_02313_amd import synth
from paper_1705_02313_amd.pg import PG_EINVAL, PG_ENOMEM, Batch, PgError

pytestmark = pytest.mark.gpu


def _mix(count, seed_base, nmin=100, nmax=20000):
    games = synth.mixed_batch(count, seed_base, nmin=nmin, nmax=nmax)
    games.append(synth.chain_game(3000, seed_base))
    games.append(synth.random_game(3, 2, 2, seed_base))
    return games


def _check(game, out):
    ref = orc.solve(game)
    assert ref["status"] == 0
    np.testing.assert_array_equal(out["winner"], ref["winner"])
    np.testing.assert_array_equal(out["sigma"], ref["sigma"])
    np.testing.assert_array_equal(out["tau"], ref["tau_orig"])
    st = out["stats"]
    assert st["n_major"] == ref["n_major"]
    assert st["n_valuations"] == ref["n_valuations"]
    assert st["n_odd_switches"] == ref["n_odd_switches"]
    assert st["n_even_switches"] == ref["n_even_switches"]


def _drain(b, tickets, max_steps=100000):
    out = {}
    for _ in range(max_steps):
        live, queued, _ = b.step()
        for t in list(tickets):
            r = b.poll(t)
            if r is not None:
                out[t] = r
                tickets.remove(t)
        if not tickets:
            return out
    raise AssertionError("batch did not finish")


def test_batch_all_at_once_matches_solo():
    games = _mix(24, 7000)
    with Batch(10_000_000, 60_000_000) as b:
        tickets = [b.submit(g) for g in games]
        out = _drain(b, list(tickets))
    for g, t in zip(games, tickets):
        _check(g, out[t])


def test_batch_small_arena_queues_and_rebuilds():
    games = _mix(16, 7100, nmin=500, nmax=8000)
    biggest = max(orc.preprocess(g)["n"] for g in games)
    edges = max(orc.preprocess(g)["m"] for g in games)
    # room for only a few games at a time: admission and rebuilds mid-run
    with Batch(3 * biggest, 3 * edges) as b:
        tickets = [b.submit(g) for g in games]
        assert b.info()["queued"] == len(games)
        out = _drain(b, list(tickets))
        assert b.info()["live"] == 0
    for g, t in zip(games, tickets):
        _check(g, out[t])


def test_batch_staggered_arrivals():
    games = _mix(12, 7200, nmin=200, nmax=6000)
    with Batch(2_000_000, 12_000_000) as b:
        pending = []
        out = {}
        for i, g in enumerate(games):
            pending.append((g, b.submit(g)))
            for _ in range(i % 3 + 1):       # some steps between arrivals
                b.step()
            for gg, t in list(pending):
                r = b.poll(t)
                if r is not None:
                    out[t] = (gg, r)
                    pending.remove((gg, t))
        rest = _drain(b, [t for _, t in pending])
        for gg, t in pending:
            out[t] = (gg, rest[t])
    assert len(out) == len(games)
    for g, r in out.values():
        _check(g, r)


def test_batch_errors():
    with Batch(1000, 6000) as b:
        with pytest.raises(PgError) as e:
            b.submit(synth.random_game(5000, 2, 5, 1))
        assert e.value.status == PG_ENOMEM
        g = synth.random_game(50, 2, 3, 2)
        g["pri"] = g["pri"].copy()
        g["pri"][3] = g["pri"][4]
        with pytest.raises(PgError) as e:
            b.submit(g)
        assert e.value.status == PG_EINVAL
        # the preprocessing shift pushes a priority past INT32_MAX
        g = synth.random_game(200, 2, 5, 8)
        g["pri"] = g["pri"].copy()
        g["pri"][0] = 2**31 - 2
        with pytest.raises(PgError) as e:
            b.submit(g)
        assert e.value.status == PG_EINVAL
        # the batch still works
        h = synth.random_game(300, 2, 5, 3)
        t = b.submit(h)
        _check(h, _drain(b, [t])[t])


def test_submissions_from_another_thread():
    """pg_batch_submit may run on another thread while this one steps the
    batch (submissions preprocess on the batch's own stream and take its
    lock only to queue the game): every result equals the oracle's."""
    import threading
    import time
    games = _mix(24, 7300, nmin=300, nmax=12000)
    biggest = max(orc.preprocess(g)["n"] for g in games)
    edges = max(orc.preprocess(g)["m"] for g in games)
    tickets, failure = [], []

    def submitter():
        try:
            for g in games:
                tickets.append(b.submit(g))
                time.sleep(0.0005)
        except Exception as e:
            failure.append(e)

    with Batch(4 * biggest, 4 * edges) as b:
        th = threading.Thread(target=submitter)
        th.start()
        out = {}
        for _ in range(200000):
            b.step()
            for t in b.finished():
                out[t] = b.poll(t)
            if not th.is_alive() and len(out) == len(games):
                break
        th.join()
    assert not failure
    assert len(out) == len(games)
    for g, t in zip(games, tickets):
        _check(g, out[t])


@pytest.mark.parametrize("thread", [True, False])
def test_serve_with_and_without_a_submitter_thread(thread):
    """serve(): submissions on their own thread (overlapping the steps) or
    between steps; either way every game's result is the oracle's."""
    from paper_1705_02313_amd.serve import poisson_arrivals, serve
    games = _mix(20, 7300)
    nv = sum(int(g["n"]) for g in games)
    ne = sum(int(g["m"]) for g in games)
    arr = poisson_arrivals(len(games), 400.0, 7301)
    r = serve(games, arr, nv // 2 + 40000, ne // 2 + 200000,
              submit_thread=thread)
    assert len(r["results"]) == len(games)
    assert (r["latency"] >= 0).all()
    for i, g in enumerate(games):
        _check(g, r["results"][i])


def test_submit_many_matches_the_oracle_and_refuses_per_game():
    """pg_batch_submit_many: the games queued in one call (preprocessed over
    their union) finish with the oracle's results; bad games are refused
    one by one without stopping the others."""
    games = _mix(20, 7500, nmin=200, nmax=30000)
    games.append(synth.random_game(40000, 2, 6, 7501, offsets_dtype=np.int32))
    dup = synth.random_game(300, 2, 4, 7502)
    dup["pri"] = dup["pri"].copy()
    dup["pri"][5] = dup["pri"][6]                 # repeated priority
    badt = synth.random_game(300, 2, 4, 7503)
    badt["targets"] = badt["targets"].copy()
    badt["targets"][7] = 300                      # target out of range
    bado = synth.random_game(300, 2, 4, 7504)
    bado["offsets"] = bado["offsets"].copy()
    bado["offsets"][10] = bado["offsets"][9]      # an empty row
    over = synth.random_game(300, 2, 5, 7505)
    over["pri"] = over["pri"].copy()
    over["pri"][0] = 2**31 - 2                    # overflows after the shift
    huge = synth.random_game(600000, 2, 3, 7506)  # beyond the arena
    order = [0, 1, "dup", 2, "badt", 3, "bado", 4, "over", "huge"] + \
        list(range(5, len(games)))
    extra = {"dup": dup, "badt": badt, "bado": bado, "over": over,
             "huge": huge}
    sub = [extra[k] if isinstance(k, str) else games[k] for k in order]
    with Batch(500_000, 3_000_000) as b:
        res = b.submit_many(sub)
        expect = {"dup": PG_EINVAL, "badt": PG_EINVAL, "bado": PG_EINVAL,
                  "over": PG_EINVAL, "huge": PG_ENOMEM}
        tickets = {}
        for k, r in zip(order, res):
            if isinstance(k, str):
                assert isinstance(r, PgError) and r.status == expect[k], k
            else:
                assert isinstance(r, int) and r > 0, k
                tickets[r] = games[k]
        # tickets in submission order
        assert list(tickets) == sorted(tickets)
        out = _drain(b, list(tickets))
        # a second call on the same batch, then single submissions beside it
        more = _mix(6, 7600, nmin=500, nmax=5000)
        t2 = b.submit_many(more[:4]) + [b.submit(g) for g in more[4:]]
        out2 = _drain(b, list(t2))
    for t, g in tickets.items():
        _check(g, out[t])
    for t, g in zip(t2, more):
        _check(g, out2[t])


def test_submit_many_int64_offsets_and_empty_call():
    games = [synth.random_game(n, 2, 5, 7700 + n) for n in (3, 50, 999, 4000)]
    games.append(synth.chain_game(5000, 7701))
    with Batch(1_000_000, 6_000_000) as b:
        assert b.submit_many([]) == []
        ts = b.submit_many(games)
        out = _drain(b, list(ts))
    for t, g in zip(ts, games):
        _check(g, out[t])


def test_submit_many_tiny_and_degenerate_games():
    """One-vertex games, self-loops and repeated edges, one player only:
    submitted together, each finishes with the oracle's result."""
    games = []
    for seed in range(12):
        rng = np.random.Generator(np.random.PCG64(7800 + seed))
        n = [1, 1, 2, 2, 3, 5, 8, 13, 40, 100, 300, 1000][seed]
        deg = rng.integers(1, 4, size=n)
        rows = [np.sort(rng.integers(0, n, size=d)) for d in deg]
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(deg)
        p_odd = [0.0, 1.0, 0.5, 1.0, 0.0, 0.5, 0.5, 0.9, 0.5, 0.1, 0.5, 0.5]
        games.append({"n": n, "m": int(off[-1]), "offsets": off,
                      "targets": np.concatenate(rows).astype(np.int32),
                      "owner": (rng.random(n) < p_odd[seed]).astype(np.uint8),
                      "pri": rng.permutation(n).astype(np.int32)})
    with Batch(100_000, 600_000) as b:
        ts = b.submit_many(games)
        assert all(isinstance(t, int) for t in ts)
        out = _drain(b, list(ts))
    for t, g in zip(ts, games):
        _check(g, out[t])


def test_poll_many_and_queries_keep_the_ticket():
    """pg_batch_poll_many hands out every finished game at once; a poll
    with no outputs (a query) keeps the ticket, also after the game has
    left the arena at a rebuild."""
    games = _mix(10, 7900, nmin=300, nmax=5000)
    biggest = max(orc.preprocess(g)["n"] for g in games)
    edges = max(orc.preprocess(g)["m"] for g in games)
    with Batch(3 * biggest, 3 * edges) as b:
        ts = b.submit_many(games)
        # step until everything finished, polling nothing (rebuilds move
        # finished games out of the arena meanwhile)
        for _ in range(100000):
            live, queued, _ = b.step()
            if live == 0 and queued == 0:
                break
        # queries: done, and the tickets stay
        from paper_1705_02313_amd.pg import Stats, lib
        import ctypes
        for t in ts:
            d = ctypes.c_int32()
            st = Stats()
            assert lib().pg_batch_poll(b._h, t, ctypes.byref(d), None, None,
                                       None, ctypes.byref(st), 0) == 0
            assert d.value == 1
        assert sorted(b.finished()) == sorted(ts)
        res = b.poll_many(ts)
        assert b.finished() == []
        with pytest.raises(PgError) as e:
            b.poll_many(ts[:1])
        assert e.value.status == PG_EINVAL
    for g, r in zip(games, res):
        _check(g, r)
