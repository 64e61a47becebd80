"""Shared test helpers: stepwise oracle runs and array hashing."""
from __future__ import annotations

import numpy as np

from oracle import orc

KEY_TOP = 2**31 - 1
_HASH_MUL = np.uint64(1099511628211)


def np_hash(a) -> int:
    """The same polynomial hash as orc_hash: h = h*M + (uint32)a[i] + 1."""
    x = np.ascontiguousarray(a).astype(np.int64).astype(np.uint32)
    x = x.astype(np.uint64) + np.uint64(1)
    n = x.size
    if n == 0:
        return 0
    with np.errstate(over="ignore"):
        pw = np.ones(n, dtype=np.uint64)
        if n > 1:
            pw[1:] = _HASH_MUL
            pw = np.cumprod(pw)[::-1].copy()
        return int((x * pw).sum(dtype=np.uint64))


def oracle_trajectory(aug: dict, max_vals: int = 10**9):
    """Runs Algorithm 1 stepwise on the modified game with the C oracle and
    yields (sigma, tau, key) for every valuation, in order."""
    sigma, tau = orc.initial_strategies(aug)
    by_pri = orc.order_by_pri(aug["pri"])
    own = np.asarray(aug["owner"])
    count = 0
    while True:
        while True:
            succ = np.where(own == 1, tau, sigma).astype(np.int32)
            key, nf, rc = orc.valuation(succ, aug["pri"], by_pri=by_pri)
            assert rc == 0
            yield sigma.copy(), tau.copy(), key
            count += 1
            if count >= max_vals:
                return
            tau, c = orc.odd_switch(aug, key, tau)
            if c == 0:
                break
        sigma, c = orc.even_switch(aug, key, sigma)
        if c == 0:
            return


def to_np(x):
    if hasattr(x, "detach"):
        return x.detach().cpu().numpy()
    return np.asarray(x)


def dense_oracle_trajectory(aug: dict, max_vals: int = 10**9):
    """As oracle_trajectory, with the count-valuation oracle; yields
    (sigma, tau, counts, top) for every valuation, in order."""
    sigma, tau = orc.initial_strategies(aug)
    own = np.asarray(aug["owner"])
    count = 0
    while True:
        while True:
            succ = np.where(own == 1, tau, sigma).astype(np.int32)
            counts, top, values, rc = orc.dense_valuation(succ, aug["pri"])
            assert rc == 0
            yield sigma.copy(), tau.copy(), counts, top
            count += 1
            if count >= max_vals:
                return
            tau, c = orc.dense_odd_switch(aug, counts, top, values, tau)
            if c == 0:
                break
        sigma, c = orc.dense_even_switch(aug, counts, top, values, sigma)
        if c == 0:
            return


def off_row_tau(aug: dict, tau, k: int, seed: int):
    """tau with k Odd vertices pointed at Even vertices outside their rows
    (a strategy the C ABI accepts).  While every Even vertex takes the sink,
    such a play stays admissible."""
    rng = np.random.default_rng(seed)
    own = np.asarray(aug["owner"])
    off = np.asarray(aug["offsets"])
    tgt = np.asarray(aug["targets"])
    evens = np.flatnonzero(own == 0)
    odds = np.flatnonzero(own == 1)
    t = np.array(tau, dtype=np.int32, copy=True)
    for v in rng.choice(odds, size=min(k, odds.size), replace=False):
        row = set(tgt[off[v]:off[v + 1]].tolist())
        u = int(rng.choice(evens))
        while u in row:
            u = int(rng.choice(evens))
        t[v] = u
    return t


def stands_for(aug_off, aug_tgt, n_orig: int) -> np.ndarray:
    """For every vertex of a modified game, the original vertex it stands
    for: itself, or w for a dummy d_w (whose row is [w])."""
    off = np.asarray(aug_off, np.int64)
    tgt = np.asarray(aug_tgt)
    n = off.size - 1
    sf = np.arange(n, dtype=np.int64)
    if n > n_orig:
        sf[n_orig:] = tgt[off[n_orig:n]]
    return sf


def tau_to_aug(aug_off, aug_tgt, owner, tau, n_orig: int) -> np.ndarray:
    """A solve's reported tau (dummy choices given as their w) back in the
    modified game's ids: each Odd choice becomes the row entry that stands
    for it (unique: an edge to w is either kept or redirected to d_w)."""
    off = np.asarray(aug_off, np.int64)
    tgt = np.asarray(aug_tgt, np.int64)
    own = np.asarray(owner)
    tau = np.asarray(tau, np.int64)
    n = off.size - 1
    sf = stands_for(off, tgt, n_orig)
    src = np.repeat(np.arange(n), np.diff(off))
    hit = (own[src] == 1) & (sf[tgt] == tau[src])
    out = tau.copy()
    # the first matching edge of each Odd row (rows are contiguous)
    e = np.flatnonzero(hit)
    first = np.full(n, -1, np.int64)
    first[src[e][::-1]] = e[::-1]
    odd = own == 1
    assert (first[odd] >= 0).all(), "a reported Odd choice is not a row edge"
    out[odd] = tgt[first[odd]]
    return out.astype(np.int32)


def is_original_edge(game: dict, tau, n_orig: int) -> bool:
    """Whether every Odd original vertex's choice in tau is an edge of the
    original game."""
    off = np.asarray(game["offsets"], np.int64)
    tgt = np.asarray(game["targets"], np.int64)
    own = np.asarray(game["owner"])
    tau = np.asarray(tau, np.int64)[:n_orig]
    src = np.repeat(np.arange(n_orig), np.diff(off[:n_orig + 1]))
    ok = np.zeros(n_orig, bool)
    ok[src[tgt == tau[src]]] = True
    return bool(ok[own[:n_orig] == 1].all())
