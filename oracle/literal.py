"""Literal oracle (test infrastructure only; never part of the product path).

A plain, slow transcription of the paper's definitions, for small games
(a few thousand vertices at most).  Valuations are the paper's dense count
vectors over the priorities in use, compared with the Maxdiff rule; nothing
here uses the compact rank representation of the GPU path.

Paper passages followed (Fearnley, "Efficient Parallel Strategy Improvement
for Parity Games"):

* section 2 (Preliminaries): games, positional strategies, plays, MaxIo.
* section 3, "A modified game": the sink s and the Even edges v -> s.
* section 3, "Admissible strategies" and "The algorithm": sigma_init = s and
  the admissibility preprocessing with dummy Even vertices.
* section 3, "Valuations": Val(v) = top for an infinite play, else the count of
  each priority on v0..vk (the sink excluded); the order with Maxdiff.
* section 3, "Switching rules": greedy all-switches.
* section 4: best responses by one-player strategy improvement, All_Odd,
  Algorithm 1 (nested loops, tau warm-started); Bellman-Ford best response.
* section 5, "Constructing the list ranking instance in parallel": the
  sequential start/end pointer construction of the Euler-tour list.

Readings of points the paper leaves open (each also listed in the design
notes of the repository):

* sigma_init sends every Even vertex (dummies included) to the sink; the
  "arbitrary" initial Odd strategy is the first entry of each row.
* Preprocessing: X is the greatest set of Odd vertices each having a successor
  in X (Odd can avoid Even vertices forever from X).  X' is the part of X with
  a predecessor in X.  Each w in X' gets a dummy Even vertex d_w (ids n, n+1,
  ... in increasing w) whose only real edge goes to w; every edge (u, w) with
  u, w in X is redirected to d_w in place.  Dummy priorities are 0..|X'|-1 (the
  index of w in X'); original priorities are shifted up by K = |X'| rounded
  up to an even number, which keeps their order and parity.
* top equals top (no switch between two top options); ties go to the lowest
  row position, the sink being slot 0 of an Even row; a switch needs a strict
  improvement.
* n_major counts every outer iteration including the last one, which switches
  nothing; n_valuations counts every valuation.
"""
from __future__ import annotations

import itertools
from functools import cmp_to_key

import numpy as np

SINK = -1
KEY_TOP = 2**31 - 1
TOP = None  # the valuation "top" (an infinite play)


# --------------------------------------------------------------------------
# section 3: the admissibility preprocessing
# --------------------------------------------------------------------------
def preprocess(game: dict) -> dict:
    """Insert dummy Even vertices so that Odd cannot close an Odd-only cycle.

    Returns the modified game (same dict layout, int64 offsets) plus
    ``dummy_of`` (int64[n_aug - n]: the vertex w each dummy leads to) and
    ``n_orig``.
    """
    n = int(game["n"])
    off = np.asarray(game["offsets"], dtype=np.int64)
    tgt = np.asarray(game["targets"], dtype=np.int64)
    owner = np.asarray(game["owner"], dtype=np.int64)
    pri = np.asarray(game["pri"], dtype=np.int64)
    rows = [tgt[off[v]:off[v + 1]].tolist() for v in range(n)]

    # X: start from all Odd vertices and drop those with no successor in X
    in_x = [owner[v] == 1 for v in range(n)]
    changed = True
    while changed:
        changed = False
        for v in range(n):
            if in_x[v] and not any(in_x[u] for u in rows[v]):
                in_x[v] = False
                changed = True
    # X': members of X with a predecessor in X
    in_xp = [False] * n
    for u in range(n):
        if in_x[u]:
            for w in rows[u]:
                if in_x[w]:
                    in_xp[w] = True
    xprime = [w for w in range(n) if in_xp[w]]
    dummy = {w: n + i for i, w in enumerate(xprime)}
    k_shift = len(xprime) + (len(xprime) & 1)

    new_rows = []
    for u in range(n):
        if in_x[u]:
            new_rows.append([dummy[w] if in_x[w] else w for w in rows[u]])
        else:
            new_rows.append(list(rows[u]))
    for w in xprime:
        new_rows.append([w])
    n_aug = n + len(xprime)
    deg = np.array([len(r) for r in new_rows], dtype=np.int64)
    offsets = np.zeros(n_aug + 1, dtype=np.int64)
    np.cumsum(deg, out=offsets[1:])
    targets = np.array([t for r in new_rows for t in r], dtype=np.int64)
    owner2 = np.concatenate([owner, np.zeros(len(xprime), np.int64)])
    pri2 = np.concatenate([pri + k_shift,
                           np.arange(len(xprime), dtype=np.int64)])
    return {"n": n_aug, "m": int(offsets[-1]), "offsets": offsets,
            "targets": targets, "owner": owner2, "pri": pri2,
            "dummy_of": np.array(xprime, dtype=np.int64), "n_orig": n,
            "in_x": np.array(in_x, dtype=bool)}


def identity_augment(game: dict) -> dict:
    """The game without preprocessing (for inputs known to be safe)."""
    n = int(game["n"])
    return {"n": n, "m": int(game["m"]),
            "offsets": np.asarray(game["offsets"], np.int64),
            "targets": np.asarray(game["targets"], np.int64),
            "owner": np.asarray(game["owner"], np.int64),
            "pri": np.asarray(game["pri"], np.int64),
            "dummy_of": np.zeros(0, np.int64), "n_orig": n,
            "in_x": np.zeros(n, bool)}


def rows_of(g: dict) -> list:
    off = g["offsets"]
    tgt = g["targets"]
    return [tgt[off[v]:off[v + 1]].tolist() for v in range(int(g["n"]))]


# --------------------------------------------------------------------------
# section 3: valuations and their order
# --------------------------------------------------------------------------
class Vals:
    """Dense valuations: one count per priority in D_G (the priorities used)."""

    def __init__(self, pri):
        self.pri = np.asarray(pri, dtype=np.int64)
        self.dom = np.unique(self.pri)            # D_G, ascending
        self.index = {int(p): i for i, p in enumerate(self.dom)}

    def zero(self):
        return np.zeros(self.dom.size, dtype=np.int64)

    def unit(self, p: int, sign: int = 1):
        """A_p (sign +1) or A_{-p} (sign -1) of the formal reduction."""
        a = self.zero()
        a[self.index[int(p)]] = sign
        return a


def maxdiff(l1: np.ndarray, l2: np.ndarray, dom: np.ndarray):
    """Largest priority whose counts differ, or None when l1 == l2."""
    d = np.flatnonzero(l1 != l2)
    if d.size == 0:
        return None
    return int(d[-1])


def val_le(l1, l2, dom) -> bool:
    """l1 below-or-equal l2 in the paper's order (top is the largest)."""
    if l2 is TOP:
        return True
    if l1 is TOP:
        return False            # L below top, and top not below any L
    i = maxdiff(l1, l2, dom)
    if i is None:
        return True
    p = int(dom[i])
    if p % 2 == 0:
        return l1[i] < l2[i]
    return l1[i] > l2[i]


def val_lt(l1, l2, dom) -> bool:
    return val_le(l1, l2, dom) and not val_le(l2, l1, dom)


def successor(g: dict, sigma, tau, v: int) -> int:
    return sigma[v] if g["owner"][v] == 0 else tau[v]


def valuation(g: dict, vals: Vals, sigma, tau):
    """Val^{sigma,tau}: the paper's sequential algorithm, working backwards on
    the tree rooted at the sink and counting each priority on the way.

    Returns (list of dense vectors or TOP, cycles) where cycles lists, for
    every cycle of the play graph, its vertices.
    """
    n = int(g["n"])
    succ = [successor(g, sigma, tau, v) for v in range(n)]
    kids = [[] for _ in range(n)]
    roots = []
    for v in range(n):
        if succ[v] == SINK:
            roots.append(v)
        else:
            kids[succ[v]].append(v)
    val = [TOP] * n
    stack = []
    for r in roots:
        val[r] = vals.unit(g["pri"][r])
        stack.append(r)
    while stack:
        u = stack.pop()
        for c in kids[u]:
            val[c] = val[u] + vals.unit(g["pri"][c])
            stack.append(c)
    # every vertex not reached lies on or leads into a cycle
    cycles = []
    state = [0] * n  # 0 new, 1 on current walk, 2 done
    for v in range(n):
        if val[v] is not TOP or state[v]:
            continue
        walk = []
        u = v
        while u != SINK and state[u] == 0 and val[u] is TOP:
            state[u] = 1
            walk.append(u)
            u = succ[u]
        if u != SINK and state[u] == 1:
            cyc = walk[walk.index(u):]
            cycles.append(cyc)
        for w in walk:
            state[w] = 2
    return val, cycles


def cycle_is_even(g: dict, cyc) -> bool:
    return max(int(g["pri"][v]) for v in cyc) % 2 == 0


def keys_of(vals_list, dom) -> np.ndarray:
    """Rank of each finite valuation among all finite vertices and the sink
    (the sink's valuation is the zero vector); KEY_TOP for top.  The last
    entry is the sink's key."""
    n = len(vals_list)
    fin = [v for v in range(n) if vals_list[v] is not TOP]
    zero = np.zeros(dom.size, dtype=np.int64)
    items = fin + [SINK]

    def get(v):
        return zero if v == SINK else vals_list[v]

    def cmp(a, b):
        la, lb = get(a), get(b)
        if val_le(la, lb, dom) and val_le(lb, la, dom):
            return 0
        return -1 if val_le(la, lb, dom) else 1

    order = sorted(items, key=cmp_to_key(cmp))
    key = np.full(n + 1, KEY_TOP, dtype=np.int64)
    for r, v in enumerate(order):
        key[n if v == SINK else v] = r
    # distinct priorities make finite valuations pairwise distinct
    for a, b in zip(order, order[1:]):
        assert cmp(a, b) < 0, "two finite vertices share a valuation"
    return key


# --------------------------------------------------------------------------
# sections 3 and 4: switching
# --------------------------------------------------------------------------
def odd_switches(g, vals, rows, sigma, tau, val):
    """All_Odd(sigma, tau): every Odd vertex with an Odd-switchable edge moves
    to the first successor of minimal valuation."""
    dom = vals.dom
    new_tau = list(tau)
    count = 0
    for v in range(int(g["n"])):
        if g["owner"][v] != 1:
            continue
        best = rows[v][0]
        for u in rows[v][1:]:
            if val_lt(val[u], val[best], dom):
                best = u
        if val_lt(val[best], val[tau[v]], dom):
            new_tau[v] = best
            count += 1
    return new_tau, count


def even_switches(g, vals, rows, sigma, val):
    """All_Even(sigma): greedy all-switches for Even; the sink is option 0."""
    dom = vals.dom
    zero = vals.zero()

    def vv(u):
        return zero if u == SINK else val[u]

    new_sigma = list(sigma)
    count = 0
    for v in range(int(g["n"])):
        if g["owner"][v] != 0:
            continue
        best = SINK
        for u in rows[v]:
            if val_lt(vv(best), vv(u), dom):
                best = u
        if val_lt(vv(sigma[v]), vv(best), dom):
            new_sigma[v] = best
            count += 1
    return new_sigma, count


def initial_strategies(g, rows):
    n = int(g["n"])
    sigma = [SINK if g["owner"][v] == 0 else SINK for v in range(n)]
    tau = [rows[v][0] if g["owner"][v] == 1 else SINK for v in range(n)]
    return sigma, tau


class Inadmissible(Exception):
    pass


def best_response_si(g, vals, rows, sigma, tau, trace=None, max_inner=None):
    """The inner loop of Algorithm 1: one-player SI for Odd against sigma.
    Returns (tau, val, n_valuations)."""
    count_val = 0
    while True:
        val, cycles = valuation(g, vals, sigma, tau)
        count_val += 1
        for cyc in cycles:
            if not cycle_is_even(g, cyc):
                raise Inadmissible("odd cycle under sigma")
        if trace is not None:
            trace.append(keys_of(val, vals.dom))
        tau, c = odd_switches(g, vals, rows, sigma, tau, val)
        if c == 0:
            return tau, val, count_val
        if max_inner is not None and count_val >= max_inner:
            raise RuntimeError("inner iteration limit")


def solve(game: dict, preprocess_game: bool = True, trace: bool = False):
    """Algorithm 1 on the game; returns winners and the final strategies."""
    g = preprocess(game) if preprocess_game else identity_augment(game)
    rows = rows_of(g)
    vals = Vals(g["pri"])
    sigma, tau = initial_strategies(g, rows)
    n_major = 0
    n_val = 0
    keys = [] if trace else None
    majors = []
    while True:
        n_major += 1
        tau, val, k = best_response_si(g, vals, rows, sigma, tau, keys)
        n_val += k
        majors.append((list(sigma), list(tau), val))
        sigma, c = even_switches(g, vals, rows, sigma, val)
        if c == 0:
            break
    n0 = g["n_orig"]
    winner = np.array([0 if val[v] is TOP else 1 for v in range(n0)],
                      dtype=np.uint8)
    return {"aug": g, "winner": winner, "sigma": np.array(sigma),
            "tau": np.array(tau), "val": val, "vals": vals,
            "n_major": n_major, "n_valuations": n_val, "keys": keys,
            "majors": majors}


# --------------------------------------------------------------------------
# section 4: Bellman-Ford best response
# --------------------------------------------------------------------------
def bellman_ford(g, vals, rows, sigma):
    """Val^sigma by Jacobi rounds of Bellman-Ford: labels start at top with
    the sink at the zero vector; an Even vertex adds its priority to its
    sigma-successor's label, an Odd vertex takes the smallest successor label
    plus its priority.  Returns (labels, rounds)."""
    n = int(g["n"])
    dom = vals.dom
    zero = vals.zero()
    lab = [TOP] * n

    def get(u):
        return zero if u == SINK else lab[u]

    def plus(p, l):
        return TOP if l is TOP else l + vals.unit(p)

    for rnd in range(n + 2):
        new = list(lab)
        for v in range(n):
            p = g["pri"][v]
            if g["owner"][v] == 0:
                new[v] = plus(p, get(sigma[v]))
            else:
                best = TOP
                for u in rows[v]:
                    cand = plus(p, get(u))
                    if val_lt(cand, best, dom):
                        best = cand
                new[v] = best
        same = all((a is TOP and b is TOP) or
                   (a is not TOP and b is not TOP and np.array_equal(a, b))
                   for a, b in zip(lab, new))
        lab = new
        if same:
            return lab, rnd + 1
    raise AssertionError("Bellman-Ford did not reach a fixpoint")


# --------------------------------------------------------------------------
# brute force over positional strategies (tiny games only)
# --------------------------------------------------------------------------
def brute_force_tau_min(g, vals, rows, sigma):
    """The pointwise minimum of Val^{sigma,tau} over every positional tau."""
    n = int(g["n"])
    dom = vals.dom
    odd = [v for v in range(n) if g["owner"][v] == 1]
    best = None
    for choice in itertools.product(*[rows[v] for v in odd]):
        tau = [SINK] * n
        for v, u in zip(odd, choice):
            tau[v] = u
        val, _ = valuation(g, vals, sigma, tau)
        if best is None:
            best = list(val)
        else:
            for v in range(n):
                if val_lt(val[v], best[v], dom):
                    best[v] = val[v]
    return best


def play_maxio(pri, succ, v):
    """MaxIo of the (lasso-shaped) play from v in a graph with one edge per
    vertex: the largest priority on its cycle."""
    seen = {}
    path = []
    u = v
    while u not in seen:
        seen[u] = len(path)
        path.append(u)
        u = succ[u]
    return max(int(pri[w]) for w in path[seen[u]:])


def brute_force_winners(game: dict, limit: int = 400000):
    """W_Even by enumerating every positional sigma and tau of the original
    game (no sink): v is Even's iff some sigma wins every tau from v."""
    n = int(game["n"])
    g = identity_augment(game)
    rows = rows_of(g)
    pri = g["pri"]
    even = [v for v in range(n) if g["owner"][v] == 0]
    odd = [v for v in range(n) if g["owner"][v] == 1]
    total = 1
    for v in range(n):
        total *= len(rows[v])
    if total > limit:
        raise ValueError("game too large for brute force")
    win = np.zeros(n, dtype=bool)
    for sc in itertools.product(*[rows[v] for v in even]):
        good = np.ones(n, dtype=bool)
        for tc in itertools.product(*[rows[v] for v in odd]):
            succ = [0] * n
            for v, u in zip(even, sc):
                succ[v] = u
            for v, u in zip(odd, tc):
                succ[v] = u
            for v in range(n):
                if good[v] and play_maxio(pri, succ, v) % 2 == 1:
                    good[v] = False
        win |= good
    return np.where(win, 0, 1).astype(np.uint8)


# --------------------------------------------------------------------------
# section 5: the sequential start/end construction of the Euler-tour list
# --------------------------------------------------------------------------
def euler_list_sequential(parent: dict, order):
    """Build the list of the tree given by ``parent`` (child -> parent; the
    root has no entry) by the start/end pointer procedure: start(v) is first
    the down edge of v and end(v) its up edge; processing v with parent u
    links the element at start(u) to start(v) and then sets start(u) to
    end(v); finally each start(v) is linked to end(v).

    ``order`` is the order in which vertices are processed.  Elements are the
    tuples (u, v) of the paper: the down edge of v is (parent, v) and its up
    edge (v, parent).  Returns the successor map over elements and the head.
    """
    nodes = set(parent) | set(parent.values())
    root = [v for v in nodes if v not in parent]
    assert len(root) == 1
    root = root[0]
    start = {}
    end = {}
    for v in nodes:
        if v == root:
            start[v] = ("head", root)
            end[v] = ("tail", root)
        else:
            start[v] = (parent[v], v)
            end[v] = (v, parent[v])
    # Step 2 links start(u) to the down edge of v (the value start(v) had
    # before any child of v was processed).  Read literally, "the element
    # pointed to by start(v)" would skip v's down edge whenever a child of v
    # is processed before v; the arbitrary processing order and the parallel
    # atomic-exchange version both need this reading.
    down = {v: start[v] for v in nodes}
    succ = {}
    for v in order:
        u = parent[v]
        succ[start[u]] = down[v]
        start[u] = end[v]
    for v in nodes:
        succ[start[v]] = end[v]
    return succ, ("head", root)


def walk_list(succ, head):
    out = []
    e = head
    while e in succ:
        out.append(e)
        e = succ[e]
    out.append(e)
    return out
