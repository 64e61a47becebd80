"""ctypes wrapper of the scalable C oracle (oracle/orc.c for distinct
priorities with rank valuations, oracle/orc_dense.c for repeated priorities
with the paper's count valuations).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never does.  See the C files for
the passages of the paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SRC_PATHS = [os.path.join(HERE, "orc.c"), os.path.join(HERE, "orc_dense.c")]

SINK = -1
KEY_TOP = 2**31 - 1
OK, EINVAL, EINADMISSIBLE, EITERLIMIT, ENOMEM = 0, 1, 2, 3, 4
RANK_KRUSKAL, RANK_PATHSORT = 0, 1
BR_SI, BR_SI_RESET, BR_BELLMAN_FORD = 0, 1, 2

_P = ctypes.c_void_p
_I64 = ctypes.c_int64


class Stats(ctypes.Structure):
    _fields_ = [("n_major", ctypes.c_int64), ("n_valuations", ctypes.c_int64),
                ("n_even_switches", ctypes.c_int64),
                ("n_odd_switches", ctypes.c_int64)]


def build(force: bool = False) -> str:
    """Compile the C files with gcc into liborc.so next to them."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < max(os.path.getmtime(p)
                                             for p in SRC_PATHS):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC",
                               "-o", tmp, *SRC_PATHS])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_x_sets.restype = _I64
        L.orc_x_sets.argtypes = [_I64, _P, _P, _P, _P, _P]
        L.orc_preprocess.restype = _I64
        L.orc_preprocess.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.orc_valuation.restype = ctypes.c_int
        L.orc_valuation.argtypes = [_I64, _P, _P, _P, ctypes.c_int, _P, _P]
        L.orc_odd_switch.restype = _I64
        L.orc_odd_switch.argtypes = [_I64, _P, _P, _P, _P, _P]
        L.orc_even_switch.restype = _I64
        L.orc_even_switch.argtypes = [_I64, _P, _P, _P, _P, _P]
        L.orc_hash.restype = ctypes.c_uint64
        L.orc_hash.argtypes = [_I64, _P]
        L.orc_order_by_pri.restype = None
        L.orc_order_by_pri.argtypes = [_I64, _P, _P]
        L.orc_solve.restype = ctypes.c_int
        L.orc_solve.argtypes = [_I64, _P, _P, _P, _P, ctypes.c_int, _I64, _I64,
                                ctypes.c_int, _P, _P, _P,
                                ctypes.POINTER(Stats), _P, _I64]
        L.orc_dense_preprocess.restype = _I64
        L.orc_dense_preprocess.argtypes = [_I64] + [_P] * 9
        L.orc_dense_priorities.restype = _I64
        L.orc_dense_priorities.argtypes = [_I64, _P, _P, _P]
        L.orc_dense_valuation.restype = ctypes.c_int
        L.orc_dense_valuation.argtypes = [_I64, _P, _P, _I64, _P, _P, _P]
        L.orc_dense_compare.restype = ctypes.c_int
        L.orc_dense_compare.argtypes = [_I64, _I64, _P, _P, _P, _I64, _I64]
        L.orc_dense_odd_switch.restype = _I64
        L.orc_dense_odd_switch.argtypes = [_I64, _P, _P, _P, _I64, _P, _P, _P,
                                           _P]
        L.orc_dense_even_switch.restype = _I64
        L.orc_dense_even_switch.argtypes = [_I64, _P, _P, _P, _I64, _P, _P,
                                            _P, _P]
        L.orc_dense_solve.restype = ctypes.c_int
        L.orc_dense_solve.argtypes = [_I64, _P, _P, _P, _P, _I64, _I64,
                                      ctypes.c_int, _P, _P, _P, _P,
                                      ctypes.POINTER(Stats), _P, _I64]
        L.orc_dense_bellman_ford.restype = _I64
        L.orc_dense_bellman_ford.argtypes = [_I64, _P, _P, _P, _P, _I64, _P,
                                             _P, _P, _P, _P]
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def preprocess(game: dict) -> dict:
    """The modified game with dummy Even vertices (see orc_preprocess)."""
    n = int(game["n"])
    off = _c(game["offsets"], np.int64)
    tgt = _c(game["targets"], np.int32)
    own = _c(game["owner"], np.uint8)
    pri = _c(game["pri"], np.int32)
    m = int(off[-1])
    off2 = np.zeros(2 * n + 1, np.int64)
    tgt2 = np.zeros(m + n, np.int32)
    own2 = np.zeros(2 * n, np.uint8)
    pri2 = np.zeros(2 * n, np.int32)
    dum = np.zeros(max(n, 1), np.int32)
    n_aug = lib().orc_preprocess(n, _ptr(off), _ptr(tgt), _ptr(own), _ptr(pri),
                                 _ptr(off2), _ptr(tgt2), _ptr(own2),
                                 _ptr(pri2), _ptr(dum))
    if n_aug < 0:
        raise ValueError("preprocessing failed (priority overflow)")
    k = n_aug - n
    m_aug = m + k
    return {"n": n_aug, "m": m_aug, "offsets": off2[:n_aug + 1].copy(),
            "targets": tgt2[:m_aug].copy(), "owner": own2[:n_aug].copy(),
            "pri": pri2[:n_aug].copy(), "dummy_of": dum[:k].copy(),
            "n_orig": n}


def identity(game: dict) -> dict:
    n = int(game["n"])
    return {"n": n, "m": int(game["m"]),
            "offsets": _c(game["offsets"], np.int64),
            "targets": _c(game["targets"], np.int32),
            "owner": _c(game["owner"], np.uint8),
            "pri": _c(game["pri"], np.int32),
            "dummy_of": np.zeros(0, np.int32), "n_orig": n}


def x_sets(game: dict):
    n = int(game["n"])
    inx = np.zeros(n, np.uint8)
    inxp = np.zeros(n, np.uint8)
    lib().orc_x_sets(n, _ptr(_c(game["offsets"], np.int64)),
                     _ptr(_c(game["targets"], np.int32)),
                     _ptr(_c(game["owner"], np.uint8)), _ptr(inx), _ptr(inxp))
    return inx.astype(bool), inxp.astype(bool)


def order_by_pri(pri) -> np.ndarray:
    pri = _c(pri, np.int32)
    out = np.zeros(pri.size, np.int32)
    lib().orc_order_by_pri(pri.size, _ptr(pri), _ptr(out))
    return out


def valuation(succ, pri, method: int = RANK_KRUSKAL, by_pri=None):
    """Ranks of Val^{sigma,tau}; succ uses SINK for the sink.
    Returns (key[n+1], n_finite, status)."""
    succ = _c(succ, np.int32)
    pri = _c(pri, np.int32)
    n = succ.size
    if by_pri is None and method == RANK_KRUSKAL:
        by_pri = order_by_pri(pri)
    bp = _c(by_pri, np.int32) if by_pri is not None else None
    key = np.zeros(n + 1, np.int32)
    nf = ctypes.c_int64(0)
    rc = lib().orc_valuation(n, _ptr(succ), _ptr(pri),
                             _ptr(bp) if bp is not None else None, method,
                             _ptr(key), ctypes.byref(nf))
    return key, int(nf.value), int(rc)


def odd_switch(g: dict, key, tau) -> tuple:
    tau = _c(tau, np.int32).copy()
    c = lib().orc_odd_switch(int(g["n"]), _ptr(_c(g["offsets"], np.int64)),
                             _ptr(_c(g["targets"], np.int32)),
                             _ptr(_c(g["owner"], np.uint8)),
                             _ptr(_c(key, np.int32)), _ptr(tau))
    return tau, int(c)


def even_switch(g: dict, key, sigma) -> tuple:
    sigma = _c(sigma, np.int32).copy()
    c = lib().orc_even_switch(int(g["n"]), _ptr(_c(g["offsets"], np.int64)),
                              _ptr(_c(g["targets"], np.int32)),
                              _ptr(_c(g["owner"], np.uint8)),
                              _ptr(_c(key, np.int32)), _ptr(sigma))
    return sigma, int(c)


def key_hash(key) -> int:
    key = _c(key, np.int32)
    return int(lib().orc_hash(key.size, _ptr(key)))


def initial_strategies(g: dict):
    """sigma_init = the sink for every Even vertex; tau = first row entry."""
    n = int(g["n"])
    off = _c(g["offsets"], np.int64)
    tgt = _c(g["targets"], np.int32)
    own = _c(g["owner"], np.uint8)
    sigma = np.full(n, SINK, np.int32)
    tau = np.where(own == 1, tgt[off[:-1]], SINK).astype(np.int32)
    return sigma, tau


def report_tau(g: dict, tau) -> np.ndarray:
    """tau as a solve reports it: an Odd choice of a dummy d_w (section 3,
    "The algorithm": the dummy only stands in the middle of the original
    edge to w) is reported as w, so the Odd choices of the original
    vertices are edges of the original game."""
    t = np.array(tau, dtype=np.int32, copy=True)
    n0 = int(g["n_orig"])
    dummy_of = np.asarray(g["dummy_of"], dtype=np.int32)
    d = t >= n0
    t[d] = dummy_of[t[d] - n0]
    return t


def solve(game: dict, preprocess_game: bool = True,
          method: int = RANK_KRUSKAL, trace: bool = False,
          max_major: int = 0, max_inner: int = 0, aug: dict = None,
          reset: bool = False) -> dict:
    """Algorithm 1; returns winners, strategies, counts, the last key array
    and (with trace) the hash of every valuation.  reset: SI-Reset (every
    best response starts from the initial Odd strategy)."""
    g = aug if aug is not None else (
        preprocess(game) if preprocess_game else identity(game))
    n = int(g["n"])
    sigma, tau = initial_strategies(g)
    key = np.zeros(n + 1, np.int32)
    st = Stats()
    cap = 100000 if trace else 0
    tr = np.zeros(max(cap, 1), np.uint64)
    rc = lib().orc_solve(n, _ptr(_c(g["offsets"], np.int64)),
                         _ptr(_c(g["targets"], np.int32)),
                         _ptr(_c(g["owner"], np.uint8)),
                         _ptr(_c(g["pri"], np.int32)), method, max_major,
                         max_inner, int(reset), _ptr(sigma), _ptr(tau),
                         _ptr(key),
                         ctypes.byref(st), _ptr(tr) if trace else None, cap)
    n0 = int(g["n_orig"])
    winner = (key[:n0] != KEY_TOP).astype(np.uint8)
    return {"aug": g, "status": int(rc), "winner": winner, "sigma": sigma,
            "tau": tau, "tau_orig": report_tau(g, tau), "key": key,
            "n_major": int(st.n_major),
            "n_valuations": int(st.n_valuations),
            "n_even_switches": int(st.n_even_switches),
            "n_odd_switches": int(st.n_odd_switches),
            "trace": tr[:min(int(st.n_valuations), cap)].copy()
            if trace else None}


# --------------------------------------------------------------------------
# count valuations (oracle/orc_dense.c): priorities may repeat
# --------------------------------------------------------------------------
def dense_preprocess(game: dict) -> dict:
    """The modified game of the count-valuation path: dummies get priority
    0 and, when there is a dummy, the original priorities are raised by 2."""
    n = int(game["n"])
    off = _c(game["offsets"], np.int64)
    tgt = _c(game["targets"], np.int32)
    own = _c(game["owner"], np.uint8)
    pri = _c(game["pri"], np.int32)
    m = int(off[-1])
    off2 = np.zeros(2 * n + 1, np.int64)
    tgt2 = np.zeros(m + n, np.int32)
    own2 = np.zeros(2 * n, np.uint8)
    pri2 = np.zeros(2 * n, np.int32)
    dum = np.zeros(max(n, 1), np.int32)
    n_aug = lib().orc_dense_preprocess(n, _ptr(off), _ptr(tgt), _ptr(own),
                                       _ptr(pri), _ptr(off2), _ptr(tgt2),
                                       _ptr(own2), _ptr(pri2), _ptr(dum))
    if n_aug < 0:
        raise ValueError("preprocessing failed (priority overflow)")
    k = n_aug - n
    m_aug = m + k
    return {"n": n_aug, "m": m_aug, "offsets": off2[:n_aug + 1].copy(),
            "targets": tgt2[:m_aug].copy(), "owner": own2[:n_aug].copy(),
            "pri": pri2[:n_aug].copy(), "dummy_of": dum[:k].copy(),
            "n_orig": n}


def dense_priorities(pri):
    """(values, idx): the distinct priorities in increasing order and each
    vertex's position among them."""
    pri = _c(pri, np.int32)
    values = np.zeros(max(pri.size, 1), np.int32)
    idx = np.zeros(pri.size, np.int32)
    d = lib().orc_dense_priorities(pri.size, _ptr(pri), _ptr(values),
                                   _ptr(idx))
    return values[:d].copy(), idx


def dense_valuation(succ, pri):
    """Count valuations of the play graph succ (SINK for the sink).
    Returns (counts[n+1, d], top[n], values[d], status); row n is the sink
    and column j counts priority values[j]."""
    succ = _c(succ, np.int32)
    values, idx = dense_priorities(pri)
    n, d = succ.size, values.size
    counts = np.zeros((n + 1, d), np.int32)
    top = np.zeros(max(n, 1), np.uint8)
    rc = lib().orc_dense_valuation(n, _ptr(succ), _ptr(idx), d,
                                   _ptr(values), _ptr(counts), _ptr(top))
    return counts, top[:n].copy(), values, int(rc)


def dense_compare(counts, top, values, a: int, b: int) -> int:
    """-1, 0 or 1: Val(a) below, equal to or above Val(b) (n = the sink)."""
    counts = _c(counts, np.int32)
    top = _c(top, np.uint8)
    values = _c(values, np.int32)
    n = top.size
    return int(lib().orc_dense_compare(n, values.size, _ptr(values),
                                       _ptr(counts), _ptr(top), a, b))


def dense_odd_switch(g: dict, counts, top, values, tau) -> tuple:
    tau = _c(tau, np.int32).copy()
    c = lib().orc_dense_odd_switch(
        int(g["n"]), _ptr(_c(g["offsets"], np.int64)),
        _ptr(_c(g["targets"], np.int32)), _ptr(_c(g["owner"], np.uint8)),
        int(np.size(values)), _ptr(_c(values, np.int32)),
        _ptr(_c(counts, np.int32)), _ptr(_c(top, np.uint8)), _ptr(tau))
    return tau, int(c)


def dense_even_switch(g: dict, counts, top, values, sigma) -> tuple:
    sigma = _c(sigma, np.int32).copy()
    c = lib().orc_dense_even_switch(
        int(g["n"]), _ptr(_c(g["offsets"], np.int64)),
        _ptr(_c(g["targets"], np.int32)), _ptr(_c(g["owner"], np.uint8)),
        int(np.size(values)), _ptr(_c(values, np.int32)),
        _ptr(_c(counts, np.int32)), _ptr(_c(top, np.uint8)), _ptr(sigma))
    return sigma, int(c)


def dense_solve(game: dict, preprocess_game: bool = True, trace: bool = False,
                max_major: int = 0, max_inner: int = 0,
                aug: dict = None, br: int = BR_SI) -> dict:
    """Algorithm 1 with count valuations; returns winners, strategies,
    counts, the last valuation (counts, top, values) and with trace the two
    hashes (counts, top flags) of every valuation.  br: BR_SI, BR_SI_RESET
    or BR_BELLMAN_FORD (n_valuations then counts Bellman-Ford rounds)."""
    g = aug if aug is not None else (
        dense_preprocess(game) if preprocess_game else identity(game))
    n = int(g["n"])
    sigma, tau = initial_strategies(g)
    values, _ = dense_priorities(g["pri"])
    d = values.size
    counts = np.zeros((n + 1, d), np.int32)
    top = np.zeros(max(n, 1), np.uint8)
    st = Stats()
    cap = 200000 if trace else 0
    tr = np.zeros(max(cap, 1), np.uint64)
    rc = lib().orc_dense_solve(n, _ptr(_c(g["offsets"], np.int64)),
                               _ptr(_c(g["targets"], np.int32)),
                               _ptr(_c(g["owner"], np.uint8)),
                               _ptr(_c(g["pri"], np.int32)), max_major,
                               max_inner, int(br), _ptr(sigma), _ptr(tau),
                               _ptr(counts), _ptr(top), ctypes.byref(st),
                               _ptr(tr) if trace else None, cap)
    n0 = int(g["n_orig"])
    top = top[:n].copy()
    winner = (top[:n0] == 0).astype(np.uint8)
    nv = int(st.n_valuations)
    return {"aug": g, "status": int(rc), "winner": winner, "sigma": sigma,
            "tau": tau, "tau_orig": report_tau(g, tau), "counts": counts,
            "top": top, "values": values,
            "n_major": int(st.n_major), "n_valuations": nv,
            "n_even_switches": int(st.n_even_switches),
            "n_odd_switches": int(st.n_odd_switches),
            "trace": tr[:min(2 * nv, cap)].reshape(-1, 2).copy()
            if trace else None}


def dense_bellman_ford(g: dict, sigma) -> dict:
    """Bellman-Ford best response against sigma on a count game: returns
    tau, counts, top (no path to the sink), values and the number of rounds."""
    values, idx = dense_priorities(g["pri"])
    n, d = int(g["n"]), values.size
    tau = _c(initial_strategies(g)[1], np.int32).copy()
    counts = np.zeros((n + 1, d), np.int32)
    top = np.zeros(max(n, 1), np.uint8)
    r = lib().orc_dense_bellman_ford(
        n, _ptr(_c(g["offsets"], np.int64)), _ptr(_c(g["targets"], np.int32)),
        _ptr(_c(g["owner"], np.uint8)), _ptr(idx), d, _ptr(values),
        _ptr(_c(sigma, np.int32)), _ptr(tau), _ptr(counts), _ptr(top))
    return {"tau": tau, "counts": counts, "top": top[:n].copy(),
            "values": values, "rounds": int(r)}
