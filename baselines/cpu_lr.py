"""ctypes wrapper of baselines/cpu_lr.c: a multi-core CPU best-response
iteration with parallel list ranking (the paper's CPU-LR, section 6), timed
by bench.py next to the single-threaded oracle.  Neither the device library
nor the oracle uses it."""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_lr.c")
LIB_PATH = os.path.join(HERE, "libcpulr.so")

_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        subprocess.run(["gcc", "-O3", "-march=native", "-fopenmp", "-shared",
                        "-fPIC", "-o", LIB_PATH, SRC], check=True)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.cl_valuation.argtypes = [I64, P, P, P, P, I32, P, P]
        L.cl_valuation.restype = I32
        L.cl_odd_switch.argtypes = [I64, P, P, P, P, P, I32]
        L.cl_odd_switch.restype = I64
        L.cl_max_threads.restype = I32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def orders(pri):
    """The vertices in increasing priority and in signed-priority order
    (odd priorities descending, then even ascending)."""
    pri = np.asarray(pri, np.int64)
    by_pri = np.argsort(pri, kind="stable").astype(np.int32)
    sk = np.where(pri & 1, -pri, pri + (1 << 40))
    by_signed = np.argsort(sk, kind="stable").astype(np.int32)
    return by_pri, by_signed


def valuation(succ, pri, by_pri=None, by_signed=None, threads: int = 0):
    """Rank keys (key[n] is the sink; KEY_TOP for top vertices), the finite
    count (sink included) and the status (0 ok, 2 an odd cycle)."""
    succ = np.ascontiguousarray(succ, np.int32)
    pri = np.ascontiguousarray(pri, np.int32)
    if by_pri is None:
        by_pri, by_signed = orders(pri)
    n = succ.size
    key = np.zeros(n + 1, np.int32)
    nf = ctypes.c_int64()
    rc = lib().cl_valuation(n, _p(succ), _p(pri), _p(by_pri), _p(by_signed),
                            threads, _p(key), ctypes.byref(nf))
    return key, int(nf.value), int(rc)


def odd_switch(g: dict, key, tau, threads: int = 0):
    tau = np.array(tau, np.int32, copy=True)
    c = lib().cl_odd_switch(int(g["n"]),
                            _p(np.ascontiguousarray(g["offsets"], np.int64)),
                            _p(np.ascontiguousarray(g["targets"], np.int32)),
                            _p(np.ascontiguousarray(g["owner"], np.uint8)),
                            _p(np.ascontiguousarray(key, np.int32)), _p(tau),
                            threads)
    return tau, int(c)


def time_iterations(g: dict, sigma, tau, iters: int = 3,
                    threads: int = 0) -> dict:
    """Seconds per best-response iteration (valuation + All_Odd) from the
    given strategies on the modified game g, median of `iters`."""
    by_pri, by_signed = orders(g["pri"])
    own = np.asarray(g["owner"])
    ts = []
    for _ in range(iters):
        t0 = time.perf_counter()
        succ = np.where(own == 1, tau, sigma).astype(np.int32)
        key, nf, rc = valuation(succ, g["pri"], by_pri, by_signed, threads)
        assert rc == 0
        tau, _ = odd_switch(g, key, tau, threads)
        ts.append(time.perf_counter() - t0)
    return {"seconds_median": float(np.median(ts)),
            "threads": threads if threads > 0 else lib().cl_max_threads()}
