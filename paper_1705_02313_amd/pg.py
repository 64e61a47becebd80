"""Python binding of the C ABI in include/pg.h (ctypes; argument marshalling
only -- every step of the solver runs in the HIP library).

Arrays may be numpy arrays (host memory) or torch tensors on the GPU (device
memory, passed with PG_PTR_DEVICE on torch's current stream).  The library
must have been built (``python -m paper_1705_02313_amd.build_lib``); without
it every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpgsi.so")

PG_OK, PG_EINVAL, PG_ENOMEM, PG_EDEVICE = 0, 1, 2, 3
PG_EITERLIMIT, PG_EINADMISSIBLE, PG_EINTERNAL = 4, 5, 6
PG_SINK = -1
PG_KEY_TOP = 2**31 - 1
PG_PTR_DEVICE, PG_NO_PREPROCESS, PG_OFFSETS_I32 = 1, 2, 4
PG_CAREFUL_WALKS, PG_COUNT_VALUATION, PG_NO_GRAPH = 8, 16, 32
PG_HOST_REDUCED_LIST = 64
PG_SWITCH_ROWS, PG_SWITCH_BUCKETS = 128, 256
PG_KEEP_DUMMIES = 512
PG_ODD_REGION = 1024
PG_BR_SI, PG_BR_SI_RESET, PG_BR_BELLMAN_FORD = 0, 1, 2
PG_NOALLOC_MAX_VERTICES, PG_NOALLOC_MAX_EDGES = 65536, 1048576

STATUS_NAMES = {0: "PG_OK", 1: "PG_EINVAL", 2: "PG_ENOMEM", 3: "PG_EDEVICE",
                4: "PG_EITERLIMIT", 5: "PG_EINADMISSIBLE", 6: "PG_EINTERNAL"}

EXPORTS = ["pg_load_csr", "pg_game_info", "pg_count_info", "pg_export_game",
           "pg_initial_strategies", "pg_valuation", "pg_valuation_counts",
           "pg_best_response",
           "pg_solve", "pg_profile_enable", "pg_profile_kinds",
           "pg_profile_read", "pg_batch_create", "pg_batch_submit",
           "pg_batch_submit_many", "pg_batch_poll_many",
           "pg_batch_step", "pg_batch_poll", "pg_batch_finished",
           "pg_batch_info", "pg_batch_free",
           "pg_free", "pg_release_cache", "pg_solve_noalloc",
           "pg_get_tuning", "pg_set_tuning", "pg_tuning_table",
           "pg_last_error"]


def release_cache():
    """Hands the memory that freed games left cached back to the runtime
    (pg_release_cache)."""
    _check(lib().pg_release_cache())


class PgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class SolveOpts(ctypes.Structure):
    _fields_ = [("max_major", ctypes.c_int32), ("max_inner", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("best_response", ctypes.c_int32),
                ("init_sigma", ctypes.c_void_p), ("init_tau", ctypes.c_void_p),
                ("trace_cap", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("trace_key_hash", ctypes.c_void_p),
                ("trace_finite", ctypes.c_void_p),
                ("trace_switches", ctypes.c_void_p),
                ("trace_ms", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("n_aug", ctypes.c_int64), ("m_aug", ctypes.c_int64),
                ("n_major", ctypes.c_int64), ("n_valuations", ctypes.c_int64),
                ("n_odd_switches", ctypes.c_int64),
                ("n_even_switches", ctypes.c_int64),
                ("seconds", ctypes.c_double),
                ("iteration_ms", ctypes.c_double),
                ("n_traced", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def write_trace_jsonl(path: str, out: dict, extra: dict = None):
    """Appends one JSON line per traced valuation of a solve (the dict
    Game.solve(trace=...) returns): its index, key hash, finite vertices,
    Odd switches and device milliseconds, plus the `extra` fields."""
    import json
    tr = out.get("trace")
    if tr is None:
        raise ValueError("the solve was run without a trace")
    with open(path, "a") as f:
        for i in range(len(tr["finite"])):
            rec = {"valuation": i, "key_hash": int(tr["key_hash"][i]),
                   "finite": int(tr["finite"][i]),
                   "odd_switches": int(tr["switches"][i]),
                   "device_ms": float(tr["ms"][i])}
            if extra:
                rec.update(extra)
            f.write(json.dumps(rec) + "\n")


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1705_02313_amd.build_lib`")
        # torch ships its own HIP runtime (same soname as the system one).
        # Loading torch first makes the library bind to that runtime, so one
        # process never holds two HIP runtimes (a second one leaves torch
        # without devices).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, U32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                            ctypes.c_uint32)
        L.pg_load_csr.argtypes = [I64, I64, P, P, P, P, U32, P,
                                  ctypes.POINTER(P)]
        L.pg_game_info.argtypes = [P] + [ctypes.POINTER(I64)] * 4
        L.pg_count_info.argtypes = [P, ctypes.POINTER(I32), P]
        L.pg_valuation_counts.argtypes = [P, P, P, P, P, ctypes.POINTER(I64),
                                          U32, P]
        L.pg_export_game.argtypes = [P, P, P, P, P, U32, P]
        L.pg_initial_strategies.argtypes = [P, P, P, U32, P]
        L.pg_valuation.argtypes = [P, P, P, P, ctypes.POINTER(I64), U32, P]
        L.pg_best_response.argtypes = [P, P, P, P, ctypes.POINTER(I32), I32,
                                       U32, P]
        L.pg_solve.argtypes = [P, ctypes.POINTER(SolveOpts), P, P, P,
                               ctypes.POINTER(Stats), P]
        L.pg_release_cache.argtypes = []
        L.pg_profile_enable.argtypes = [P, I32]
        L.pg_profile_kinds.argtypes = []
        L.pg_profile_read.argtypes = [P, I32, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(I64),
                                      ctypes.POINTER(ctypes.c_double)]
        L.pg_batch_create.argtypes = [I64, I64, I32, P, ctypes.POINTER(P)]
        L.pg_batch_submit.argtypes = [P, I64, I64, P, P, P, P, U32,
                                      ctypes.POINTER(I64)]
        L.pg_batch_submit_many.argtypes = [P, I32, P, P, P, P, P, P, U32, P,
                                           P]
        L.pg_batch_poll_many.argtypes = [P, I32, P, P, P, P, P, P, U32]
        L.pg_batch_step.argtypes = [P] + [ctypes.POINTER(I32)] * 3
        L.pg_batch_poll.argtypes = [P, I64, ctypes.POINTER(I32), P, P, P,
                                    ctypes.POINTER(Stats), U32]
        L.pg_batch_info.argtypes = [P, ctypes.POINTER(I32),
                                    ctypes.POINTER(I32), ctypes.POINTER(I64),
                                    ctypes.POINTER(I64)]
        L.pg_batch_finished.argtypes = [P, P, I32, ctypes.POINTER(I32)]
        L.pg_batch_free.argtypes = [P]
        L.pg_free.argtypes = [P]
        L.pg_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.pg_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.pg_tuning_table.argtypes = [ctypes.POINTER(Tuning),
                                      ctypes.POINTER(I64), I32]
        L.pg_solve_noalloc.argtypes = [I64, I64, P, P, P, P, U32,
                                       ctypes.POINTER(SolveOpts), P, P, P,
                                       ctypes.POINTER(Stats), P]
        L.pg_last_error.argtypes = []
        L.pg_last_error.restype = ctypes.c_char_p
        for name in EXPORTS[:-1]:
            getattr(L, name).restype = ctypes.c_int
        L.pg_tuning_table.restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(status: int):
    if status != PG_OK:
        raise PgError(status, lib().pg_last_error().decode())


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        return ctypes.c_void_p(x.data_ptr())
    return x.ctypes.data_as(ctypes.c_void_p)


def _pinned_bytes(nbytes: int) -> np.ndarray:
    """A uint8 array of nbytes in pinned host memory (torch's caching host
    allocator), or in ordinary memory when that is not available."""
    try:
        import torch
        return torch.empty(max(nbytes, 1), dtype=torch.uint8,
                           pin_memory=True).numpy()[:nbytes]
    except (ImportError, RuntimeError):
        return np.empty(nbytes, np.uint8)


def _stream(device: bool):
    if not device:
        return None
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Tuning(ctypes.Structure):
    """pg_tuning: launch and walk parameters of the rank valuation."""
    _fields_ = [("stride0", ctypes.c_int32), ("per_thread", ctypes.c_int32),
                ("walk_full", ctypes.c_int32), ("walk_round", ctypes.c_int32),
                ("walk_rounds", ctypes.c_int32),
                ("walk_block", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def tuning_table() -> list:
    """The library's table: [(min_n_aug, tuning dict), ...]."""
    n = int(lib().pg_tuning_table(None, None, 0))
    ent = (Tuning * n)()
    lo = (ctypes.c_int64 * n)()
    lib().pg_tuning_table(ent, lo, n)
    return [(int(lo[i]), ent[i].as_dict()) for i in range(n)]


def solve_noalloc(g: dict, device: bool = False, max_major: int = 0,
                  max_inner: int = 0, best_response: int = PG_BR_SI,
                  keep_dummies: bool = False, odd_region: bool = False) -> dict:
    """pg_solve_noalloc: load, solve and release in one call that allocates
    no device memory (the library's static scratch), for games of at most
    PG_NOALLOC_MAX_VERTICES vertices and PG_NOALLOC_MAX_EDGES edges.  The
    caller's outputs are sized 2 n (n_aug <= 2 n) and cut to n_aug (to n
    with ``odd_region``, PG_ODD_REGION)."""
    n = int(g["n"])
    if device:
        import torch
        arr = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda()
               for k in ("offsets", "targets", "owner", "pri")}
        off_i32 = arr["offsets"].dtype == torch.int32
        if not off_i32:
            arr["offsets"] = arr["offsets"].to(torch.int64)
        arr["targets"] = arr["targets"].to(torch.int32)
        arr["owner"] = arr["owner"].to(torch.uint8)
        arr["pri"] = arr["pri"].to(torch.int32)
        out = lambda c, t: torch.empty(c, dtype=t, device="cuda")  # noqa
        dt = {"u8": torch.uint8, "i32": torch.int32}
    else:
        off = np.ascontiguousarray(g["offsets"])
        off_i32 = off.dtype == np.int32
        arr = {"offsets": off if off_i32 else off.astype(np.int64),
               "targets": np.ascontiguousarray(g["targets"], np.int32),
               "owner": np.ascontiguousarray(g["owner"], np.uint8),
               "pri": np.ascontiguousarray(g["pri"], np.int32)}
        out = lambda c, t: np.empty(c, dtype=t)  # noqa
        dt = {"u8": np.uint8, "i32": np.int32}
    m = int(arr["targets"].numel() if device else arr["targets"].size)
    flags = (PG_PTR_DEVICE if device else 0) | \
        (PG_OFFSETS_I32 if off_i32 else 0) | \
        (PG_ODD_REGION if odd_region else 0)
    oflags = (PG_PTR_DEVICE if device else 0) | \
        (PG_KEEP_DUMMIES if keep_dummies else 0)
    opts = SolveOpts(max_major, max_inner, oflags, best_response, None, None,
                     0, 0, None, None, None, None)
    winner = out(n, dt["u8"])
    sigma = out(2 * n, dt["i32"])
    tau = out(2 * n, dt["i32"])
    st = Stats()
    _check(lib().pg_solve_noalloc(
        n, m, _ptr(arr["offsets"]), _ptr(arr["targets"]), _ptr(arr["owner"]),
        _ptr(arr["pri"]), flags, ctypes.byref(opts), _ptr(winner),
        _ptr(sigma), _ptr(tau), ctypes.byref(st), _stream(device)))
    na = n if odd_region else int(st.n_aug)
    return {"winner": winner, "sigma": sigma[:na], "tau": tau[:na],
            "stats": st.as_dict()}


class Game:
    """A game loaded on the device (modified by preprocessing unless
    ``preprocess=False``; ``careful_walks=True`` sets PG_CAREFUL_WALKS,
    ``count_valuation=True`` PG_COUNT_VALUATION, ``graph=False``
    PG_NO_GRAPH, ``host_reduced_list=True`` PG_HOST_REDUCED_LIST,
    ``switch="rows"`` PG_SWITCH_ROWS and ``switch="buckets"``
    PG_SWITCH_BUCKETS; ``switch=None`` lets the library choose by size;
    ``odd_region=True`` PG_ODD_REGION: Odd's own winning region is removed
    instead of inserting dummies, and solve() then takes and returns n
    entries in the original ids).  Games whose priorities repeat use count
    valuations by themselves (``self.d > 0``)."""

    def __init__(self, offsets, targets, owner, priority, n: int = None,
                 preprocess: bool = True, careful_walks: bool = False,
                 count_valuation: bool = False, graph: bool = True,
                 host_reduced_list: bool = False, switch: str = None,
                 odd_region: bool = False):
        if switch not in (None, "rows", "buckets"):
            raise ValueError("switch must be None, 'rows' or 'buckets'")
        device = _is_torch(targets)
        if device:
            import torch
            offsets = offsets.contiguous()
            targets = targets.to(torch.int32).contiguous()
            owner = owner.to(torch.uint8).contiguous()
            priority = priority.to(torch.int32).contiguous()
            off_i32 = offsets.dtype == torch.int32
            if not off_i32:
                offsets = offsets.to(torch.int64)
            m = int(targets.numel())
        else:
            offsets = np.ascontiguousarray(offsets)
            off_i32 = offsets.dtype == np.int32
            if not off_i32:
                offsets = offsets.astype(np.int64, copy=False)
            targets = np.ascontiguousarray(targets, dtype=np.int32)
            owner = np.ascontiguousarray(owner, dtype=np.uint8)
            priority = np.ascontiguousarray(priority, dtype=np.int32)
            m = int(targets.size)
        if n is None:
            n = int(offsets.numel() if device else offsets.size) - 1
        flags = (PG_PTR_DEVICE if device else 0) | \
            (0 if preprocess else PG_NO_PREPROCESS) | \
            (PG_OFFSETS_I32 if off_i32 else 0) | \
            (PG_CAREFUL_WALKS if careful_walks else 0) | \
            (PG_COUNT_VALUATION if count_valuation else 0) | \
            (0 if graph else PG_NO_GRAPH) | \
            (PG_HOST_REDUCED_LIST if host_reduced_list else 0) | \
            {None: 0, "rows": PG_SWITCH_ROWS,
             "buckets": PG_SWITCH_BUCKETS}[switch] | \
            (PG_ODD_REGION if odd_region else 0)
        h = ctypes.c_void_p()
        _check(lib().pg_load_csr(n, m, _ptr(offsets), _ptr(targets),
                                 _ptr(owner), _ptr(priority), flags,
                                 _stream(device), ctypes.byref(h)))
        self._h = h
        self.device = device
        self.odd_region = bool(odd_region)
        vals = [ctypes.c_int64() for _ in range(4)]
        _check(lib().pg_game_info(self._h, *[ctypes.byref(v) for v in vals]))
        self.n, self.m, self.n_aug, self.m_aug = [int(v.value) for v in vals]
        d = ctypes.c_int32()
        values = np.zeros(32, np.int32)
        _check(lib().pg_count_info(self._h, ctypes.byref(d), _ptr(values)))
        self.d = int(d.value)
        self.values = values[:self.d].copy()

    @classmethod
    def from_dict(cls, g: dict, device: bool = False, preprocess: bool = True,
                  careful_walks: bool = False, count_valuation: bool = False,
                  graph: bool = True, host_reduced_list: bool = False,
                  switch: str = None, odd_region: bool = False):
        kw = {"n": int(g["n"]), "preprocess": preprocess,
              "careful_walks": careful_walks,
              "count_valuation": count_valuation, "graph": graph,
              "host_reduced_list": host_reduced_list, "switch": switch,
              "odd_region": odd_region}
        if device:
            import torch
            t = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda()
                 for k in ("offsets", "targets", "owner", "pri")}
            return cls(t["offsets"], t["targets"], t["owner"], t["pri"], **kw)
        return cls(g["offsets"], g["targets"], g["owner"], g["pri"], **kw)

    # -- helpers -------------------------------------------------------------
    def _out(self, count: int, dtype):
        if self.device:
            import torch
            tdt = {np.int32: torch.int32, np.int64: torch.int64,
                   np.uint8: torch.uint8}[dtype]
            return torch.empty(count, dtype=tdt, device="cuda")
        return np.empty(count, dtype=dtype)

    def _in(self, x, dtype=np.int32):
        if self.device:
            import torch
            if not _is_torch(x):
                x = torch.from_numpy(np.ascontiguousarray(x, dtype=dtype))
            return x.to(device="cuda", dtype=torch.int32).contiguous()
        if _is_torch(x):
            x = x.cpu().numpy()
        return np.ascontiguousarray(x, dtype=dtype)

    @property
    def _flags(self) -> int:
        return PG_PTR_DEVICE if self.device else 0

    # -- calls ---------------------------------------------------------------
    def export(self) -> dict:
        off = np.empty(self.n_aug + 1, np.int64)
        tgt = np.empty(self.m_aug, np.int32)
        own = np.empty(self.n_aug, np.uint8)
        pri = np.empty(self.n_aug, np.int32)
        _check(lib().pg_export_game(self._h, _ptr(off), _ptr(tgt), _ptr(own),
                                    _ptr(pri), 0, _stream(self.device)))
        return {"n": self.n_aug, "m": self.m_aug, "offsets": off,
                "targets": tgt, "owner": own, "pri": pri}

    def initial_strategies(self):
        sigma = self._out(self.n_aug, np.int32)
        tau = self._out(self.n_aug, np.int32)
        _check(lib().pg_initial_strategies(self._h, _ptr(sigma), _ptr(tau),
                                           self._flags,
                                           _stream(self.device)))
        return sigma, tau

    def valuation(self, sigma, tau):
        """Returns (key[n_aug+1], n_finite)."""
        sigma = self._in(sigma)
        tau = self._in(tau)
        key = self._out(self.n_aug + 1, np.int32)
        nf = ctypes.c_int64()
        _check(lib().pg_valuation(self._h, _ptr(sigma), _ptr(tau), _ptr(key),
                                  ctypes.byref(nf), self._flags,
                                  _stream(self.device)))
        return key, int(nf.value)

    def valuation_counts(self, sigma, tau):
        """Count valuations: returns (counts[n_aug+1, d], top[n_aug],
        n_finite); column j counts priority self.values[j]."""
        sigma = self._in(sigma)
        tau = self._in(tau)
        counts = self._out((self.n_aug + 1) * self.d, np.int32)
        top = self._out(self.n_aug, np.uint8)
        nf = ctypes.c_int64()
        _check(lib().pg_valuation_counts(self._h, _ptr(sigma), _ptr(tau),
                                         _ptr(counts), _ptr(top),
                                         ctypes.byref(nf), self._flags,
                                         _stream(self.device)))
        return counts.reshape(self.n_aug + 1, self.d), top, int(nf.value)

    def best_response(self, sigma, tau, max_inner: int = 0):
        """Returns (tau, key, n_valuations); key is None for a game with
        count valuations."""
        sigma = self._in(sigma)
        tau = self._in(tau)
        tau = tau.clone() if self.device else tau.copy()
        key = None if self.d else self._out(self.n_aug + 1, np.int32)
        nv = ctypes.c_int32()
        _check(lib().pg_best_response(self._h, _ptr(sigma), _ptr(tau),
                                      _ptr(key), ctypes.byref(nv), max_inner,
                                      self._flags, _stream(self.device)))
        return tau, key, int(nv.value)

    def solve(self, max_major: int = 0, max_inner: int = 0,
              best_response: int = PG_BR_SI, init_sigma=None, init_tau=None,
              trace: int = 0, keep_dummies: bool = False,
              checkpoint: bool = False) -> dict:
        """Algorithm 1 (pg_solve).  init_sigma / init_tau: a warm start (in
        the modified game's ids).  trace: valuations to trace (key hash,
        finite vertices, switches, device ms; out["trace"]).  keep_dummies:
        tau in the modified game's ids (PG_KEEP_DUMMIES).  checkpoint: a
        cap that stops the run returns {"stopped": True, "sigma", "tau",
        "stats"} instead of raising."""
        flags = self._flags | (PG_KEEP_DUMMIES if keep_dummies else 0)
        isg = None if init_sigma is None else self._in(init_sigma)
        itau = None if init_tau is None else self._in(init_tau)
        tr = None
        if trace:
            tr = {"key_hash": np.zeros(trace, np.uint64),
                  "finite": np.zeros(trace, np.int64),
                  "switches": np.zeros(trace, np.int64),
                  "ms": np.zeros(trace, np.float32)}
        opts = SolveOpts(max_major, max_inner, flags, best_response,
                         _ptr(isg), _ptr(itau), int(trace), 0,
                         *([_ptr(tr[k]) for k in ("key_hash", "finite",
                                                  "switches", "ms")]
                           if tr else [None] * 4))
        winner = self._out(self.n, np.uint8)
        ns = self.n if self.odd_region else self.n_aug
        sigma = self._out(ns, np.int32)
        tau = self._out(ns, np.int32)
        st = Stats()
        rc = lib().pg_solve(self._h, ctypes.byref(opts), _ptr(winner),
                            _ptr(sigma), _ptr(tau), ctypes.byref(st),
                            _stream(self.device))
        if tr is not None:
            k = int(st.n_traced)
            tr = {key: v[:k].copy() for key, v in tr.items()}
        if rc == PG_EITERLIMIT and checkpoint:
            return {"stopped": True, "sigma": sigma, "tau": tau,
                    "stats": st.as_dict(), "trace": tr}
        _check(rc)
        return {"winner": winner, "sigma": sigma, "tau": tau,
                "stats": st.as_dict(), "trace": tr}

    def tuning(self) -> dict:
        """The game's launch and walk parameters (pg_get_tuning)."""
        t = Tuning()
        _check(lib().pg_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Replaces some of the parameters (pg_set_tuning)."""
        cur = self.tuning()
        cur.update(kw)
        t = Tuning(**cur)
        _check(lib().pg_set_tuning(self._h, ctypes.byref(t)))

    def profile(self, on: bool = True):
        """Enables (and clears) or disables the per-kernel event profiler."""
        _check(lib().pg_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kernel kind: {"ms", "calls", "bytes"}} for kinds that ran."""
        out = {}
        for k in range(lib().pg_profile_kinds()):
            name = ctypes.c_char_p()
            ms = ctypes.c_double()
            calls = ctypes.c_int64()
            by = ctypes.c_double()
            _check(lib().pg_profile_read(self._h, k, ctypes.byref(name),
                                         ctypes.byref(ms), ctypes.byref(calls),
                                         ctypes.byref(by)))
            if calls.value:
                out[name.value.decode()] = {"ms": ms.value,
                                            "calls": int(calls.value),
                                            "bytes": by.value}
        return out

    def free(self):
        if getattr(self, "_h", None):
            lib().pg_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


class Batch:
    """Many games solved together on the device (see pg_batch_* in pg.h)."""

    def __init__(self, max_vertices: int, max_edges: int,
                 max_games: int = 65536, stream=None):
        h = ctypes.c_void_p()
        _check(lib().pg_batch_create(max_vertices, max_edges, max_games,
                                     stream, ctypes.byref(h)))
        self._h = h

    def submit(self, g: dict, device: bool = False) -> int:
        """Queues a game (dict as produced by synth); returns its ticket.
        May run on another thread than step() (pg_batch_submit)."""
        if device:
            import torch
            arr = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda()
                   for k in ("offsets", "targets", "owner", "pri")}
            off = arr["offsets"]
            flags = PG_PTR_DEVICE | (PG_OFFSETS_I32 if off.dtype ==
                                     torch.int32 else 0)
            arr["offsets"] = off if off.dtype == torch.int32 else \
                off.to(torch.int64)
            arr["targets"] = arr["targets"].to(torch.int32)
            arr["owner"] = arr["owner"].to(torch.uint8)
            arr["pri"] = arr["pri"].to(torch.int32)
            # pg_batch_submit reads them on the batch's own stream: the
            # copies and conversions queued on torch's stream finish first
            torch.cuda.current_stream().synchronize()
        else:
            off = np.ascontiguousarray(g["offsets"])
            flags = PG_OFFSETS_I32 if off.dtype == np.int32 else 0
            arr = {"offsets": off if off.dtype == np.int32 else
                   off.astype(np.int64),
                   "targets": np.ascontiguousarray(g["targets"], np.int32),
                   "owner": np.ascontiguousarray(g["owner"], np.uint8),
                   "pri": np.ascontiguousarray(g["pri"], np.int32)}
        t = ctypes.c_int64()
        _check(lib().pg_batch_submit(self._h, int(g["n"]), int(g["m"]),
                                     _ptr(arr["offsets"]),
                                     _ptr(arr["targets"]), _ptr(arr["owner"]),
                                     _ptr(arr["pri"]), flags,
                                     ctypes.byref(t)))
        return int(t.value)

    def submit_many(self, games: list) -> list:
        """Queues several games in one call (pg_batch_submit_many): their
        preprocessing runs over their disjoint union.  Returns one entry per
        game: its ticket, or the PgError that refused it."""
        if not games:
            return []
        i32 = all(np.asarray(g["offsets"]).dtype == np.int32 for g in games)
        odt = np.int32 if i32 else np.int64
        keep = []   # the arrays must live until the call returns
        cnt = len(games)
        ns = np.array([int(g["n"]) for g in games], np.int64)
        ms = np.array([int(g["m"]) for g in games], np.int64)
        ptrs = {k: (ctypes.c_void_p * cnt)() for k in
                ("offsets", "targets", "owner", "pri")}
        for i, g in enumerate(games):
            arr = {"offsets": np.ascontiguousarray(g["offsets"], odt),
                   "targets": np.ascontiguousarray(g["targets"], np.int32),
                   "owner": np.ascontiguousarray(g["owner"], np.uint8),
                   "pri": np.ascontiguousarray(g["pri"], np.int32)}
            keep.append(arr)
            for k, a in arr.items():
                ptrs[k][i] = a.ctypes.data
        tickets = np.full(cnt, -1, np.int64)
        status = np.zeros(cnt, np.int32)
        _check(lib().pg_batch_submit_many(
            self._h, cnt, _ptr(ns), _ptr(ms), ptrs["offsets"],
            ptrs["targets"], ptrs["owner"], ptrs["pri"],
            PG_OFFSETS_I32 if i32 else 0, _ptr(tickets), _ptr(status)))
        out = []
        for i in range(cnt):
            if status[i] == PG_OK:
                out.append(int(tickets[i]))
            else:
                out.append(PgError(int(status[i]),
                                   f"game {i} refused by the batch"))
        return out

    def step(self):
        """One step; returns (live, queued, finished by this step)."""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pg_batch_step(self._h, ctypes.byref(a), ctypes.byref(b),
                                   ctypes.byref(c)))
        return int(a.value), int(b.value), int(c.value)

    def poll(self, ticket: int):
        """None while running; else a dict like Game.solve() (host arrays)."""
        st = Stats()
        done = ctypes.c_int32()
        _check(lib().pg_batch_poll(self._h, ticket, ctypes.byref(done), None,
                                   None, None, ctypes.byref(st), 0))
        if not done.value:
            return None
        n = int(st.n)
        n_aug = int(st.n_aug)
        winner = np.empty(n, np.uint8)
        sigma = np.empty(n_aug, np.int32)
        tau = np.empty(n_aug, np.int32)
        _check(lib().pg_batch_poll(self._h, ticket, ctypes.byref(done),
                                   _ptr(winner), _ptr(sigma), _ptr(tau),
                                   ctypes.byref(st), 0))
        return {"winner": winner, "sigma": sigma, "tau": tau,
                "stats": st.as_dict()}

    def poll_many(self, tickets) -> list:
        """poll() for several tickets with one wait for all the copies
        (pg_batch_poll_many): a result dict per finished ticket, None for
        the others."""
        tickets = np.ascontiguousarray(tickets, np.int64)
        cnt = int(tickets.size)
        if cnt == 0:
            return []
        done = np.zeros(cnt, np.int32)
        st = (Stats * cnt)()
        _check(lib().pg_batch_poll_many(self._h, cnt, _ptr(tickets),
                                        _ptr(done), None, None, None, st, 0))
        outs = [None] * cnt
        pw = (ctypes.c_void_p * cnt)()
        ps = (ctypes.c_void_p * cnt)()
        pt = (ctypes.c_void_p * cnt)()
        # every output in one pinned host block (the copies then go to it
        # directly instead of through the runtime's bounce buffers); the
        # result arrays are views that keep the block alive
        lay, total = [], 0
        for i in range(cnt):
            if done[i]:
                n, na = int(st[i].n), int(st[i].n_aug)
                lay.append((i, total, n, na))
                total += (n + 15) // 16 * 16 + 8 * na
        buf = _pinned_bytes(total)
        for i, at, n, na in lay:
            w = buf[at:at + n]
            sg = buf[at + (n + 15) // 16 * 16:][:4 * na].view(np.int32)
            ta = buf[at + (n + 15) // 16 * 16 + 4 * na:][:4 * na].view(
                np.int32)
            outs[i] = (w, sg, ta)
            pw[i], ps[i], pt[i] = (a.ctypes.data for a in outs[i])
        _check(lib().pg_batch_poll_many(self._h, cnt, _ptr(tickets),
                                        _ptr(done), pw, ps, pt, st, 0))
        return [None if o is None else
                {"winner": o[0], "sigma": o[1], "tau": o[2],
                 "stats": st[i].as_dict()} for i, o in enumerate(outs)]

    def finished(self) -> list:
        """Tickets of finished games not yet polled."""
        c = ctypes.c_int32()
        _check(lib().pg_batch_finished(self._h, None, 0, ctypes.byref(c)))
        if c.value == 0:
            return []
        buf = np.empty(c.value, np.int64)
        _check(lib().pg_batch_finished(self._h, _ptr(buf), c.value,
                                       ctypes.byref(c)))
        return [int(x) for x in buf[:c.value]]

    def info(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        c, d = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().pg_batch_info(self._h, ctypes.byref(a), ctypes.byref(b),
                                   ctypes.byref(c), ctypes.byref(d)))
        return {"live": int(a.value), "queued": int(b.value),
                "arena_vertices": int(c.value), "arena_edges": int(d.value)}

    def free(self):
        if getattr(self, "_h", None):
            lib().pg_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()
