"""The built HIP library loads on a machine without a GPU and exports every
function include/pg.h declares (no compute calls here)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pg_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pg_load_csr", "pg_best_response", "pg_solve",
                 "pg_valuation", "pg_free", "pg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1705_02313_amd import pg
    if not os.path.exists(pg.LIB_PATH):
        pytest.fail("libpgsi.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(pg.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(pg.EXPORTS) <= set(declared_functions())


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1705_02313_amd import pg
    monkeypatch.setattr(pg, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pg, "_lib", None)
    with pytest.raises(ImportError):
        pg.lib()


def header_constants():
    """NAME = value entries of the header's enums and its integer #defines."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for name, val in re.findall(r"\b(PG_[A-Z0-9_]+)\s*=\s*([0-9]+)u?\b", text):
        out[name] = int(val)
    for name, val in re.findall(r"#define\s+(PG_[A-Z0-9_]+)\s+\(?(-?[0-9]+)\)?",
                                text):
        out[name] = int(val)
    return out


def test_binding_constants_mirror_the_header():
    from paper_1705_02313_amd import pg
    consts = header_constants()
    for name in ("PG_OK", "PG_EINVAL", "PG_ENOMEM", "PG_EDEVICE",
                 "PG_EITERLIMIT", "PG_EINADMISSIBLE", "PG_EINTERNAL",
                 "PG_PTR_DEVICE", "PG_NO_PREPROCESS", "PG_OFFSETS_I32",
                 "PG_CAREFUL_WALKS", "PG_COUNT_VALUATION", "PG_NO_GRAPH",
                 "PG_HOST_REDUCED_LIST", "PG_SWITCH_ROWS", "PG_SWITCH_BUCKETS",
                 "PG_KEEP_DUMMIES", "PG_BR_SI", "PG_BR_SI_RESET", "PG_BR_BELLMAN_FORD",
                 "PG_SINK", "PG_KEY_TOP", "PG_NOALLOC_MAX_VERTICES",
                 "PG_NOALLOC_MAX_EDGES", "PG_NOALLOC_SCRATCH_MIB"):
        assert name in consts, name
        if hasattr(pg, name):
            assert getattr(pg, name) == consts[name], name
    # the load flags are distinct bits
    flags = [consts[k] for k in consts if k in (
        "PG_PTR_DEVICE", "PG_NO_PREPROCESS", "PG_OFFSETS_I32",
        "PG_CAREFUL_WALKS", "PG_COUNT_VALUATION", "PG_NO_GRAPH",
        "PG_HOST_REDUCED_LIST", "PG_SWITCH_ROWS", "PG_SWITCH_BUCKETS",
        "PG_KEEP_DUMMIES")]
    assert all(f & (f - 1) == 0 for f in flags)
    assert len(set(flags)) == len(flags)


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of pg_solve_opts and pg_stats have the header's
    size and field offsets (a C program built with gcc prints them)."""
    import shutil
    import subprocess
    from paper_1705_02313_amd import pg
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    prog = ["#include <stddef.h>", "#include <stdio.h>",
            f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in (("pg_solve_opts", pg.SolveOpts),
                       ("pg_stats", pg.Stats), ("pg_tuning", pg.Tuning)):
        prog.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            prog.append(f'printf("{cname} {f} %zu\\n", '
                        f'offsetof({cname}, {f}));')
    prog.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True,
                         text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln}
    for cname, cls in (("pg_solve_opts", pg.SolveOpts),
                       ("pg_stats", pg.Stats), ("pg_tuning", pg.Tuning)):
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_tuning_table_is_ordered_and_valid():
    """The table read through the library (no device needed): entries by
    increasing size bound from 0, every value in its documented set."""
    from paper_1705_02313_amd import pg
    table = pg.tuning_table()
    assert table and table[0][0] == 0
    bounds = [lo for lo, _ in table]
    assert bounds == sorted(set(bounds))
    for _, t in table:
        assert t["stride0"] in (8, 16, 32, 64)
        assert t["per_thread"] in (1, 2, 4, 8)
        assert 2 <= t["walk_full"] <= 64
        assert 8 <= t["walk_round"] <= 256
        assert 1 <= t["walk_rounds"] <= 8
        assert t["walk_block"] in (64, 128, 256)


def test_odd_region_flag_conflict_is_refused_before_the_device():
    """PG_ODD_REGION with PG_NO_PREPROCESS is refused by the argument checks,
    which run before any device call."""
    import numpy as np
    from paper_1705_02313_amd import pg
    consts = header_constants()
    assert consts["PG_ODD_REGION"] == pg.PG_ODD_REGION
    flags = [consts[k] for k in consts if k.startswith("PG_") and k in (
        "PG_PTR_DEVICE", "PG_NO_PREPROCESS", "PG_OFFSETS_I32",
        "PG_CAREFUL_WALKS", "PG_COUNT_VALUATION", "PG_NO_GRAPH",
        "PG_HOST_REDUCED_LIST", "PG_SWITCH_ROWS", "PG_SWITCH_BUCKETS",
        "PG_KEEP_DUMMIES", "PG_ODD_REGION")]
    assert len(set(flags)) == len(flags) == 11
    off = np.array([0, 1, 2], np.int64)
    tgt = np.array([1, 0], np.int32)
    own = np.array([1, 1], np.uint8)
    pri = np.array([0, 1], np.int32)
    h = ctypes.c_void_p()
    L = pg.lib()
    rc = L.pg_load_csr(2, 2, pg._ptr(off), pg._ptr(tgt), pg._ptr(own),
                       pg._ptr(pri), pg.PG_ODD_REGION | pg.PG_NO_PREPROCESS,
                       None, ctypes.byref(h))
    assert rc == pg.PG_EINVAL
    assert b"PG_ODD_REGION" in L.pg_last_error()
