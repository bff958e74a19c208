"""The C-ABI library loads and exports every entry point that include/rwr.h
declares (no GPU needed: nothing here launches device work)."""

import ctypes
import os
import re

import pytest

import paper_1712_00595_amd as pkg
from paper_1712_00595_amd import rwr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rwr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rwr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_list():
    assert _declared() == sorted(rwr.EXPORTED)


def test_every_declared_symbol_is_exported():
    L = pkg.load_library()
    for name in _declared():
        assert hasattr(L, name), name


def test_struct_layouts_match_header(tmp_path):
    # every field's offset and every struct's size, as a C compiler lays out
    # rwr.h, equals the binding's ctypes mirror
    import subprocess

    structs = {"rwr_config": rwr.Config, "rwr_batch": rwr.BatchStruct, "rwr_stats": rwr.StatsStruct}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rwr.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c11", f"-I{inc}", str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_config_default_and_host_side_rejection():
    L = pkg.load_library()
    cfg = rwr.Config()
    assert L.rwr_config_default(ctypes.byref(cfg)) == 0
    assert cfg.c == 0.15 and cfg.eps == 1e-9 and cfg.precision == 0 and cfg.max_iters == 10000
    assert cfg.reorder == 1 and cfg.autotune == 1
    out = ctypes.c_void_p(None)
    # invalid arguments are rejected before any device call
    seeds = (ctypes.c_int32 * 1)(0)
    assert L.rwr_build(ctypes.byref(cfg), 0, 0, None, None, 1, seeds, 0, ctypes.byref(out)) == -1
    assert L.rwr_build(ctypes.byref(cfg), 10, 0, None, None, 0, seeds, 0, ctypes.byref(out)) == -1
    bad = (ctypes.c_int32 * 1)(11)
    assert L.rwr_build(ctypes.byref(cfg), 10, 0, None, None, 1, bad, 0, ctypes.byref(out)) == -1
    assert b"seed" in L.rwr_last_error(None)
    cfg.c = 1.5
    assert L.rwr_build(ctypes.byref(cfg), 10, 0, None, None, 1, seeds, 0, ctypes.byref(out)) == -1
    assert L.rwr_update(None, None, None) == -1
    L.rwr_destroy(None)


def test_checkpoint_and_hook_rejection_on_the_host(tmp_path):
    """rwr_load refuses a file that is not a checkpoint, and builds refuse an
    allocator hook given without its partner, before any device call."""
    L = pkg.load_library()
    out = ctypes.c_void_p(None)
    assert L.rwr_load(str(tmp_path / "absent.ckpt").encode(), None, ctypes.byref(out)) == -9
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"RWRCKPT0" + bytes(4096))
    assert L.rwr_load(str(junk).encode(), None, ctypes.byref(out)) == -9
    assert b"not a checkpoint" in L.rwr_last_error(None)
    short = tmp_path / "short.ckpt"
    short.write_bytes(b"RWRCKPT1")
    assert L.rwr_load(str(short).encode(), None, ctypes.byref(out)) == -9
    assert not out.value
    assert L.rwr_save(None, b"x") == -1
    cfg = rwr.Config()
    L.rwr_config_default(ctypes.byref(cfg))
    keep = rwr.ALLOC_FN(lambda n, s, u: None)
    cfg.dev_alloc = ctypes.cast(keep, ctypes.c_void_p)
    seeds = (ctypes.c_int32 * 1)(0)
    src = (ctypes.c_int32 * 1)(0)
    assert L.rwr_build(ctypes.byref(cfg), 4, 1, src, src, 1, seeds, 0, ctypes.byref(out)) == -1
    assert b"together" in L.rwr_last_error(None)
    assert L.rwr_load(str(junk).encode(), ctypes.byref(cfg), ctypes.byref(out)) == -1


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        rwr.load_library.__wrapped__ if hasattr(rwr.load_library, "__wrapped__") else None
        saved = rwr._lib
        rwr._lib = None
        try:
            rwr.load_library(str(tmp_path / "absent.so"))
        finally:
            rwr._lib = saved
