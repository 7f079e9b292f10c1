"""The C-ABI library loads, exports every symbol include/bpt.h declares, and its
host-side arithmetic and argument checks behave as declared.  No compute call
needs a GPU here."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_2311_10201_amd as bpt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bpt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bpt_[a-z0-9_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert declared_functions() == sorted(bpt.EXPORTED_SYMBOLS)


def test_counters_struct_matches_header():
    """The binding's bpt_counters mirrors the header's, field by field."""
    with open(HEADER) as f:
        text = f.read()
    body = re.search(r"typedef struct bpt_counters \{(.*?)\} bpt_counters;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"uint64_t\s+(\w+);", body)
    assert fields == [name for name, _ in bpt._Counters._fields_]
    assert ctypes.sizeof(bpt._Counters) == 8 * len(fields)


MIRRORED_STRUCTS = [("bpt_counters", bpt._Counters), ("bpt_job", bpt._Job), ("bpt_request", bpt._Request),
                    ("bpt_server_info", bpt._ServerInfo)]


def test_structs_match_header_layout(tmp_path):
    """Every struct the binding mirrors has the header's fields in the header's
    order, and each field sits at the offset and has the size that a C
    compiler gives it (gcc, compiling the header as plain C)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "bpt.h"', "int main(void) {"]
    for cname, cls in MIRRORED_STRUCTS:
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), text, re.S).group(1)
        assert re.findall(r"(\w+)\s*;", body) == [f for f, _ in cls._fields_], cname
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu %zu\\n", offsetof({cname}, {f}), sizeof((({cname}*)0)->{f}));')
    lines += ["return 0;", "}"]
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", f"-I{os.path.dirname(HEADER)}", str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    got = dict(line.split(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                              text=True).stdout.splitlines())
    for cname, cls in MIRRORED_STRUCTS:
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            desc = getattr(cls, f)
            assert got[f"{cname}.{f}"] == f"{desc.offset} {desc.size}", (cname, f)


def test_library_exports_every_declared_symbol():
    lib = bpt.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", bpt.library_path()], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in exported, name


def test_library_is_gfx950_code_object():
    blob = open(bpt.library_path(), "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_version():
    assert "gfx950" in bpt.bpt_version()


def test_threshold_matches_oracle():
    rng = np.random.Generator(np.random.PCG64(11))
    ps = np.concatenate([rng.random(20000, dtype=np.float32),
                         np.array([0.0, 1.0, 0.5, 0.1, 0.01, 2**-9, 2**-24, 2**-126, 2**-149,
                                   np.nextafter(np.float32(1), np.float32(0))], dtype=np.float32)])
    for p in ps.tolist():
        assert bpt.bpt_thr32(p) == oracle.thr32(p), p


def test_coin_and_start_match_oracle():
    rng = np.random.Generator(np.random.PCG64(12))
    for _ in range(3000):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        s = int(rng.integers(0, 2**34))
        e = int(rng.integers(0, 2**32))
        n = int(rng.integers(1, 2**32))
        assert bpt.bpt_coin_word(seed, s, e) == oracle.coin_word(seed, s, e)
        assert bpt.bpt_start_vertex(seed, s, n) == oracle.start_vertex(seed, s, n)


@pytest.mark.parametrize("case", ["dup", "range", "nan", "above1", "below0", "n0", "nullptr"])
def test_invalid_graphs_rejected_before_device(case):
    lib = bpt.load_library()
    s = np.array([0, 1], np.uint32)
    d = np.array([1, 2], np.uint32)
    p = np.array([0.5, 0.5], np.float32)
    n = 3
    if case == "dup":
        s, d = np.array([0, 0], np.uint32), np.array([1, 1], np.uint32)
    elif case == "range":
        d = np.array([1, 3], np.uint32)
    elif case == "nan":
        p = np.array([0.5, np.nan], np.float32)
    elif case == "above1":
        p = np.array([0.5, 1.0001], np.float32)
    elif case == "below0":
        p = np.array([-0.0001, 0.5], np.float32)
    elif case == "n0":
        n = 0
    if case == "nullptr":
        h = lib.bpt_create_graph(3, 2, None, None, None)
        assert not h
        assert lib.bpt_last_status() == bpt.BPT_EINVAL
        return
    with pytest.raises(bpt.BptError) as ei:
        bpt.bpt_create_graph(n, s, d, p)
    assert ei.value.status == bpt.BPT_EINVAL
    assert bpt.bpt_last_error()


def test_bad_handles_are_reported():
    lib = bpt.load_library()
    junk = (ctypes.c_uint32 * 16)(*([0x12345678] * 16))
    lib.bpt_free(ctypes.addressof(junk))
    assert lib.bpt_last_status() == bpt.BPT_EINVAL
    lib.bpt_free(None)
    assert lib.bpt_last_status() == bpt.BPT_OK
    assert lib.bpt_sample_rrr(None, 10, 64, 1) is None
    assert lib.bpt_last_status() == bpt.BPT_EINVAL
    assert lib.bpt_graph_info(None, None, None, None) == bpt.BPT_EINVAL
    total = ctypes.c_uint64(0)
    st = lib.bpt_sample_rrr_device(None, 0, 10, 64, 1, 0, None, None, None, 0, ctypes.byref(total), None)
    assert st == bpt.BPT_EINVAL
    assert lib.bpt_plan_create(None, 10, 64, 0) is None
    assert lib.bpt_last_status() == bpt.BPT_EINVAL
    st = lib.bpt_plan_enqueue(None, 0, 10, 1, None, None, None, None, 0, None)
    assert st == bpt.BPT_EINVAL
    st = lib.bpt_plan_enqueue(ctypes.addressof(junk), 0, 10, 1, None, None, None, None, 0, None)
    assert st == bpt.BPT_EINVAL
