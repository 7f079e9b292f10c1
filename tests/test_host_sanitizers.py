"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle's C code and the library's graph-store builder, each compiled
with the sanitizers into a small checking program and run.  GPU code is not
involved."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(tmp_path, compiler, sources, extra, name):
    if not shutil.which(compiler):
        pytest.skip(f"{compiler} not available")
    exe = str(tmp_path / name)
    cmd = [compiler] + SAN + extra + sources + ["-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    return run.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", [os.path.join(HERE, "oracle_check.c"),
                                           os.path.join(ROOT, "oracle", "rrr_oracle.c")],
                         ["-std=c11"], "oracle_check")
    assert "ok" in out


def test_graph_builder_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2311_10201_amd", "csrc")
    out = _build_and_run(tmp_path, "g++", [os.path.join(HERE, "graph_check.cpp"), os.path.join(csrc, "bpt_graph.cpp")],
                         ["-std=c++17", f"-I{csrc}", f"-I{os.path.join(ROOT, 'include')}"], "graph_check")
    assert "ok" in out
