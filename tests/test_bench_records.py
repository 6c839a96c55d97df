"""Host logic of bench.py's measurement records (no GPU): the source digest
that keys the committed HBM counter records ignores comments and spacing but
not code, every record in profiles/traffic.json names a summary that exists
and a source group bench.py knows, and the multi-GPU request is refused."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_only_drops_comments_and_space_keeps_literals():
    code = 'int a = 1; // one\n/* two\n   lines */ const char* s = "x // y /* z */";\nint  b;'
    assert bench._code_only(code) == 'int a = 1; const char* s = "x // y /* z */"; int b;'
    assert bench._code_only("a = '\\'';  // c") == "a = '\\'';"
    assert bench._code_only("x/ y / z") == "x/ y / z"


def test_digest_follows_code_not_comments(tmp_path, monkeypatch):
    pkg = tmp_path / "paper_2112_03229_amd" / "csrc"
    pkg.mkdir(parents=True)
    (tmp_path / "include").mkdir()
    files = {"csrc/k.hip": "__global__ void k(int* p) { p[0] = 1; }  // store\n",
             "../include/h.h": "#define N 8 /* entries */\n"}
    for name, text in files.items():
        path = os.path.normpath(os.path.join(tmp_path, "paper_2112_03229_amd", name))
        with open(path, "w") as f:
            f.write(text)
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    monkeypatch.setitem(bench.KERNEL_SOURCES, "t", tuple(files))
    d0 = bench.kernel_source_digest("t")
    with open(pkg / "k.hip", "w") as f:
        f.write("// a new comment\n__global__ void k(int* p) {\n  p[0] = 1;\n}\n")
    assert bench.kernel_source_digest("t") == d0
    with open(pkg / "k.hip", "w") as f:
        f.write("__global__ void k(int* p) { p[0] = 2; }\n")
    assert bench.kernel_source_digest("t") != d0


def test_traffic_records_are_well_formed():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    assert rec
    for key, ent in rec.items():
        assert ent["sources"] in bench.KERNEL_SOURCES, key
        assert os.path.isfile(os.path.join(ROOT, ent["summary"])), key
        # each figure is rounded to whole bytes on its own
        assert abs(ent["bytes_per_launch"] - ent["fetch_bytes"] - ent["write_bytes"]) <= 1, key
        # counters within a few percent of the algorithmic bytes
        assert 0.99 <= ent["bytes_per_launch"] / ent["algorithmic_bytes"] <= 1.1, key


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
