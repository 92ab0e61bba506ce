"""The banded fold's per-cell supports (paper_1812_05686_amd/csrc/gs_support.h), compiled for
the host: conservative against a brute-force scan of every bin, at most a few bins wider than
needed, and the arithmetic bin search for uniform binnings equal to the binary search."""
import json
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cell_supports(tmp_path):
    exe = tmp_path / "support_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1812_05686_amd", "csrc"),
                           os.path.join(ROOT, "tests", "support_check.cpp"), "-o", str(exe)])
    r = json.loads(subprocess.check_output([str(exe)], timeout=600).decode())
    assert r["cells"] > 10000, r
    assert r["missed"] == 0, r
    assert r["empty_bad"] == 0, r
    assert r["idx_mismatch"] == 0, r
    assert r["max_extra"] <= 3, r
