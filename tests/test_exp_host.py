"""The device exponential (paper_1812_05686_amd/csrc/gs_exp.h) compiled for the host and checked
against long-double expl: relative error below 1.7e-14 over the log-densities a banded fold keeps
([-60, 1]), within the stated bound 1.45e-14 + |n| 2.4e-17 over the normal range, underflow handled,
special values right (exp(0) within the polynomial's error of 1), and the unclamped variant equal
to it bit for bit on its domain [-1e9, 709]."""
import json
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exp_cw_accuracy(tmp_path):
    exe = tmp_path / "exp_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1812_05686_amd", "csrc"),
                           os.path.join(ROOT, "tests", "exp_check.cpp"), "-o", str(exe)])
    r = json.loads(subprocess.check_output([str(exe)]).decode())
    assert r["bad_special"] == 0, r
    assert r["unclamped_diff"] == 0, r
    assert r["max_rel_kept"] <= 1.7e-14, r
    assert r["max_bound_ratio"] <= 1.0, r
    assert r["max_rel"] <= 4.0e-14, r
    assert r["max_subnormal_ulps"] <= 1.0, r


def test_exp_tb_accuracy(tmp_path):
    """The table-driven exponential the pair loops use: relative error below 2e-14 over the
    kept log-densities, within 1.8e-14 + |n| 1.0e-19 over the normal range (n = round(256 x /
    ln2)), table entries within half an ulp, NaN read inside the table, and the unclamped
    variant equal to it bit for bit on [-1e6, 709]."""
    exe = tmp_path / "exp_tb_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1812_05686_amd", "csrc"),
                           os.path.join(ROOT, "tests", "exp_tb_check.cpp"), "-o", str(exe)])
    r = json.loads(subprocess.check_output([str(exe)]).decode())
    assert r["bad_special"] == 0, r
    assert r["unclamped_diff"] == 0, r
    assert r["max_rel_kept"] <= 2.0e-14, r
    assert r["max_bound_ratio"] <= 1.0, r
    assert r["max_rel"] <= 4.5e-14, r
    assert r["max_subnormal_ulps"] <= 1.0, r
    assert r["max_table_rel"] <= 1.12e-16, r
