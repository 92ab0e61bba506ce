"""The tile-relative pair exponent of the 1-D fold and the adjoint (rel_cell, rel_offsets,
rel_exponent in paper_1812_05686_amd/csrc/gs_dev.h), compiled for the host and compared with
the exponent a cell record defines, evaluated in quadruple precision, on every pair that a
banded fold keeps (log-density above -60) for Borexino-scale and sharper responses.  Also the
property the pair loops' range check rests on: within a tile (or an adjoint block) the relative
exponent of a cell is lowest at one of the two end bins, up to rounding."""
import json
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_relative_exponent_error(tmp_path):
    exe = tmp_path / "relexp_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1812_05686_amd", "csrc"),
                           os.path.join(ROOT, "tests", "relexp_check.cpp"), "-o", str(exe), "-lquadmath"])
    r = json.loads(subprocess.check_output([str(exe)], timeout=600).decode())
    for fam in ("gamma", "gauss"):
        q = r[fam]
        assert q["pairs"] > 100000, r
        # the rounding bound u (|A u| + |B v| + |Eref| + |E|) holds up to a small factor
        assert q["max_ratio"] <= 4.0, r
        # relative error of every kept density: far inside the 1e-12 per-bin bound
        assert q["max_rel_density"] <= 1e-13, r
        assert q["max_err"] <= 1e-13, r
        # no interior bin of a tile below the lower end bin by more than its rounding
        assert q["tiles"] > 10000 and q["max_below_ends"] <= 4.0, r
