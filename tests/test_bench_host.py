"""Host logic of bench.py: the key under which measured HBM traffic is reused ignores comments
and whitespace but not code."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_strip_c_comments_keeps_code_and_literals():
    src = 'a = "x // y";   // note\n\n\nb = \'/\'; /* block\n comment */ c = "\\" /* kept */";\n#define X 1\nint y;'
    assert bench.strip_c_comments(src) == 'a = "x // y";\nb = \'/\'; c = "\\" /* kept */";\n#define X 1\nint y;'


def test_comment_and_whitespace_edits_do_not_change_the_key():
    code = "int f(int x) {\n  return x + 1;\n}\n"
    edited = "// helper\nint f(int x) {  /* adds one */\n\n  return x + 1;   // the result\n}\n"
    changed = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench.strip_c_comments(code) == bench.strip_c_comments(edited)
    assert bench.strip_c_comments(code) != bench.strip_c_comments(changed)


def test_sources_key_is_a_sha256():
    h = bench.sources_sha256()
    assert len(h) == 64 and int(h, 16) >= 0
