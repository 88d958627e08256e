"""The key under which bench.py keeps measured HBM traffic: a hash of the force
kernel's sources with comments and whitespace runs removed, so that a comment
edit keeps a recorded counter valid and any code edit drops it."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench_for_tests", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)

SRC = '''// header comment
#include "x.h"
/* block
   comment */ int f(int a) {   // trailing
    const char *s = "http://not-a-comment /* nor this */";
    return a + '/';
}
'''


def test_comments_and_whitespace_are_dropped():
    out = bench.code_only(SRC)
    assert "header comment" not in out and "block" not in out and "trailing" not in out
    assert '"http://not-a-comment /* nor this */"' in out
    assert "'/'" in out
    assert out == bench.code_only(out)


def test_comment_edit_keeps_the_hash_code_edit_changes_it(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "k.hip").write_text(SRC)
    h0 = bench.source_hash(["k.hip"])
    (tmp_path / "k.hip").write_text(SRC.replace("// trailing", "// another note").replace("block", "other"))
    assert bench.source_hash(["k.hip"]) == h0
    (tmp_path / "k.hip").write_text(SRC.replace("a + '/'", "a - '/'"))
    assert bench.source_hash(["k.hip"]) != h0


def test_force_sources_exist_and_hash():
    h = bench.source_hash(bench.FORCE_SOURCES)
    assert len(h) == 16 and int(h, 16) >= 0
