"""The benchmark's command line on the host: it measures one GPU and says so
for any other count, before touching a device; the operator source hash
ignores comments, so edits to comments keep stored counters valid."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) { return x + 1; }  // one\n/* block */\n")
    b.write_text("// another comment\nint f(int x)   {\n  return x + 1;\n}\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    hashes = []
    for path in (a, b, c):
        monkeypatch.setattr(bench, "SRC", [str(path)])
        hashes.append(bench.source_hash())
    assert hashes[0] == hashes[1] != hashes[2]
