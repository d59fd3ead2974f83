"""Host-side checks of bench.py's bookkeeping (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_hash_ignores_comments_only(tmp_path):
    a = tmp_path / "a.h"
    b = tmp_path / "b.h"
    c = tmp_path / "c.h"
    a.write_text("int f(int x) {\n  return x + 1;  // one more\n}\n")
    b.write_text("/* header */\nint f(int x)   {\n  // different comment\n  return x + 1;\n}\n")
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.sources_sha1([str(a)]) == bench.sources_sha1([str(b)])
    assert bench.sources_sha1([str(a)]) != bench.sources_sha1([str(c)])


def test_work_per_query_table():
    # 8 FP64 operations per candidate distance, 17 per box test
    assert abs(bench.ops_per_query(16) - (8 * 92.0 + 17 * 49.21)) < 1e-9
    assert bench.ops_per_query(17) is None
    for leaf, (cand, box) in bench.WORK_PER_QUERY.items():
        assert cand > 0 and box > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
