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


def test_build_bytes_follow_the_compulsory_traffic():
    # 3D: 112 B per point (24 read, 8 key, 20 sort pass, 48 gather, 8 keys,
    # 4 id map) + 64 B per node; 2D: 88 B per point + 48 B per node
    assert bench.build_bytes(10, 3) == 10 * 112 + 3 * 64
    assert bench.build_bytes(10, 3, dim=2) == 10 * 88 + 3 * 48
    assert 24 + 8 + 20 + 48 + 8 + 4 == 112


def test_cpu_baseline_threads_match_serial():
    import numpy as np
    import workloads as W
    P = W.uniform(20000, 3, 0)
    _, qids, (ids, d2), cb = bench.cpu_baseline(P, 2000, 16)
    assert cb["threaded_rows_equal_serial"]
    assert cb["cores"] >= 1 and cb["nproc"] >= 1 and cb["cpu_model"]
    assert len(qids) == 2000 and ids.shape == (2000, 10)
