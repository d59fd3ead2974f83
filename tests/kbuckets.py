"""The k buckets of the query kernels, read from the kernel source: one
kernel instantiation per (dimension, bucket, all-points | external)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def k_buckets():
    src = open(os.path.join(ROOT, "paper_2111_04182_amd", "csrc", "zd_knn_impl.h")).read()
    m = re.search(r"#define ZD_FOR_EACH_K\(X\)((?:\s*X\(\d+\))+)", src)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def k_max():
    src = open(os.path.join(ROOT, "include", "zd.h")).read()
    return int(re.search(r"#define ZD_KMAX (\d+)", src).group(1))


def bucket_cases():
    """(k, bucket) pairs: every bucket's top and top - 1 (so its padding
    slots are exercised), once each."""
    out = []
    for b in k_buckets():
        for k in sorted({b, max(1, b - 1)}):
            out.append((k, b))
    return out
