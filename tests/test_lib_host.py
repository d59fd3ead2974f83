"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/zd.h declares, and rejects bad arguments before it
touches the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "zd.h")).read()
    return re.findall(r"^ZD_API\s+[\w\s\*]+?\b(zd_\w+)\s*\(", src, flags=re.M)


@pytest.fixture(scope="module")
def L():
    pytest.importorskip("torch")
    import paper_2111_04182_amd as zd
    return zd.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("zd_build", "zd_knn", "zd_insert_batch", "zd_delete_batch", "zd_free"):
        assert n in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_symbol(L):
    import paper_2111_04182_amd._lib as B
    for n in declared_functions():
        assert hasattr(L, n), n
    # the binding wraps exactly the declared calls
    assert sorted(B.EXPORTED) == sorted(declared_functions())


def test_status_strings(L):
    for code in range(8):
        assert L.zd_status_str(code) and L.zd_status_str(code) != b"unknown status"
    assert L.zd_status_str(99) == b"unknown status"


def test_argument_errors_need_no_device(L):
    import paper_2111_04182_amd._lib as B
    vp = C.c_void_p
    out = vp()
    assert L.zd_build(None, None, 0, None, C.byref(out)) == B.ZD_EINVAL
    # n above 2^30 - 1: node links (node << 1) | side would overflow int32
    for dim, leaf, n in ((4, 16, 10), (1, 16, 10), (3, 0, 10), (3, 16, -1), (2, 16, 2**31),
                         (3, 16, 2**30), (2, 1, 2**30)):
        p = B._Params(dim, leaf, 0, None, None, None)
        assert L.zd_build(C.byref(p), vp(1), n, None, C.byref(out)) == B.ZD_EINVAL
    for w in (-1, 3, 5, 8):  # query_waves must be 0, 1, 2 or 4
        p = B._Params(3, 16, 0, None, None, None, w)
        assert L.zd_build(C.byref(p), vp(1), 10, None, C.byref(out)) == B.ZD_EINVAL
    p = B._Params(3, 16, 0, None, None, None)
    assert L.zd_build(C.byref(p), None, 0, None, C.byref(out)) == B.ZD_EINVAL  # n=0, no box
    assert L.zd_build(C.byref(p), None, 5, None, C.byref(out)) == B.ZD_EINVAL  # NULL coords
    assert L.zd_knn(None, None, 0, 1, None, None, None) == B.ZD_EINVAL
    assert L.zd_insert_batch(None, None, 1, None, None) == B.ZD_EINVAL
    assert L.zd_delete_batch(None, None, 1, None) == B.ZD_EINVAL
    assert L.zd_info(None, None, None, None, None, None) == B.ZD_EINVAL
    assert L.zd_check(None) == B.ZD_EINVAL
    assert L.zd_pending(None, None, None) == B.ZD_EINVAL
    assert L.zd_set_walk_limit(None, 0) == B.ZD_EINVAL
    assert L.zd_free(None) == B.ZD_OK
    assert L.zd_knn_backward(4, None, 0, 0, 1, None, None, None, None) == B.ZD_EINVAL
    for k, want in ((0, B.ZD_EINVAL), (B.ZD_KMAX + 1, B.ZD_EKMAX), (4, B.ZD_EINVAL)):
        assert L.zd_forest_plan_persistent(None, None, 0, None, 0, None, k, None, None, None,
                                           C.byref(out)) == want
    assert L.zd_knn_backward(3, None, 10, 20, 1, None, None, None, None) == B.ZD_EINVAL
    assert out.value is None


def test_params_layout_matches_the_header(tmp_path):
    """The binding's zd_params mirror has the C struct's size and offsets."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("needs gcc")
    import paper_2111_04182_amd._lib as B
    fields = [f[0] for f in B._Params._fields_]
    prog = tmp_path / "layout.c"
    prog.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"zd.h\"\nint main(void) {\n"
                    "  printf(\"%zu\\n\", sizeof(zd_params));\n"
                    + "".join(f"  printf(\"%zu\\n\", offsetof(zd_params, {f}));\n" for f in fields)
                    + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got[0] == C.sizeof(B._Params)
    assert got[1:] == [getattr(B._Params, f).offset for f in fields]


def test_k_buckets_cover_kmax():
    """The bucket list the GPU tests iterate over is the kernels' own, rising,
    and its top bucket is ZD_KMAX."""
    from tests.kbuckets import bucket_cases, k_buckets, k_max
    b = k_buckets()
    assert b == sorted(set(b)) and b[0] == 1 and b[-1] == k_max()
    import paper_2111_04182_amd._lib as B
    assert B.ZD_KMAX == k_max()
    assert len(bucket_cases()) == 2 * len(b) - 1
