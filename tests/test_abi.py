"""The C-ABI library loads (no GPU needed) and exports every function that
include/sad.h declares; the header and the Python binding agree on the names."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sad.h")
LIB = os.path.join(ROOT, "paper_0901_2742_amd", "libsad.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sad_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for f in ("sad_kmer_rank", "sad_partition", "sad_align_buckets", "sad_refine"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsad.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_names_match_header():
    import ast
    src = open(os.path.join(ROOT, "paper_0901_2742_amd", "binding.py")).read()
    tree = ast.parse(src)
    exports = None
    for node in tree.body:
        if isinstance(node, ast.Assign) and getattr(node.targets[0], "id", "") == "EXPORTS":
            exports = ast.literal_eval(node.value)
    assert sorted(exports) == declared_functions()


def test_product_path_does_not_touch_the_oracle():
    """The package and the HIP sources never import, link or name the oracle."""
    pkg = os.path.join(ROOT, "paper_0901_2742_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "sad_oracle" not in text and "sadref_" not in text, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsad.so not built")
def test_host_only_workspace_queries():
    """The rank and partition workspace queries are host arithmetic (no device
    call): exact sizes of 256-byte aligned buffers plus 256 bytes of slack,
    and the same input checks as the calls."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_0901_2742_amd import binding as B

    def up(x):
        return (max(x, 1) + 255) // 256 * 256

    L = B.lib()
    n, total, p = 2000, 646_000, 16
    seqs = B.SadSeqs(n, 20, 1, 1, total, 600)   # device pointers are never read
    prm = B.SadParams(3, p, 1024, 1, 10, 1, 1)
    got = ctypes.c_size_t(0)
    assert L.sad_kmer_rank_workspace(ctypes.byref(seqs), ctypes.byref(prm),
                                     ctypes.byref(got)) == B.SAD_OK
    assert got.value == up(4 * total) + up(4 * n) + up(8 * n) + up(4 * n) + 256
    assert L.sad_partition_workspace(ctypes.byref(seqs), ctypes.byref(prm),
                                     ctypes.byref(got)) == B.SAD_OK
    ny, nblk = p * (p - 1), (n + 255) // 256
    part = up(4 * n) + 2 * up(8 * ny) + 2 * up(4 * ny) + up(4 * nblk * p) + up(4 * p)
    assert got.value == up(part) + 256
    bad = B.SadParams(3, 1001, 1024, 1, 10, 1, 1)   # N < 2p
    assert L.sad_partition_workspace(ctypes.byref(seqs), ctypes.byref(bad),
                                     ctypes.byref(got)) == B.SAD_E_INVAL
    short = B.SadSeqs(n, 20, 1, 1, total, 2)        # sequences shorter than k
    assert L.sad_kmer_rank_workspace(ctypes.byref(short), ctypes.byref(prm),
                                     ctypes.byref(got)) == B.SAD_E_INVAL
