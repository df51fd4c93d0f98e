"""Host-side checks of the C ABI: the library loads, exports every function
that include/knnjoin.h declares, and its binding signatures match the header.
No compute calls (no GPU needed)."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "knnjoin.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(knn_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_boundary():
    names = _declared()
    for must in ["knn_build_index", "knn_build_index_device", "knn_self_join",
                 "knn_self_join_device", "knn_destroy_index", "knn_last_error",
                 "knn_server_create", "knn_server_submit", "knn_server_wait",
                 "knn_server_stats_get", "knn_server_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1810_04758_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libknnjoin.so not built")
    L = _lib.load()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert missing == []
    # every declared function has a binding signature, and vice versa
    assert sorted(_lib.SIGNATURES) == _declared()


def test_last_error_is_empty_string_initially():
    from paper_1810_04758_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libknnjoin.so not built")
    assert _lib.load().knn_last_error() in (b"",)


def test_struct_sizes_match_header():
    # compile a tiny C program against the header and compare sizeof with ctypes
    import ctypes
    import subprocess
    import tempfile
    from paper_1810_04758_amd import _lib
    prog = r'''
#include <stdio.h>
#include "knnjoin.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(knn_build_opts),
         sizeof(knn_join_opts), sizeof(knn_join_stats), sizeof(knn_index_info),
         sizeof(knn_server_opts), sizeof(knn_server_stats), sizeof(knn_autotune_result),
         sizeof(knn_eps_join_stats), sizeof(knn_hybrid_opts), sizeof(knn_hybrid_stats));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    assert sizes == [ctypes.sizeof(t) for t in (_lib.BuildOpts, _lib.JoinOpts, _lib.JoinStats,
                                                _lib.IndexInfo, _lib.ServerOpts,
                                                _lib.ServerStats, _lib.AutotuneResult,
                                                _lib.EpsJoinStats, _lib.HybridOpts,
                                                _lib.HybridStats)]
