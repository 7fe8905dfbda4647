"""The C ABI library loads on a machine without a GPU and exports every
function include/orbf.h declares; the Python binding declares the same
names.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "orbf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(orbf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("orbf_build_nodes_knn", "orbf_select_overlapped_stencils",
                 "orbf_compute_weights", "orbf_assemble_csr", "orbf_create",
                 "orbf_destroy", "orbf_sync", "orbf_last_error",
                 "orbf_workspace_size"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1606_03135_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("liborbf.so not built")
    L = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding marshals the same entry points
    for n in ("build_nodes_knn", "select_overlapped_stencils",
              "compute_weights", "assemble_csr"):
        assert callable(getattr(P, n))


def test_workspace_size_is_host_only():
    import paper_1606_03135_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("liborbf.so not built")
    a = P.workspace_size(10_000, 3, 50, 3)
    b = P.workspace_size(1_000_000, 3, 50, 3)
    assert 0 < a < b
