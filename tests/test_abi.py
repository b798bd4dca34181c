"""The C-ABI library builds, loads and exports every entry point its header
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssort.h")
LIB = os.path.join(ROOT, "paper_1403_2056_amd", "libssort.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ssort_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_1403_2056_amd import build
        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for must in ("ssort_create", "ssort_sort", "ssort_sort_batched", "ssort_workspace_bytes",
                 "ssort_query_error", "ssort_destroy", "ssort_debug_step", "ssort_merge",
                 "ssort_merge_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol(built):
    out = subprocess.check_output(["nm", "-D", "--defined-only", built], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(built)
    for n in declared():
        getattr(L, n)


def test_binding_signatures_cover_header(built):
    from paper_1403_2056_amd import ssort
    names = set(declared())
    covered = set(ssort._SIGS)
    assert names <= covered, sorted(names - covered)
    L = ssort.lib()
    assert L.ssort_strerror(0) == b"ok"
    assert L.ssort_strerror(3) == b"workspace too small"


def test_no_torch_types_in_header():
    src = open(HEADER).read()
    code = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    for bad in ("torch", "Tensor", "at::", "c10", "#include <hip"):
        assert bad not in code
    assert 'extern "C"' in code
