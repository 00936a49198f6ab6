"""The C-ABI library loads and exports every entry point include/tt_kernel.h
declares (no compute calls: runs without a GPU)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tt_kernel.h")
LIB = os.path.join(ROOT, "paper_2406_06344_amd", "libttk.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:tt_status|const char\*)\s+(tt_kernel_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        subprocess.run([sys.executable, os.path.join(ROOT, "paper_2406_06344_amd", "build.py")], check=True)
    return LIB


def test_header_declares_the_three_north_calls():
    names = declared()
    for n in ("tt_kernel_build_offline", "tt_kernel_online_core", "tt_kernel_apply"):
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (tt_kernel_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_matches(lib_path):
    from paper_2406_06344_amd import _lib
    lib = _lib.load()
    for n in declared():
        assert hasattr(lib, n)
    assert sorted(_lib.EXPORTS) == declared()


def test_param_struct_layout_matches_header():
    """The ctypes structs mirror the C structs field by field."""
    from paper_2406_06344_amd import _lib
    txt = open(HEADER).read()
    body = txt[txt.index("typedef struct {\n  int d;"):txt.index("} tt_kernel_params;")]
    names = re.findall(r"\b(\w+)(?:\[\d+\])?\s*;", body)
    assert names == [f[0] for f in _lib.Params._fields_]


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2406_06344_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()
