"""C-ABI checks that need no GPU: the built library loads and exports every
function that include/*.h declares, and the binding covers them."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+[\s\*]+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_headers_declare_functions():
    names = declared_functions()
    assert "sgtv_iterate" in names and "sgtv_set_system" in names and "sgtv_objective" in names


def test_library_exports_every_declared_symbol():
    from paper_1601_08201_amd.build import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    from paper_1601_08201_amd import sgtv
    missing = [n for n in declared_functions() if n.startswith("sgtv_") and not hasattr(sgtv, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1601_08201_amd import sgtv
    monkeypatch.setattr(sgtv, "_lib", None)
    monkeypatch.setattr(sgtv, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        sgtv.lib()


def test_workspace_query_runs_on_the_host():
    from paper_1601_08201_amd import sgtv
    small = sgtv.sgtv_workspace_bytes(4096, 8192, 131072, "f32")
    big = sgtv.sgtv_workspace_bytes(1 << 20, 1 << 21, 1 << 27, "f32")
    half = sgtv.sgtv_workspace_bytes(1 << 20, 1 << 21, 1 << 27, "bf16")
    assert 0 < small < big and half < big
    # the two tiled copies of A dominate the paper-scale scan: about 2 x 1.08 x nnz x 7 bytes
    assert 1.9e9 < big < 2.6e9
    assert sgtv.sgtv_workspace_bytes(-1, 1, 1, "f32") == -1
    assert sgtv.sgtv_workspace_bytes(1, 1, 1, 7) == -1
