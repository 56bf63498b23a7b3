"""The C-ABI library loads and exports every symbol include/emogi.h declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "emogi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(emogi_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("emogi_graph_create", "emogi_graph_destroy", "emogi_bfs", "emogi_sssp",
                 "emogi_cc", "emogi_last_stats", "emogi_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2006_06890_amd import emogi
    if not os.path.exists(emogi.LIB_PATH):
        pytest.fail("libemogi.so not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(emogi.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_without_gpu():
    from paper_2006_06890_amd import emogi
    L = emogi.lib()
    assert L.emogi_strerror(0) == b"ok"
    assert L.emogi_strerror(-6) == b"distance overflow"
    assert L.emogi_strerror(-8) == b"unsupported"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2006_06890_amd import emogi
    monkeypatch.setattr(emogi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(emogi, "_lib", None)
    with pytest.raises(ImportError):
        emogi.lib()
