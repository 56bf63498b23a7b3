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


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes mirror in the binding has the C struct's size and each
    field's offset (compiled from include/emogi.h with the host C compiler)."""
    import shutil
    import subprocess
    from paper_2006_06890_amd import emogi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = [("emogi_stats_t", emogi.Stats), ("emogi_link_profile_t", emogi.LinkProfile),
             ("emogi_batch_params_t", emogi.BatchParams), ("emogi_batch_trial_t", emogi.BatchTrial),
             ("emogi_train_config_t", emogi.TrainConfig)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "emogi.h"', "int main(void) {"]
    expect = []
    for cname, py in pairs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(py))
        for name, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {name}));')
            expect.append(getattr(py, name).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect
