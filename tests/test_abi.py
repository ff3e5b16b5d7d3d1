"""The C-ABI library loads on any host and exports every function the
header declares (no compute call: that needs a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svf.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(svf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("svf_create", "svf_insert", "svf_delete", "svf_search", "svf_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2601_08528_amd as svf
    if not os.path.exists(svf.LIB_PATH):
        pytest.fail("libsvf.so missing: run python -m paper_2601_08528_amd.build")
    out = subprocess.run(["nm", "-D", "--defined-only", svf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (svf_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    L = svf.lib()
    for n in declared():
        assert hasattr(L, n)
    assert sorted(svf.EXPORTED) == declared()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2601_08528_amd as svf
    monkeypatch.setattr(svf, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(svf, "_lib", None)
    with pytest.raises(ImportError):
        svf.lib()
