"""CPU checks of the C-ABI boundary: the built library loads and exports
every entry point that include/csi.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csi.h")
LIB = os.path.join(ROOT, "paper_2403_03440_amd", "libcsi.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csi_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("csi_set_grid", "csi_set_mechanism", "csi_residual", "csi_implicit_op",
                     "csi_consistency_correct", "csi_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcsi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcsi.so not built")
def test_binding_names_match_header():
    from paper_2403_03440_amd import csi
    assert sorted(csi.EXPORTED) == declared_functions()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2403_03440_amd import csi
    monkeypatch.setattr(csi, "_lib", None)
    monkeypatch.setattr(csi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        csi.load()
