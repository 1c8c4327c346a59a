"""CPU-side checks of the C-ABI library: it loads and exports every function its header declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hpdg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpdg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_documented_calls():
    names = _declared()
    for must in ("hpdg_create", "hpdg_mesh_upload", "hpdg_apply", "hpdg_smooth", "hpdg_vcycle",
                 "hpdg_solve", "hpdg_setup_smoother", "hpdg_assemble_rhs"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1907_01572_amd as hp
    if not os.path.exists(hp.LIB_PATH):
        pytest.skip("library not built")
    lib = hp.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(hp.EXPORTED) == _declared()


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1907_01572_amd as hp
    saved = hp._lib
    hp._lib = None
    try:
        with pytest.raises(ImportError):
            hp.load_library(str(tmp_path / "missing.so"))
    finally:
        hp._lib = saved
