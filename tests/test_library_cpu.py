"""CPU-side checks of the C-ABI library: it loads and exports every function its header declares,
and the binding's ctypes structures have the header's sizes and field offsets."""
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


# the binding's ctypes structures against the C header: size and the offset of every field,
# as the host C compiler lays the header's structs out
_STRUCTS = {
    "MeshDesc": "hpdg_mesh_desc", "DiscParams": "hpdg_disc_params", "MeshInfo": "hpdg_mesh_info",
    "SmootherParams": "hpdg_smoother_params", "SolveParams": "hpdg_solve_params",
    "SolveStats": "hpdg_solve_stats", "RhsDesc": "hpdg_rhs_desc", "ServerParams": "hpdg_server_params",
    "Request": "hpdg_request", "RequestStatus": "hpdg_request_status",
    "NonlinearDesc": "hpdg_nonlinear_desc", "NewtonParams": "hpdg_newton_params",
    "NewtonStats": "hpdg_newton_stats",
}


def test_binding_structs_match_the_header(tmp_path):
    import ctypes
    import shutil
    import subprocess

    import paper_1907_01572_amd as hp

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hpdg.h"', "int main(void) {"]
    for py, c in _STRUCTS.items():
        cls = getattr(hp, py)
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (py, c))
        for name, _ in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (py, name, c, name))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for py in _STRUCTS:
        cls = getattr(hp, py)
        assert got[(py, "size")] == ctypes.sizeof(cls), py
        for name, _ in cls._fields_:
            assert got[(py, name)] == getattr(cls, name).offset, (py, name)
