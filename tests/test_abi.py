"""The C ABI library loads and exports every symbol include/bca.h declares
(no compute: runs without a GPU)."""
import os
import re
import subprocess

import paper_2405_16267_amd as bca

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "bca.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bca_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(bca.EXPORTS)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", bca.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (bca_\w+)", out))
    missing = [f for f in header_functions() if f not in exported]
    assert not missing, missing


def test_library_is_gfx950_code():
    # the embedded device code object names its target
    data = open(bca.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_params_struct_layout_matches_header():
    import ctypes
    # loss..kappa (6 x int32), rows ptr, 4 doubles, 2 int32, 3 doubles, 2 int32 + uint32
    assert ctypes.sizeof(bca.Params) == 24 + 8 + 32 + 8 + 24 + 12 + 4


def test_last_error_is_empty_string_initially():
    assert isinstance(bca.lib().bca_last_error(), bytes)
