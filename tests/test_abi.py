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


def header_enums():
    """Every BCA_* enumerator of include/bca.h with its value."""
    src = open(os.path.join(ROOT, "include", "bca.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    vals = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", src, flags=re.S):
        for name, val in re.findall(r"\b(BCA_\w+)\s*=\s*(-?\d+)", body):
            vals[name] = int(val)
    return vals


def test_binding_constants_match_header_enums():
    from paper_2405_16267_amd import bca as b
    h = header_enums()
    assert h["BCA_OK"] == b.BCA_OK
    for code, name in b.ERRORS.items():
        assert h[name] == code, name
    for name, v in b.LOSS.items():
        assert h["BCA_LOSS_" + name.upper()] == v
    for name, v in b.DTYPE.items():
        assert h["BCA_" + name.upper()] == v
    assert (h["BCA_MEM_HOST"], h["BCA_MEM_DEVICE"]) == (b.MEM_HOST, b.MEM_DEVICE)
    assert (h["BCA_FLAG_EXACT_X"], h["BCA_FLAG_WOODBURY"]) == (b.FLAG_EXACT_X, b.FLAG_WOODBURY)
    for name in ("X", "U", "Z", "S", "OMEGA", "NU", "TV"):
        assert h["BCA_VEC_" + name] == getattr(bca, "VEC_" + name), name
    for name in ("STREAM", "SOLVE", "GLOBAL", "GRAM", "FACTOR"):
        assert h["BCA_KC_" + name] == getattr(bca, "KC_" + name), name
    for name in ("QUEUED", "RUNNING", "DONE", "FAILED", "CANCELLED"):
        assert h["BCA_REQ_" + name] == getattr(b, "REQ_" + name), name


def test_create_rejects_rows_wider_than_the_streaming_pass():
    """One-class problems stream every row through one workgroup of at most 1,024
    threads x 8 chunks of 16 bytes; wider rows are refused at create (argument
    validation runs before any device call, so no GPU is needed)."""
    import ctypes
    from paper_2405_16267_amd import bca as b
    for dtype, nmax in (("f64", 16384), ("f32", 32768), ("bf16", 65536)):
        rows = (ctypes.c_int64 * 1)(10)
        p = b.Params(loss=0, n_features=nmax + 1, n_classes=1, n_partitions=1, n_blocks=64, kappa=5,
                     rows=rows, gamma=10.0, rho_c=1.0, rho_b=0.5, rho_l=1.0, inner_iters=5,
                     max_iters=10, tol_p=1e-6, tol_d=1e-6, tol_b=1e-6, a_dtype=b.DTYPE[dtype],
                     check_every=10, flags=0)
        h = ctypes.c_void_p()
        rc = b.lib().bca_create(ctypes.byref(p), ctypes.c_void_p(None), ctypes.byref(h))
        assert rc == -1 and not h.value, (dtype, rc)
        assert b"widest streaming row" in b.lib().bca_last_error()
