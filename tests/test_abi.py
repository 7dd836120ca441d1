"""The C-ABI library loads and exports every function declared in include/srp.h (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(srp_[a-z0-9_]+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("srp_scene_create", "srp_scene_set_design", "srp_trace", "srp_trace_records", "srp_frames",
              "srp_scene_destroy", "srp_sync", "srp_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2602_10712_amd", "libsrp.so")
    if not os.path.exists(lib_path):
        pytest.skip("libsrp.so not built")
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_last_error_callable_without_gpu():
    lib_path = os.path.join(ROOT, "paper_2602_10712_amd", "libsrp.so")
    if not os.path.exists(lib_path):
        pytest.skip("libsrp.so not built")
    lib = ctypes.CDLL(lib_path)
    lib.srp_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.srp_last_error(), bytes)
    # argument validation happens before any device call
    lib.srp_scene_create.restype = ctypes.c_int32
    out = ctypes.c_void_p()
    st = lib.srp_scene_create(None, ctypes.c_int64(0), None, ctypes.c_int64(0), None, None, 0, None,
                              ctypes.byref(out))
    assert st == -1
    assert b"empty" in lib.srp_last_error()


def test_every_exported_entry_point_is_declared():
    import shutil
    import subprocess
    lib_path = os.path.join(ROOT, "paper_2602_10712_amd", "libsrp.so")
    if not os.path.exists(lib_path) or not shutil.which("nm"):
        pytest.skip("libsrp.so not built or nm missing")
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.split() and ln.split()[-2] == "T"}
    exported = {n for n in exported if n.startswith("srp_")}
    undeclared = sorted(exported - declared_functions())
    assert not undeclared, undeclared


def test_ray_mask_bits_layout():
    """ray_mask_bits packs pixel p of direction j into bit p & 31 of word p >> 5 (host-side packing,
    checked on the CPU)."""
    lib_path = os.path.join(ROOT, "paper_2602_10712_amd", "libsrp.so")
    if not os.path.exists(lib_path):
        pytest.skip("libsrp.so not built")
    import numpy as np
    import paper_2602_10712_amd as p
    rng = np.random.default_rng(0)
    m = rng.random((3, 70)) < 0.3
    w = p.ray_mask_bits(m, device="cpu").numpy().view(np.uint32)
    assert w.shape == (3, 3)
    for j in range(3):
        for q in range(96):
            bit = (int(w[j, q >> 5]) >> (q & 31)) & 1
            assert bit == (int(m[j, q]) if q < 70 else 0)
