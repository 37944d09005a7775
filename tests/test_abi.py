"""The C-ABI library loads on the CPU and exports every entry point that
include/grmhd.h declares; host-side argument validation works without a GPU."""

import ast
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grmhd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(grmhd_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("grmhd_create", "grmhd_init_state", "grmhd_rhs", "grmhd_step", "grmhd_diagnostics"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2508_18221_amd import _lib
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_query_bytes_and_validation_on_host():
    from paper_2508_18221_amd import _lib, make_grid
    lib = _lib.load()
    res, scr = ctypes.c_size_t(), ctypes.c_size_t()
    g = make_grid(64, 64, 128)
    assert lib.grmhd_query_bytes(ctypes.byref(g), 0, ctypes.byref(res), ctypes.byref(scr)) == 0
    P = 64 * 64 * 128
    assert scr.value >= 241 * P * 8
    assert res.value >= 39 * P * 8
    bad = make_grid(16, 16, 15)
    assert lib.grmhd_query_bytes(ctypes.byref(bad), 0, ctypes.byref(res), ctypes.byref(scr)) == -1
    assert b"even" in lib.grmhd_last_error()
    small = make_grid(3, 16, 16)
    assert lib.grmhd_query_bytes(ctypes.byref(small), 0, ctypes.byref(res), ctypes.byref(scr)) == -1
    with pytest.raises(Exception):
        _lib.check(lib.grmhd_query_bytes(ctypes.byref(bad), 0, ctypes.byref(res), ctypes.byref(scr)))


def test_library_shares_torch_hip_runtime():
    """The library must bind to the HIP runtime that allocated the device
    memory and streams it is handed (PyTorch ships its own copy); a second
    runtime in the process sees no device."""
    import subprocess
    import sys
    code = ("from paper_2508_18221_amd import _lib; _lib.load(); "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True,
                         cwd=str(__import__("pathlib").Path(__file__).resolve().parents[1])).stdout
    libs = ast.literal_eval(out.strip().splitlines()[-1])
    assert len(libs) == 1, libs


def test_create_rejects_parameters_out_of_range_on_host():
    """grmhd_create checks its parameters before it touches the device, so
    the checks run here without a GPU (the buffer arguments are never used)."""
    from paper_2508_18221_amd import _lib, make_grid, make_phys
    lib = _lib.load()
    g = make_grid(16, 16, 16)
    ctx = ctypes.c_void_p()
    cases = [(dict(gamma_ad=1.0), b"Gamma"), (dict(M=1.0, a=1.2), b"|a|"), (dict(cfl=0.0), b"cfl"),
             (dict(rho_floor=0.0), b"floors"), (dict(p_floor=float("nan")), b"floors"),
             (dict(eta=float("inf")), b"eta"), (dict(split=True, cowling=True), b"split")]
    for over, msg in cases:
        p = make_phys(**over)
        rc = lib.grmhd_create(ctypes.byref(g), ctypes.byref(p), 0, ctypes.c_void_p(256), ctypes.c_void_p(512),
                              None, ctypes.byref(ctx))
        assert rc == -1 and msg in lib.grmhd_last_error(), (over, lib.grmhd_last_error())
    p = make_phys()
    p.glm, p.glm_ch = 1, 0.0
    rc = lib.grmhd_create(ctypes.byref(g), ctypes.byref(p), 0, ctypes.c_void_p(256), ctypes.c_void_p(512),
                          None, ctypes.byref(ctx))
    assert rc == -1 and b"GLM" in lib.grmhd_last_error()
    rc = lib.grmhd_create(ctypes.byref(g), ctypes.byref(p), 0, ctypes.c_void_p(300), ctypes.c_void_p(512),
                          None, ctypes.byref(ctx))
    assert rc == -1
