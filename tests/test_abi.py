"""The C-ABI library loads and exports every function declared in include/dmx.h
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dmx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dmx_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dmx_model_create", "dmx_rollout", "dmx_rollout_vjp", "dmx_tape_destroy", "dmx_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2506_14186_amd", "libdmx.so")
    assert os.path.exists(lib_path), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_opts_without_gpu():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2506_14186_amd", "libdmx.so"))
    buf = (ctypes.c_char * 512)()
    lib.dmx_default_opts(buf)
    rtol = ctypes.c_double.from_buffer(buf, 0).value
    assert rtol == 1e-6
