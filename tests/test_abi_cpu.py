"""The C-ABI library loads on a machine without a GPU and exports every entry
point its header declares; argument validation needs no device."""
import ctypes
import os
import re

import pytest

from paper_2604_12256_amd import qsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "qsim355.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = qsim.load_library()
    names = declared_functions()
    assert "sim_create" in names and "sim_run" in names and "sim_probabilities" in names
    for name in names:
        assert hasattr(lib, name), name


def test_version_string():
    assert qsim.load_library().sim_version().decode().startswith("qsim355")


def test_create_validates_arguments_without_device():
    lib = qsim.load_library()
    ctx = ctypes.c_void_p()
    o = qsim.SimOptions()
    # NULL state buffer
    assert lib.sim_create(10, 0, ctypes.byref(o), ctypes.byref(ctx)) == qsim.E_INVAL
    # buffer too small (any non-NULL pointer value: never dereferenced)
    o.dev_state = 4096
    o.dev_state_bytes = 16 * 1023
    assert lib.sim_create(10, 0, ctypes.byref(o), ctypes.byref(ctx)) == qsim.E_NOMEM
    o.dev_state_bytes = 16 * 1024
    assert lib.sim_create(0, 0, ctypes.byref(o), ctypes.byref(ctx)) == qsim.E_INVAL
    assert lib.sim_create(37, 0, ctypes.byref(o), ctypes.byref(ctx)) == qsim.E_INVAL
    assert lib.sim_create(35, 1, ctypes.byref(o), ctypes.byref(ctx)) == qsim.E_NOMEM  # 256 GiB needed
    assert lib.sim_create(10, 7, ctypes.byref(o), ctypes.byref(ctx)) == qsim.E_INVAL
    # stage chunks: 10..13 qubits in complex128, 11..14 in complex64
    for dtype, C in ((0, 9), (0, 14), (1, 10), (1, 15)):
        o.C = C
        assert lib.sim_create(10, dtype, ctypes.byref(o), ctypes.byref(ctx)) == qsim.E_INVAL, (dtype, C)
    o.C = 0
    assert lib.sim_run(None) == qsim.E_INVAL
    assert lib.sim_destroy(None) == qsim.E_INVAL
    assert lib.sim_last_error(None) == b"null context"
