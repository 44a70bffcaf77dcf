"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before touching a device (CPU only, no compute calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afqmc.h")


def _lib():
    from paper_1804_03310_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libafqmc.so is not built; run __graft_entry__.build()")
    return _abi, _abi.load()


def test_header_declarations_are_exported():
    _abi, lib = _lib()
    src = open(HEADER).read()
    declared = set(re.findall(r"\b(afqmc_[a-z_]+)\s*\(", src))
    assert declared == set(_abi.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def test_invalid_hamiltonian_arguments_rejected():
    _abi, lib = _lib()
    out = ctypes.c_void_p()
    M = 4
    h = np.eye(M)
    L = np.zeros((2, M, M))
    assert lib.afqmc_init_hamiltonian(None, 0, None, M, 2, h.ctypes.data, L.ctypes.data, 0.0) == -1
    assert lib.afqmc_init_hamiltonian(ctypes.byref(out), 0, None, 0, 2, h.ctypes.data, L.ctypes.data, 0.0) == -1
    assert lib.afqmc_init_hamiltonian(ctypes.byref(out), 0, None, M, -1, h.ctypes.data, L.ctypes.data, 0.0) == -1
    assert lib.afqmc_init_hamiltonian(ctypes.byref(out), 0, None, 300, 2, h.ctypes.data, L.ctypes.data, 0.0) == -1
    hn = h.copy()
    hn[0, 1] = 1.0
    assert lib.afqmc_init_hamiltonian(ctypes.byref(out), 0, None, M, 2, hn.ctypes.data, L.ctypes.data, 0.0) == -1
    assert b"symmetric" in lib.afqmc_last_error()
    Ln = L.copy()
    Ln[1, 2, 3] = 0.5
    assert lib.afqmc_init_hamiltonian(ctypes.byref(out), 0, None, M, 2, h.ctypes.data, Ln.ctypes.data, 0.0) == -1
    hnan = h.copy()
    hnan[2, 2] = np.nan
    assert lib.afqmc_init_hamiltonian(ctypes.byref(out), 0, None, M, 2, hnan.ctypes.data, L.ctypes.data, 0.0) == -1
    assert out.value is None


def test_null_objects_rejected():
    _abi, lib = _lib()
    b = ctypes.c_size_t()
    assert lib.afqmc_walker_workspace_bytes(None, 4, ctypes.byref(b)) == -1
    w = _abi.WalkersStruct()
    o = _abi.OptionsStruct(6, 0, 0, 0.0, 0, 0)
    assert lib.afqmc_propagate(None, None, ctypes.byref(w), 1, 0.01, 0, 0, ctypes.byref(o), None, None) == -1
    assert lib.afqmc_local_energy(None, None, ctypes.byref(w), None, None) == -1
    assert lib.afqmc_orthonormalize(None, None, ctypes.byref(w), None) == -1
    assert lib.afqmc_reconfigure(None, ctypes.byref(w), 0, 0, None, None) == -1
    assert lib.afqmc_fields(0, 0, 0, 4, 0, None, None) == -1
    out = ctypes.c_void_p()
    C = np.eye(4)
    assert lib.afqmc_init_trial(ctypes.byref(out), None, 2, 2, C.ctypes.data, C.ctypes.data, 1, None, None, 1) == -1
    lib.afqmc_free_hamiltonian(None)
    lib.afqmc_free_trial(None)


def test_struct_layouts_match_header():
    _abi, _ = _lib()
    # int32, int32, 8 pointers, size_t
    assert ctypes.sizeof(_abi.WalkersStruct) == 8 + 8 * 8 + 8
    # 3 x int32 (+4 pad), double, 2 x enum(int), 2 x int32
    assert ctypes.sizeof(_abi.OptionsStruct) == 40
    assert _abi.OptionsStruct.e_trial.offset == 16
    assert _abi.OptionsStruct.weight_mode.offset == 32


def test_package_fails_loudly_without_library(tmp_path):
    from paper_1804_03310_amd import _abi
    with pytest.raises(ImportError):
        saved = _abi._lib
        _abi._lib = None
        try:
            _abi.load(str(tmp_path / "missing.so"))
        finally:
            _abi._lib = saved


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the package before torch must not map a second HIP runtime
    (torch ships its own copy of libamdhip64 under the same soname; two copies
    in one process leave the library without a device)."""
    import subprocess
    import sys
    code = ("import paper_1804_03310_amd, torch, os\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = {os.path.realpath(l.split()[-1]) for l in maps if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1", r.stdout
