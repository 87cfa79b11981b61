"""The C-ABI library loads without a GPU and exports every entry point that
include/fire.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fire.h")
LIB = os.path.join(ROOT, "paper_1701_03549_amd", "libfiregpu.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fire_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("fire_ctx_create", "fire_run", "fire_run_dev", "fire_thresholds",
                 "fire_landscape_load", "fire_target_load", "fire_ga_step", "fire_ga_run",
                 "fire_ensemble", "fire_scan_reduce", "fire_sync", "fire_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (python -m paper_1701_03549_amd.build)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.fire_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.fire_version()


def test_binding_covers_header():
    from paper_1701_03549_amd import fire
    assert sorted(fire.EXPORTS) == declared_functions()


def test_null_context_is_rejected_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.fire_sync.restype = ctypes.c_int
    lib.fire_sync.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.fire_sync(None, None) == -1
    lib.fire_ctx_create.argtypes = [ctypes.c_int, ctypes.c_void_p]
    lib.fire_ctx_create.restype = ctypes.c_int
    assert lib.fire_ctx_create(0, None) == -1


def test_nn_library_exports():
    from paper_1701_03549_amd import nn
    text = open(os.path.join(ROOT, "include", "fire_nn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = sorted(set(re.findall(r"\b(fire_[a-z_0-9]+)\s*\(", text)))
    assert sorted(nn.EXPORTS) == declared
    lib = ctypes.CDLL(LIB)
    assert all(hasattr(lib, n) for n in declared)


def test_probe_library_exports():
    from paper_1701_03549_amd import probe
    text = open(os.path.join(ROOT, "include", "fire_probe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = sorted(set(re.findall(r"\b(fire_[a-z_0-9]+)\s*\(", text)))
    assert sorted(probe.EXPORTS) == declared
    lib = ctypes.CDLL(LIB)
    assert all(hasattr(lib, n) for n in declared)


def test_library_has_no_undefined_internal_symbols():
    """Every symbol of the library's own namespaces is defined in it."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-C", "--undefined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    bad = [l for l in out.splitlines() if "firegpu::" in l or "firenn::" in l]
    assert not bad, bad
