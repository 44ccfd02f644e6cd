"""The C-ABI library loads on a host without a GPU and exports every entry
point that include/rmhmc.h declares (no compute calls are made here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmhmc.h")
LIB = os.path.join(ROOT, "paper_2511_06407_amd", "librmhmc.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rmhmc_[a-z0-9_]+)\s*\(", text)))


def ensure_built():
    if not os.path.exists(LIB):
        from paper_2511_06407_amd.build import build
        build()


def test_header_declares_the_path():
    syms = declared_symbols()
    for name in ("rmhmc_hessian", "rmhmc_softabs_eig", "rmhmc_metric_grad", "rmhmc_glf_step",
                 "rmhmc_chain"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    ensure_built()
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_matches_header():
    ensure_built()
    from paper_2511_06407_amd import rmhmc
    assert sorted(rmhmc.EXPORTED) == declared_symbols()


def test_argument_errors_are_host_side():
    """Invalid descriptors fail on the host with RMHMC_E_ARG (no GPU needed)."""
    ensure_built()
    from paper_2511_06407_amd import rmhmc
    lib = rmhmc._lib
    h = ctypes.c_void_p()
    assert lib.rmhmc_model_create(None, 0, ctypes.byref(h)) == rmhmc.E_ARG
    assert b"NULL" in lib.rmhmc_last_error()
    desc = rmhmc.ModelDesc()
    desc.N = 1
    assert lib.rmhmc_model_create(ctypes.byref(desc), 0, ctypes.byref(h)) == rmhmc.E_ARG
    cfg = rmhmc.ChainCfg()
    assert lib.rmhmc_chain(None, ctypes.byref(cfg), None, None, None, None, None, None, None,
                           None) == rmhmc.E_ARG


def test_header_compiles_as_c():
    """include/rmhmc.h is a plain C header (no C++ or torch types)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        import pytest
        pytest.skip("no gcc")
    src = f'#include "{HEADER}"\nint main(void) {{ return 0; }}\n'
    r = subprocess.run(["gcc", "-std=c11", "-fsyntax-only", "-x", "c", "-I/opt/rocm/include",
                        "-D__HIP_PLATFORM_AMD__", "-"], input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
