"""The C-ABI library builds for gfx950, loads on the host, and exports every
entry point that include/kfbi.h declares (no device work: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_path():
    from paper_2404_15249_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "kfbi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kfbi_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_symbols()
    for must in ("kfbi_ctx_create", "kfbi_prob_create", "kfbi_apply", "kfbi_solve", "kfbi_correct",
                 "kfbi_fast_solve", "kfbi_interface_solve"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_the_header():
    _lib_path()
    from paper_2404_15249_amd import kfbi
    assert set(declared_symbols()) == set(kfbi.EXPORTED)


def test_status_strings():
    lib = ctypes.CDLL(_lib_path())
    lib.kfbi_status_str.restype = ctypes.c_char_p
    assert lib.kfbi_status_str(0) == b"ok"
    assert lib.kfbi_status_str(-2) == b"unsupported geometry"
