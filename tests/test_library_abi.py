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
    return sorted(set(re.findall(r"\b(kfbi3?_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_symbols()
    for must in ("kfbi_ctx_create", "kfbi_prob_create", "kfbi_apply", "kfbi_solve", "kfbi_correct",
                 "kfbi_fast_solve", "kfbi_interface_solve", "kfbi3_prob_create", "kfbi3_apply", "kfbi3_solve"):
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


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the C layout of kfbi_desc, kfbi_tiles, kfbi_desc3 and kfbi_gs_desc."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        import pytest
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "kfbi.h"\n'
        "#define F(T, m) printf(#T \" \" #m \" %zu\\n\", offsetof(T, m))\n"
        "int main(void) {\n"
        '  printf("kfbi_desc size %zu\\n", sizeof(kfbi_desc));\n'
        "  F(kfbi_desc, lo); F(kfbi_desc, hi); F(kfbi_desc, n); F(kfbi_desc, kappa); F(kfbi_desc, m);\n"
        "  F(kfbi_desc, xy); F(kfbi_desc, tol); F(kfbi_desc, restart); F(kfbi_desc, max_iter);\n"
        "  F(kfbi_desc, precision); F(kfbi_desc, refine_steps);\n"
        '  printf("kfbi_tiles size %zu\\n", sizeof(kfbi_tiles));\n'
        "  F(kfbi_tiles, modes_per_group); F(kfbi_tiles, modes_groups); F(kfbi_tiles, dst_cols);\n"
        "  F(kfbi_tiles, apply_us); F(kfbi_tiles, grid_solve_us);\n"
        '  printf("kfbi_desc3 size %zu\\n", sizeof(kfbi_desc3));\n'
        "  F(kfbi_desc3, n); F(kfbi_desc3, lo); F(kfbi_desc3, hi); F(kfbi_desc3, kappa); F(kfbi_desc3, axes);\n"
        "  F(kfbi_desc3, tol); F(kfbi_desc3, restart); F(kfbi_desc3, max_iter);\n"
        '  printf("kfbi_gs_desc size %zu\\n", sizeof(kfbi_gs_desc));\n'
        "  F(kfbi_gs_desc, lo); F(kfbi_gs_desc, hi); F(kfbi_gs_desc, n); F(kfbi_gs_desc, m); F(kfbi_gs_desc, xy);\n"
        "  F(kfbi_gs_desc, gamma); F(kfbi_gs_desc, kill); F(kfbi_gs_desc, eps0); F(kfbi_gs_desc, eps1);\n"
        "  F(kfbi_gs_desc, eps2); F(kfbi_gs_desc, dt); F(kfbi_gs_desc, tol); F(kfbi_gs_desc, restart);\n"
        "  F(kfbi_gs_desc, max_iter);\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    _lib_path()
    from paper_2404_15249_amd import kfbi
    structs = {"kfbi_desc": kfbi._Desc, "kfbi_tiles": kfbi.Tiles, "kfbi_desc3": kfbi._Desc3,
               "kfbi_gs_desc": kfbi._GsDesc}
    for line in filter(None, lines):
        name, field, value = line.split()
        st = structs[name]
        if field == "size":
            assert ctypes.sizeof(st) == int(value), line
        else:
            assert getattr(st, field).offset == int(value), line


def test_build_flags_register_spills():
    """The build's spill check reads the compiler's resource-usage remarks."""
    from paper_2404_15249_amd.build import spilling_kernels
    text = ("a.hip:1:1: remark: Function Name: k_one [-Rpass]\n"
            "a.hip:1:1: remark:     VGPRs Spill: 0 [-Rpass]\n"
            "a.hip:9:1: remark: Function Name: k_two [-Rpass]\n"
            "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 48 [-Rpass]\n"
            "a.hip:9:1: remark:     VGPRs Spill: 10 [-Rpass]\n")
    assert spilling_kernels(text) == [("k_two", "ScratchSize", 48), ("k_two", "VGPRs Spill", 10)]


def test_build_rejects_spills_and_scratch():
    """The build's check of the compiler's resource remarks: a VGPR spill or any
    nonzero scratch size fails it; clean kernels pass."""
    from paper_2404_15249_amd import build
    clean = ("x.hip:1:1: remark: Function Name: k_a\nx.hip:1:1: remark:     VGPRs Spill: 0\n"
             "x.hip:1:1: remark:     ScratchSize [bytes/lane]: 0\n")
    stack = ("x.hip:1:1: remark: Function Name: k_b\nx.hip:1:1: remark:     VGPRs Spill: 0\n"
             "x.hip:1:1: remark:     ScratchSize [bytes/lane]: 24\n")
    spill = ("x.hip:1:1: remark: Function Name: k_c\nx.hip:1:1: remark:     VGPRs Spill: 3\n"
             "x.hip:1:1: remark:     ScratchSize [bytes/lane]: 12\n")
    assert build.spilling_kernels(clean) == []
    assert build.spilling_kernels(stack) == [("k_b", "ScratchSize", 24)]
    assert [k[:2] for k in build.spilling_kernels(clean + spill)] == [("k_c", "VGPRs Spill"), ("k_c", "ScratchSize")]
