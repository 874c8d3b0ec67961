"""The C-ABI library loads on the CPU host and exports every declared entry point."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfcc.h")
LIB = os.path.join(ROOT, "paper_2010_04768_amd", "libgfcc.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gfcc_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_boundary():
    names = declared_functions()
    for f in ["gfcc_build_intermediates", "gfcc_sigma", "gfcc_solve_batch", "gfcc_greens", "gfcc_destroy",
              "gfcc_strerror"]:
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgfcc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgfcc.so not built")
def test_binding_declares_same_symbols():
    from paper_2010_04768_amd import gfcc
    assert sorted(gfcc.SYMBOLS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgfcc.so not built")
def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.gfcc_strerror.restype = ctypes.c_char_p
    assert lib.gfcc_strerror(0) == b"success"
    assert lib.gfcc_strerror(-1) == b"invalid argument"


@pytest.mark.parametrize("lang,std", [("c", "-std=c99"), ("c++", "-std=c++17")])
def test_header_is_plain_c_and_cpp(tmp_path, lang, std):
    """The boundary header compiles on its own as C99 (no C++ in the ABI) and as C++."""
    import shutil
    import subprocess
    cc = shutil.which("gcc" if lang == "c" else "g++")
    if cc is None:
        pytest.skip("no host compiler")
    src = tmp_path / "use_header.c"
    src.write_text('#include "gfcc.h"\nint main(void) { gfcc_solve_opts o; gfcc_shift_opts s; '
                   'gfcc_mor_opts m; (void)o; (void)s; (void)m; return 0; }\n')
    r = subprocess.run([cc, std, "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", "-x", lang,
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
