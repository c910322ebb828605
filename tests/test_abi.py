"""The C-ABI library loads and exports every symbol that include/fcirc.h declares (CPU only:
no compute calls), and the host-side validation paths that need no device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcirc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(fcirc_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("fcirc_create", "fcirc_destroy", "fcirc_matvec", "fcirc_polymul_i64", "fcirc_bigint_mul",
                 "fcirc_matvec_batched", "fcirc_matvec_fwd_shared", "fcirc_matvec_backward", "fcirc_check"):
        assert want in names


@pytest.fixture(scope="module")
def lib():
    from paper_2103_02605_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2103_02605_amd.build import build
        build()
    return _lib.lib()


def test_library_exports_every_declared_symbol(lib):
    from paper_2103_02605_amd import _lib
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_strerror(lib):
    for code in range(9):
        assert b"unknown" not in lib.fcirc_strerror(code), code
    assert b"unknown" in lib.fcirc_strerror(99)


def test_null_context_is_einval(lib):
    f = C.c_uint32(1)
    assert lib.fcirc_matvec(None, None, None, None, 8, C.byref(f), 0, None) == 1
    assert lib.fcirc_matvec_noalloc(None, None, None, None, 8, C.byref(f), 0, None) == 1
    assert lib.fcirc_check(None, None) == 1
    assert lib.fcirc_polymul_i64(None, None, 1, None, 1, None, None) == 1
    assert lib.fcirc_set_split(None, 0) == 1


def test_create_without_gpu_reports_edevice(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert lib.fcirc_create(C.byref(h), 0) == 6


def test_header_is_plain_c_and_links():
    """include/fcirc.h is a C header (no C++ or HIP types): a C99 translation unit that
    includes it and takes the address of every declared entry point compiles, and links
    against libfcirc.so (no GPU needed: nothing is called)."""
    import shutil
    import subprocess
    import tempfile
    from paper_2103_02605_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2103_02605_amd.build import build
        build()
    names = declared_functions()
    src = "#include <stdio.h>\n#include \"fcirc.h\"\ntypedef void (*fn)(void);\nint main(void) {\n  fn p[] = {\n"
    src += ",\n".join(f"    (fn)&{n}" for n in names)
    src += "\n  };\n  printf(\"%d\\n\", (int)(sizeof p / sizeof p[0]));\n  return 0;\n}\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "abi.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "abi")
        libdir = os.path.dirname(_lib.LIB_PATH)
        r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"), c,
                            "-o", exe, "-L", libdir, "-lfcirc", f"-Wl,-rpath,{libdir}", "-Wl,--unresolved-symbols=ignore-in-shared-libs"],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
