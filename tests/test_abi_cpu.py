"""CPU-only checks of the C ABI: the library loads and exports every declared entry point."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdmi.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2105_04150_amd import _binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libpdmi.so is not built (run __graft_entry__.build())")
    return B.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name


def test_binding_wraps_every_symbol():
    from paper_2105_04150_amd import _binding as B
    assert sorted(B.SYMBOLS) == _declared()
    for name in B.SYMBOLS:
        if name != "pd_last_error":
            assert callable(getattr(B, name)), name


def test_null_arguments_rejected_without_gpu(lib):
    # argument validation runs before any HIP call
    assert lib.pd_create(None, 0, 0, None) == -1
    assert b"NULL" in lib.pd_last_error(None)
    h = C.c_void_p()
    assert lib.pd_create(C.byref(h), 0, 7, None) == -1          # unknown precision
    assert lib.pd_step(None, 1) == -1
    assert lib.pd_sync(None) == -1
    assert lib.pd_destroy(None) == 0


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES", None) is None and
                    not os.path.exists("/dev/kfd"), reason="checks the no-device error path")
def test_create_without_device_fails_cleanly(lib):
    h = C.c_void_p()
    rc = lib.pd_create(C.byref(h), 0, 0, None)
    assert rc in (0, -1, -3)


def test_header_is_c99_and_links(tmp_path, lib):
    """A C99 translation unit that takes the address of every declared entry point
    compiles with -Wall -Werror and links against the library (nothing is called)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_2105_04150_amd import _binding as B
    names = _declared()
    src = tmp_path / "abi.c"
    src.write_text("#include \"pdmi.h\"\n#include <stdio.h>\n"
                   "int main(void) {\n  const void *f[] = {\n" +
                   "".join(f"    (const void *)&{n},\n" for n in names) +
                   "  };\n  printf(\"%d\\n\", (int)(sizeof f / sizeof f[0]));\n  return 0;\n}\n")
    exe = tmp_path / "abi"
    libdir = os.path.dirname(B.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-Wno-pedantic", "-I",
                        os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L", libdir, "-lpdmi",
                        f"-Wl,-rpath,{libdir}", "-Wl,--allow-shlib-undefined"],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
