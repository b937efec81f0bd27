"""The C ABI without a GPU: the header compiles as C and C++, the library loads and
exports every function the header declares, argument checks answer without
touching a device."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pxcl.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(pxcl_\w+)\s*\(", src))
    names.discard("pxcl_done_cb")
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2004_04334_amd import build, pxcl
    if not os.path.exists(pxcl.LIB_PATH):
        build.build(force=True)
    return pxcl.lib()


def test_header_compiles_as_c_and_cxx(tmp_path):
    for lang, std in (("c", "-std=c99"), ("c++", "-std=c++17")):
        src = tmp_path / ("t.c" if lang == "c" else "t.cpp")
        src.write_text('#include "pxcl.h"\nint main(void){ pxcl_config c; c.n_modules = 1; (void)c; return 0; }\n')
        cc = "gcc" if lang == "c" else "g++"
        subprocess.check_call([cc, std, "-Wall", "-Werror", "-fsyntax-only", f"-I{os.path.dirname(HEADER)}", str(src)])


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_no_device_argument_checks(lib):
    from paper_2004_04334_amd import pxcl as px
    assert px.strerror(px.E_DUP_PIXEL) == "pixel fired twice in a module"
    assert lib.pxcl_version().startswith(b"pxcl")
    assert lib.pxcl_event_workspace_bytes(None, 100) == 0
    assert lib.pxcl_batch_workspace_bytes(None, 4) == 0
    assert lib.pxcl_acquire(None, None, None, None, None) == px.E_INVAL
    assert lib.pxcl_produce(None, None) == px.E_INVAL
    assert lib.pxcl_query(None) == px.E_INVAL
    assert lib.pxcl_ctx_destroy(None) == px.E_INVAL
    assert lib.pxcl_acquire_batch(None, None, None, 0, None, None, None, 0) == px.E_INVAL
    cfg = px._Config(0, 2000)
    h = ctypes.c_void_p()
    assert lib.pxcl_ctx_create(ctypes.byref(cfg), 0, ctypes.byref(h)) == px.E_INVAL   # n_modules = 0
    cfg = px._Config(40000, 2000)
    assert lib.pxcl_ctx_create(ctypes.byref(cfg), 0, ctypes.byref(h)) == px.E_INVAL   # ids would overflow


def test_flag_callback_is_host_only(lib):
    from paper_2004_04334_amd import pxcl as px
    f = px.Flag()
    lib.pxcl_flag_cb(ctypes.addressof(f), -6)
    lib.pxcl_flag_cb(ctypes.addressof(f), 0)
    assert f.fired == 2 and f.status == 0


def test_max_modules_keeps_ids_in_int32():
    # the largest id is PXCL_MAX_MODULES*66560 - 1
    src = open(HEADER).read()
    m = int(re.search(r"#define PXCL_MAX_MODULES (\d+)u", src).group(1))
    assert m * 66560 - 1 <= 2**31 - 1 < (m + 1) * 66560 - 1


def test_oracle_and_library_share_nothing():
    """The oracle is a separate C file with its own definitions; neither includes or
    imports the other."""
    osrc = open(os.path.join(ROOT, "oracle", "ccl_oracle.c")).read()
    assert "pxcl.h" not in osrc and "pxcl_internal" not in osrc
    for f in sorted(x for x in os.listdir(os.path.join(ROOT, "paper_2004_04334_amd", "csrc"))
                    if x.endswith((".hip", ".h", ".cpp"))):
        txt = open(os.path.join(ROOT, "paper_2004_04334_amd", "csrc", f)).read()
        assert "oracle" not in txt.lower(), f
    for f in ("pxcl.py", "build.py", "synth.py", "__init__.py"):
        txt = open(os.path.join(ROOT, "paper_2004_04334_amd", f)).read()
        assert "import oracle" not in txt and "from oracle" not in txt, f
