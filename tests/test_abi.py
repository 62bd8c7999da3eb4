"""Host-side checks of the C ABI: the library loads and exports every function
include/ctm.h declares; argument validation that needs no device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctm.h")
LIB = os.path.join(ROOT, "paper_2506_19339_amd", "libctm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for fn in ("ctm_init", "ctm_iterate", "ctm_free_energy", "ctm_grad", "ctm_destroy"):
        assert fn in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libctm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for fn in declared_functions():
        assert hasattr(lib, fn), fn


@pytest.mark.skipif(not os.path.exists(LIB), reason="libctm.so not built")
def test_host_only_calls():
    from paper_2506_19339_amd import ctm
    lib = ctm.load_library()
    assert lib.ctm_abi_version() == 5
    assert lib.ctm_status_string(0) == b"ok"
    assert lib.ctm_status_string(4) == b"not converged"
    lib.ctm_destroy(None)                          # NULL-safe
    # argument validation happens before any device call
    cfg = ctm._Config(2, 16, 40, 0.0, 0, 0, 0, 0.0, 0.0, 0)
    out = ctypes.c_void_p()
    A = (ctypes.c_double * 32)()
    assert lib.ctm_init(ctypes.byref(cfg), -0.1, A, None, ctypes.byref(out)) == 1
    assert b"beta" in lib.ctm_last_error(None)
    bad = ctm._Config(0, 16, 40, 0.0, 0, 0, 0, 0.0, 0.0, 0)
    assert lib.ctm_init(ctypes.byref(bad), 0.2, A, None, ctypes.byref(out)) == 1
    assert lib.ctm_init(ctypes.byref(cfg), 0.2, None, None, ctypes.byref(out)) == 1
    bad = ctm._Config(2, 16, 40, 0.0, 3, 0, 0, 0.0, 0.0, 0)          # unknown precision
    assert lib.ctm_init(ctypes.byref(bad), 0.2, A, None, ctypes.byref(out)) == 1
    bad = ctm._Config(2, 16, 40, 0.0, 1, 0, 0, 0.0, -1.0, 0)         # negative lp_tol
    assert lib.ctm_init(ctypes.byref(bad), 0.2, A, None, ctypes.byref(out)) == 1
    assert not out.value


def test_config_struct_layout_matches_header(tmp_path):
    """The ctypes mirror of ctm_config has the C struct's size and offsets."""
    import subprocess
    from paper_2506_19339_amd import ctm
    src = tmp_path / "layout.c"
    fields = [f[0] for f in ctm._Config._fields_]
    body = "".join('printf("%%zu ", offsetof(ctm_config, %s));' % f for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ctm.h"\n'
                   'int main(void){%s printf("%%zu\\n", sizeof(ctm_config)); return 0;}\n' % body)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [getattr(ctm._Config, f).offset for f in fields] + [ctypes.sizeof(ctm._Config)]
    assert got == want


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2506_19339_amd import ctm
    with pytest.raises(OSError):
        ctm.load_library(str(tmp_path / "missing.so"))
