"""The C-ABI library: it loads without a GPU, exports every function that
include/wos.h declares, the binding's signatures cover exactly that set,
and the struct layouts of the binding match the header's sizes.  No compute
call is made (there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wos.h")
LIB = os.path.join(ROOT, "paper_2608_07017_amd", "libwos.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(wos_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("wos_toolbox_create", "wos_toolbox_build", "wos_build_toolbox", "wos_apply", "wos_solve",
                 "wos_toolbox_export", "wos_toolbox_free", "wos_last_error"):
        assert must in names


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        pytest.fail("libwos.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(so):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for name in _declared():
        assert name in exported, name
        assert getattr(so, name) is not None


def test_binding_signatures_match_header():
    from paper_2608_07017_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared()


def test_version_and_error_calls_need_no_device(so):
    so.wos_version.restype = ctypes.c_char_p
    so.wos_last_error.restype = ctypes.c_char_p
    assert so.wos_version().decode().startswith("libwos")
    assert isinstance(so.wos_last_error(), bytes)


def test_null_arguments_are_rejected_before_any_device_call(so):
    # validation happens on the host, before the runtime is touched
    from paper_2608_07017_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    st = L.wos_toolbox_create(None, None, 0, None, 0, None, ctypes.byref(h))
    assert st == -1
    assert L.wos_last_error().decode()


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2608_07017_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_libwos.so"))
    with pytest.raises(ImportError):
        _lib.lib()


_STRUCTS = ["wos_domain", "wos_build_opts", "wos_build_plan", "wos_toolbox_info", "wos_coeffs", "wos_solve_info",
            "wos_adam_opts", "wos_adam_info", "wos_hisd_opts", "wos_hisd_info", "wos_operator_opts",
            "wos_operator_info", "wos_server_opts"]


def _ctypes_struct(name):
    from paper_2608_07017_amd import _lib
    cname = "Wos" + "".join(w.capitalize() for w in name.split("_")[1:])
    return getattr(_lib, cname)


def test_struct_layouts_match_the_header(tmp_path):
    # sizeof and every field offset, from the C compiler on the header and
    # from the binding's ctypes structures
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "wos.h"', "int main(void) {"]
    for name in _STRUCTS:
        st = _ctypes_struct(name)
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in st._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            name, field, val = ln.split()
            got[(name, field)] = int(val)
    for name in _STRUCTS:
        st = _ctypes_struct(name)
        assert got[(name, "size")] == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert got[(name, f)] == getattr(st, f).offset, (name, f)


def test_load_rejects_files_that_are_not_toolboxes(tmp_path):
    # the header is checked before any device call
    from paper_2608_07017_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    bad = tmp_path / "bad.wostbx"
    bad.write_bytes(b"not a toolbox at all")
    assert L.wos_toolbox_load(str(bad).encode(), None, ctypes.byref(h)) == -1
    assert b"not a saved toolbox" in L.wos_last_error()
    old = tmp_path / "old.wostbx"
    old.write_bytes(b"WOSTBOX1" + (99).to_bytes(4, "little"))
    assert L.wos_toolbox_load(str(old).encode(), None, ctypes.byref(h)) == -1
    assert b"version" in L.wos_last_error()
    trunc = tmp_path / "trunc.wostbx"
    trunc.write_bytes(b"WOSTBOX1" + (1).to_bytes(4, "little") + (1).to_bytes(4, "little") + (8).to_bytes(8, "little"))
    assert L.wos_toolbox_load(str(trunc).encode(), None, ctypes.byref(h)) == -1
    assert L.wos_toolbox_load(str(tmp_path / "missing").encode(), None, ctypes.byref(h)) == -1
    assert not h.value
