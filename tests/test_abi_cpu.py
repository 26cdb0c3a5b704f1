"""The C ABI library loads and exports every function that include/dsg.h
declares; calls fail cleanly without a GPU.  No device work here."""
import ctypes
import os
import re

import pytest

from paper_2202_08808_amd import dsg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dsg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dsg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["dsg_ctx_create", "dsg_mat_create", "dsg_mat_apply", "dsg_prod_create_static",
                 "dsg_prod_update", "dsg_prod_recompute_static", "dsg_prod_rows", "dsg_mat_export"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(dsg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert set(declared_functions()) <= set(dsg.SIGNATURES) | {"dsg_last_error"}


def test_null_arguments_are_rejected():
    L = dsg.lib()
    assert L.dsg_ctx_create(0, None, 0, None) == dsg.E_ARG
    assert L.dsg_ctx_destroy(None) == dsg.E_ARG
    assert L.dsg_mat_apply(None, None, None, None, None, 0, 0) == dsg.E_ARG
    assert L.dsg_prod_update(None, 0, None) == dsg.E_ARG
    assert L.dsg_last_error(None)


@pytest.mark.skipif(os.path.exists("/dev/kfd") and os.access("/dev/kfd", os.R_OK),
                    reason="a GPU is present")
def test_no_device_reports_device_error():
    L = dsg.lib()
    h = ctypes.c_void_p()
    assert L.dsg_ctx_create(0, None, 0, ctypes.byref(h)) == dsg.E_DEVICE
    assert b"device" in L.dsg_last_error(None)


# ctypes mirror of each struct the header declares
MIRRORS = {"dsg_rows": "Rows", "dsg_tuning": "Tuning", "dsg_update_stats": "Stats",
           "dsg_update_set": "UpdateSet", "dsg_batch_stats": "BatchStats", "dsg_server_cfg": "ServerCfg",
           "dsg_server_result": "ServerResult", "dsg_server_stats": "ServerStats", "dsg_allocator": "Allocator"}


def test_binding_structs_match_the_header(tmp_path):
    """Size and field offsets of every struct, as a C compiler lays them out
    from include/dsg.h, equal those of the binding's ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dsg.h"', "int main(void) {"]
    for cname, pname in MIRRORS.items():
        cls = getattr(dsg, pname)
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, pname in MIRRORS.items():
        cls = getattr(dsg, pname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, f"{cname}.{f}"
