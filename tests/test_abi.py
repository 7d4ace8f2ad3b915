"""The C-ABI library loads on a machine without a GPU and exports every symbol
that ``include/*.h`` declares (no compute calls here)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_02621_amd", "libgoldbach.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(gb_[a-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2603_02621_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("gb_create", "gb_destroy", "gb_verify_range", "gb_verify_range_batched",
                 "gb_verify_one", "gb_verify_many", "gb_verify_windows", "gb_autotune",
                 "gb_status_str", "gb_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header(lib):
    from paper_2603_02621_amd import _binding
    assert set(_binding.SIGNATURES) == _declared()


def test_status_strings(lib):
    lib.gb_status_str.restype = ctypes.c_char_p
    assert lib.gb_status_str(0) == b"GB_OK"
    assert lib.gb_status_str(5) == b"GB_EUNRESOLVED"


def test_struct_layout_matches_the_c_compiler(tmp_path):
    """Every field offset of the ctypes mirrors equals what gcc computes
    from the header itself."""
    import subprocess
    from paper_2603_02621_amd import _binding as B
    structs = {"gb_params": B.Params, "gb_result": B.Result, "gb_window": B.Window,
               "gb_summary": B.Summary, "gb_request": B.Request, "gb_completion": B.Completion,
               "gb_server_stats": B.ServerStats, "gb_pc_result": B.PcResult,
               "gb_peaks": B.Peaks}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "goldbach.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_no_gpu_create_fails_cleanly(lib):
    # on this CPU-only machine gb_create must return an error, not crash
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = lib.gb_create(ctypes.byref(h), None)
    assert st != 0 and not h.value
