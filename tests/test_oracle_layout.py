"""The oracle's ctypes parameter block against its C header: the same size
and every field at the same offset (a C program compiled against oracle/pfo.h
prints them)."""
import ctypes as ct
import os
import shutil
import subprocess

import pytest

from oracle import pfo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_params_layout_matches_the_header(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    names = [f for f, _ in pfo.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"pfo.h\"\nint main(void) {\n"
                   "  printf(\"%zu\\n\", sizeof(pfo_params));\n"
                   + "".join(f"  printf(\"%zu\\n\", offsetof(pfo_params, {n}));\n" for n in names)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "oracle"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == ct.sizeof(pfo.Params)
    assert out[1:] == [getattr(pfo.Params, n).offset for n in names]
