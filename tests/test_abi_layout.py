"""The binding's ctypes structs match the C header's structs field by field.

A C program compiled with gcc against include/pbcgs.h prints every struct's
size and each field's offset; the ctypes mirrors in _lib.py must agree, or
options and reports would be read at the wrong offsets.
"""

import os
import shutil
import subprocess

import pytest

from paper_1612_01395_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = {
    "pbcgs_opts": _lib.Opts,
    "pbcgs_info": _lib.Info,
    "pbcgs_tune_report": _lib.TuneReport,
    "pbcgs_tune_entry": _lib.TuneEntry,
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_struct_layouts_match_the_header(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pbcgs.h"', "int main(void) {"]
    for cname, cls in PAIRS.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for cname, cls in PAIRS.items():
        assert int(got[cname]) == _lib.ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)
