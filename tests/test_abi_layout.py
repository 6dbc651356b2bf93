"""The ctypes mirrors of the ABI's structures have the C layout: a small C
program built with the host compiler from include/mgrhd.h prints sizeof and
the offset of every field the binding declares (a field the header lacks
fails to compile)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2407_18304_amd import mgrhd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {"mgrhd_options": mgrhd.Options, "mgrhd_opacity_params": mgrhd.OpacityParams,
           "mgrhd_patch": mgrhd.Patch}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a host C compiler")
def test_binding_structures_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mgrhd.h"',
             "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, cls in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)
