"""The binding's ctypes structures lay out exactly as include/ahf.h's structs:
a C program built against the header prints each struct's size and every
field's offset, and the binding's classes must agree, field by field (host
only, gcc)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_0904_3662_amd import ahf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("ahf_ctx_desc", ahf.CtxDesc), ("ahf_params", ahf.Params),
         ("ahf_particles", ahf.Particles), ("ahf_level_view", ahf.LevelView),
         ("ahf_structures", ahf.Structures), ("ahf_tuning", ahf.Tuning),
         ("ahf_build_info", ahf.BuildInfo), ("ahf_halo_params", ahf.HaloParams),
         ("ahf_halos_view", ahf.HalosView), ("ahf_server_desc", ahf.ServerDesc),
         ("ahf_server_stats", ahf.ServerStats)]


def c_layout(tmp_path):
    lines = ['#include <stdio.h>', '#include "ahf.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    return got


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_structures_match_the_header(tmp_path):
    got = c_layout(tmp_path)
    for cname, cls in PAIRS:
        assert C.sizeof(cls) == got[(cname, "size")], cname
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == got[(cname, fname)], (cname, fname)
