"""The C header and the ctypes binding describe the same structures: a C99
program compiled against include/aux.h (with -pedantic, so the header stays
plain C) prints the size of each ABI struct and the offset of every field,
and they must equal the ctypes layouts the binding passes across the ABI."""
import ctypes
import os
import subprocess

import pytest

import paper_1204_2586_amd as aux

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "aux_mesh": aux._Mesh,
    "aux_options": aux._Options,
    "aux_device": aux._Device,
    "aux_info": aux._Info,
    "aux_solve_info": aux._SolveInfo,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    d = tmp_path_factory.mktemp("hdr")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "aux.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["    return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        name, key, value = line.split()
        layout[(name, key)] = int(value)
    return layout


@pytest.mark.parametrize("cname", list(STRUCTS))
def test_struct_layout_matches_binding(c_layout, cname):
    py = STRUCTS[cname]
    assert c_layout[(cname, "size")] == ctypes.sizeof(py)
    for field, _ in py._fields_:
        assert c_layout[(cname, field)] == getattr(py, field).offset, field
