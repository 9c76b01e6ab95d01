"""The ctypes binding's structures match the C header's, field by field:
a C program built here with gcc prints every struct's size and its fields'
offsets, and the binding's must equal them."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2407_19396_amd import gridenv as ge

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "gx_config": ge.GxConfig, "gx_state": ge.GxState, "gx_traj": ge.GxTraj,
    "gx_info": ge.GxInfo, "gx_request": ge.GxRequest, "gx_server_info": ge.GxServerInfo,
    "gx_serve_item": ge.GxServeItem, "gx_serve_opts": ge.GxServeOpts,
    "gx_serve_stats": ge.GxServeStats,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gridenv.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        name, key, value = line.split()
        table[(name, key)] = int(value)
    return table


@pytest.mark.parametrize("cname", list(STRUCTS))
def test_binding_structs_match_the_header(c_layout, cname):
    py = STRUCTS[cname]
    assert ctypes.sizeof(py) == c_layout[(cname, "size")], cname
    for field, _ in py._fields_:
        assert getattr(py, field).offset == c_layout[(cname, field)], (cname, field)
