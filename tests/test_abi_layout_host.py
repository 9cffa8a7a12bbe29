"""CPU: every struct of the C ABI (include/argcsr.h) has, in the ctypes
binding, the same size and the same offset for every field as the C compiler
gives it -- the binding passes these structs by pointer, so a field added on
one side only would shift every field after it."""
import os
import shutil
import subprocess

import pytest

from paper_1203_5737_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")

# ctypes names that differ from the C field names (Python keywords)
C_NAME = {"in_": "in"}

PAIRS = [("argcsr_group_info", _lib.GroupInfo), ("argcsr_matrix", _lib.MatrixDesc),
         ("argcsr_tune_result", _lib.TuneResult), ("argcsr_server_config", _lib.ServerConfig),
         ("argcsr_request", _lib.Request), ("argcsr_result", _lib.Result),
         ("argcsr_server_stats", _lib.ServerStats)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_structs_match_the_header(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "argcsr.h"', "int main(void) {"]
    for cname, py in PAIRS:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {C_NAME.get(field, field)}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", INCLUDE, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, py in PAIRS:
        assert got[(cname, "sizeof")] == ctypes_sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


def ctypes_sizeof(t):
    import ctypes
    return ctypes.sizeof(t)
