"""The Python binding's ctypes mirrors of the public structs have the size and
field offsets that the C compiler gives the declarations in include/cutqc.h
(a host compile of a small program that prints them; no GPU)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2205_05836_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["cq_subcircuit", "cq_dd_instance", "cq_dd_params", "cq_dd_record", "cq_dd_bfs_params",
           "cq_dd_bfs_node", "cq_gate", "cq_cut_problem"]


def _c_layout(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    lines = ['#include <cstdio>', '#include <cstddef>', '#include "cutqc.h"', "int main() {"]
    for name in STRUCTS:
        cls = getattr(_lib, name)
        lines.append(f'  std::printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  std::printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cxx, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True,
                   capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        key, val = line.rsplit(" ", 1)
        got[key] = int(val)
    return got


def test_ctypes_mirrors_match_c_layout(tmp_path):
    c = _c_layout(tmp_path)
    for name in STRUCTS:
        cls = getattr(_lib, name)
        assert C.sizeof(cls) == c[f"{name} size"], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == c[f"{name}.{field}"], f"{name}.{field}"
