"""The ctypes structures of the binding have the sizes and field offsets the
C compiler gives the structures of include/tn.h (host only: a small C
program compiled with the system compiler prints them)."""

import ctypes as C
import re
import shutil
import subprocess
from pathlib import Path

import pytest

from paper_2104_10523_amd import _native

ROOT = Path(__file__).resolve().parent.parent

STRUCTS = {
    "tn_op": _native.TnOp,
    "tn_circuit": _native.TnCircuit,
    "tn_network_info": _native.TnNetworkInfo,
    "tn_path_opts": _native.TnPathOpts,
    "tn_path_cost": _native.TnPathCost,
    "tn_tensor": _native.TnTensor,
    "tn_report": _native.TnReport,
    "tn_exec_opts": _native.TnExecOpts,
    "tn_plan_info": _native.TnPlanInfo,
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_ctypes_structures_match_the_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tn.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", str(ROOT / "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, timeout=120)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True, timeout=60).stdout.splitlines())
    want = {}
    for cname, py in STRUCTS.items():
        want[f"{cname} size"] = str(C.sizeof(py))
        for f in py._fields_:
            want[f"{cname} {f[0]}"] = str(getattr(py, f[0]).offset)
    assert got == want


def test_every_header_structure_is_checked():
    text = (ROOT / "include" / "tn.h").read_text()
    declared = set(re.findall(r"^\}\s*(tn_\w+);", text, flags=re.M))
    assert declared == set(STRUCTS)
