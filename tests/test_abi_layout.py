"""The ctypes structures of the binding have the byte layout of include/pfmp.h
(offsets and sizes from a C program compiled against the header with gcc)."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "pfmp_solver_params": "SolverParams",
    "pfmp_solver_stats": "SolverStats",
    "pfmp_term": "Term",
    "pfmp_hmc_spec": "HmcSpec",
    "pfmp_traj_stats": "TrajStats",
    "pfmp_tuning": "Tuning",
}
# Python field names that differ from the header's (``lambda`` is a Python keyword)
RENAMED = {"lam": "lambda"}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    from paper_1609_02652_amd import pfmp
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pfmp.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in getattr(pfmp, pyname)._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, RENAMED.get(f, f)))
    lines.append("return 0; }")
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines))
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.parametrize("cname", sorted(STRUCTS))
def test_struct_layout_matches_header(c_layout, cname):
    from paper_1609_02652_amd import pfmp
    cls = getattr(pfmp, STRUCTS[cname])
    assert ctypes.sizeof(cls) == c_layout[(cname, "size")]
    for f, _ in cls._fields_:
        assert getattr(cls, f).offset == c_layout[(cname, f)], (cname, f)
