"""C ABI layout (CPU): every struct of include/gltrsv.h has the same size and
the same field offsets in C (compiled here with gcc) as in the ctypes
binding, and every constant the binding mirrors (error codes, schedule kinds,
triangles, packing modes, execution forms) has the header's value, so the
binding cannot drift from the header."""
import os
import shutil
import subprocess

import pytest

from paper_2503_05408_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {
    "gltrsv_csr": B.Csr,
    "gltrsv_plan_opts": B.PlanOpts,
    "gltrsv_plan_info": B.PlanInfo,
    "gltrsv_batch_opts": B.BatchOpts,
    "gltrsv_server_opts": B.ServerOpts,
    "gltrsv_server_stats": B.ServerStats,
}
# header macro -> the binding's value
CONSTANTS = {
    "GLTRSV_OK": B.GLTRSV_OK,
    **{"GLTRSV_" + name: code for code, name in B.ERRORS.items()},
    **{f"GLTRSV_{n}": getattr(B, n) for n in (
        "SCHED_GROWLOCAL", "SCHED_WAVEFRONT", "SCHED_AUTO", "SCHED_GIVEN", "LOWER", "UPPER",
        "PACK_AUTO", "PACK_HOST", "PACK_DEVICE", "EXEC_PERSISTENT", "EXEC_PLAIN", "EXEC_ASYNC")},
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gltrsv.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    for macro in CONSTANTS:
        lines.append(f'    printf("const {macro} %d\\n", (int)({macro}));')
    lines += ["    return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "abi.c", d / "abi"
    src.write_text("\n".join(lines) + "\n")
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    table = {}
    for line in out.splitlines():
        name, key, value = line.split()
        table[(name, key)] = int(value)
    return table


@pytest.mark.parametrize("name", list(STRUCTS))
def test_struct_matches_the_header(c_layout, name):
    import ctypes
    cls = STRUCTS[name]
    assert ctypes.sizeof(cls) == c_layout[(name, "size")], name
    for field, _ in cls._fields_:
        assert getattr(cls, field).offset == c_layout[(name, field)], (name, field)


def test_constants_match_the_header(c_layout):
    assert len(B.ERRORS) == 11
    for macro, value in CONSTANTS.items():
        assert c_layout[("const", macro)] == value, macro
    assert B.EXEC_NAMES[B.EXEC_PERSISTENT] == "persistent" and B.EXEC_NAMES[B.EXEC_ASYNC] == "async"
