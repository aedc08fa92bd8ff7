"""CPU checks of the C ABI: the library loads, exports every symbol the header declares, and
the ctypes structs match the C layout (no compute call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "varsim.h")
LIB = os.path.join(ROOT, "paper_2307_12119_amd", "libvarsim.so")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"VARSIM_API\s+[\w\s\*]*?\b(varsim_\w+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for required in ("varsim_create", "varsim_destroy", "varsim_green_table", "varsim_conv",
                     "varsim_workspace_size", "varsim_solve_steady", "varsim_solve_batch",
                     "varsim_solve_transient", "varsim_kernel_times"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    from paper_2307_12119_amd import varsim as V

    assert set(V.EXPORTS) == set(_declared())


def test_struct_layouts_match_c(tmp_path):
    from paper_2307_12119_amd import varsim as V

    structs = {"varsim_layer": V.Layer, "varsim_geometry": V.Geometry, "varsim_options": V.Options,
               "varsim_problem": V.Problem, "varsim_stats": V.Stats, "varsim_transient": V.Transient,
               "varsim_net_config": V.NetConfig}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "varsim.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    for line in filter(None, out):
        cname, field, val = line.split()
        py = structs[cname]
        if field == "size":
            assert ctypes.sizeof(py) == int(val), cname
        else:
            assert getattr(py, field).offset == int(val), (cname, field)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for several it prints one JSON error line and exits 2
    before generating inputs or touching a device."""
    import json
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
