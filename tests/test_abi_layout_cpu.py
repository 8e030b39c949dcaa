"""The binding's ctypes mirrors of the C-ABI structs (paper_1809_04352_amd/eses.py)
have the layout the header declares: each struct's size and every field's
offset, as the host C compiler lays out include/eses.h."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# ctypes class -> (C typedef, ctypes field names that differ from the C ones)
MIRRORS = {
    "Molecule": ("eses_molecule", {}),
    "Config": ("eses_config", {}),
    "CandidateStats": ("eses_candidate_stats", {}),
    "ClassifyStats": ("eses_classify_stats", {}),
    "EdgeStats": ("eses_edge_stats", {}),
    "KernelTimes": ("eses_kernel_times", {}),
    "MeshStats": ("eses_mesh_stats", {}),
    "IsectSoA": ("eses_isect_soa", {"lambda_": "lambda"}),
}


def c_layout(tmp_path):
    from paper_1809_04352_amd import eses
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "eses.h"',
             "int main(void) {"]
    for cls, (cname, rename) in MIRRORS.items():
        lines.append(f'    printf("{cls} %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(eses, cls)._fields_:
            cf = rename.get(fname, fname)
            lines.append(f'    printf("{cls}.{fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (line.split() for line in out.splitlines())}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_mirrors_match_the_header(tmp_path):
    from paper_1809_04352_amd import eses
    c = c_layout(tmp_path)
    for cls in MIRRORS:
        k = getattr(eses, cls)
        assert ctypes.sizeof(k) == c[cls], cls
        for fname, _ in k._fields_:
            assert getattr(k, fname).offset == c[f"{cls}.{fname}"], (cls, fname)
