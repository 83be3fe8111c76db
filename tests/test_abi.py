"""The C-ABI library loads, exports every entry point include/flaproj.h
declares, and the binding's struct layouts match the header (checked with a
probe compiled by gcc from the header itself).  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flaproj.h")
LIB = os.path.join(ROOT, "paper_2512_20829_amd", "libflaproj.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python paper_2512_20829_amd/build.py)"
    names = declared_functions()
    assert {"fla_ctx_create", "fla_ctx_destroy", "fla_project_sources", "psicell_accumulate",
            "fla_get_stats", "fla_last_error"} <= set(names)
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in flaproj.h but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(names) <= exported


def test_struct_layout_matches_header(tmp_path):
    import paper_2512_20829_amd as F
    structs = [F.fla_mesh, F.fla_trajectories, F.fla_params, F.fla_fields, F.fla_stats, F.fla_profile]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "flaproj.h"', "int main(void){"]
    for s in structs:
        nm = s.__name__
        lines.append(f'printf("{nm} size %zu\\n", sizeof({nm}));')
        for f, _ in s._fields_:
            lines.append(f'printf("{nm} {f} %zu\\n", offsetof({nm}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, c = l.split()
        got[(a, b)] = int(c)
    for s in structs:
        assert got[(s.__name__, "size")] == ctypes.sizeof(s), s.__name__
        for f, _ in s._fields_:
            assert got[(s.__name__, f)] == getattr(s, f).offset, (s.__name__, f)


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2512_20829_amd as F
    with pytest.raises(F.FlaError) as e:
        F.Context(0)
    assert e.value.status == F.FLA_ERR_DEVICE
    assert F.lib().fla_last_error(None)


def test_binding_has_no_cpu_fallback():
    """The binding refers to the library only; nothing under oracle/ is imported."""
    pkg = os.path.join(ROOT, "paper_2512_20829_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
