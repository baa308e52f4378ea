"""The ctypes structures of the Python binding have the sizes and field offsets
of the C structures that include/rtq.h declares (compiled here with the host C
compiler; no GPU needed)."""
import ctypes
import json
import os
import shutil
import subprocess

import pytest

rtq = pytest.importorskip("paper_2001_02620_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = {
    "rtq_prototype": rtq._Proto, "rtq_instances": rtq._Insts, "rtq_build_opts": rtq._BuildOpts,
    "rtq_scene_info": rtq._Info, "rtq_rays": rtq._Rays, "rtq_hits": rtq._Hits, "rtq_trace_opts": rtq._TraceOpts,
    "rtq_camera": rtq._Camera, "rtq_render_opts": rtq._RenderOpts,
}


def test_binding_structs_match_the_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no host C compiler or HIP headers")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rtq.h"', "int main(void) {", 'printf("{");']
    first = True
    for cname, py in PAIRS.items():
        for f, _ in [("__size__", None)] + list(py._fields_):
            expr = f"sizeof({cname})" if f == "__size__" else f"offsetof({cname}, {f})"
            sep = "" if first else ","
            first = False
            lines.append(f'printf("{sep}\\"{cname}.{f}\\": %zu", (size_t)({expr}));')
    lines += ['printf("}\\n");', "return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I",
                        "/opt/rocm/include", str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    c = json.loads(subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout)
    for cname, py in PAIRS.items():
        assert c[f"{cname}.__size__"] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert c[f"{cname}.{f}"] == getattr(py, f).offset, (cname, f)
