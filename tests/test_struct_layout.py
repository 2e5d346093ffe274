"""The binding's ctypes structures have the header's layout.

A small C program compiled against include/chi0.h prints sizeof and the
offset of every member; the ctypes mirrors in paper_1005_5340_amd/chi0.py
must agree field by field (a field added to a header struct but not to the
binding, or in another order, would shift every later member)."""
import os
import shutil
import subprocess

import pytest

from paper_1005_5340_amd import chi0

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("chi0_solve_opts", chi0.SolveOpts), ("chi0_point_stats", chi0.PointStats),
         ("chi0_ws_cfg", chi0.WsCfg), ("chi0_lanczos_opts", chi0.LanczosOpts),
         ("chi0_kernel_record", chi0.KernelRecord), ("chi0_tune_record", chi0.TuneRecord)]


@pytest.fixture(scope="module")
def layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    d = tmp_path_factory.mktemp("layout")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "chi0.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    r = subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = {}
    for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        name, member, val = ln.split()
        out[(name, member)] = int(val)
    return out


@pytest.mark.parametrize("cname,cls", PAIRS, ids=[p[0] for p in PAIRS])
def test_ctypes_mirror_matches_header(layout, cname, cls):
    import ctypes
    assert ctypes.sizeof(cls) == layout[(cname, "size")]
    for f in cls._fields_:
        assert getattr(cls, f[0]).offset == layout[(cname, f[0])], f[0]
