"""The C-ABI library loads and exports every function include/fga.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fga.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fga_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_three_steps():
    names = declared_functions()
    for n in ("fga_decompose", "fga_evolve", "fga_reconstruct_points", "fga_reconstruct_grid"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1810_06760_amd as fga
    if not os.path.exists(fga.LIB_PATH):
        fga_build = pytest.importorskip("paper_1810_06760_amd.build")
        fga_build.build()
    L = ctypes.CDLL(fga.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(fga.EXPORTED) == declared_functions()


def test_host_only_queries():
    import paper_1810_06760_amd as fga
    L = fga.lib()
    assert L.fga_version().decode().startswith("fga-gfx950")
    n = (ctypes.c_int * 3)(128, 128, 128)
    assert L.fga_medium_grid_table_bytes(n, 0) == 8 * 17 * 128 ** 3     # records + spline coefficients
    assert L.fga_medium_grid_table_bytes(n, 1) == 2 * 8 * 17 * 128 ** 3


def test_plane_layout_matches_header():
    import paper_1810_06760_amd as fga
    text = open(HEADER).read()
    for name in ("FGA_Q", "FGA_P", "FGA_ZQ_RE", "FGA_ZQ_IM", "FGA_ZP_RE", "FGA_ZP_IM", "FGA_A0_RE", "FGA_A1_IM",
                 "FGA_S", "FGA_W_RE", "FGA_W_IM", "FGA_E", "FGA_NF64", "FGA_BRANCH", "FGA_FLAGS", "FGA_NI32",
                 "FGA_FP64", "FGA_FP32", "FGA_BF16X3", "FGA_FP16X3", "FGA_FP16X2", "FGA_FP32_ACC32",
                 "FGA_COORDS_CARTESIAN", "FGA_COORDS_SPHERICAL"):
        m = re.search(r"\b%s = (\d+)" % name, text)
        assert m, name
        assert getattr(fga, name) == int(m.group(1)), name


STRUCTS = {"fga_beams": "Beams", "fga_medium": "MediumC", "fga_mesh": "MeshC", "fga_receivers": "ReceiversC",
           "fga_evolve_opts": "EvolveOptsC", "fga_evolve_stats": "EvolveStatsC",
           "fga_point_source": "PointSourceC", "fga_point_force": "PointForceC", "fga_request": "RequestC",
           "fga_completion": "CompletionC", "fga_beams_stats": "BeamsStatsC"}


def test_binding_structs_match_the_header(tmp_path):
    """Size and every field offset of the binding's ctypes mirrors equal those
    the C compiler gives the header's structs (gcc, host code only)."""
    import shutil
    import subprocess
    import paper_1810_06760_amd as fga
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fga.h"', "int main(void) {"]
    for cname, pname in STRUCTS.items():
        py = getattr(fga, pname)
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, pname in STRUCTS.items():
        py = getattr(fga, pname)
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
