"""The C-ABI library loads (no GPU needed) and exports every function that
include/sph.h declares; the ctypes layouts agree with the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sph_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_interface():
    names = declared_functions()
    for f in ("sph_build_tree", "sph_neighbors", "sph_density", "sph_forces", "sph_step"):
        assert f in names


def test_library_exports_every_declared_symbol():
    sph = pytest.importorskip("paper_2511_11425_amd")
    lib = ctypes.CDLL(sph.LIB_PATH)
    for f in declared_functions():
        assert hasattr(lib, f), f
    assert set(declared_functions()) == set(sph.SYMBOLS)


def test_defaults_and_version_without_gpu():
    sph = pytest.importorskip("paper_2511_11425_amd")
    assert "gfx950" in sph.version()
    p = sph.make_params({"n_ngb": 64})
    assert p.bucket == 32 and abs(p.oversel - 1.1) < 1e-15 and p.nr_maxit == 64


def test_struct_layouts_match_header(tmp_path):
    """Offsets of every field as the C compiler lays out include/sph.h."""
    sph = pytest.importorskip("paper_2511_11425_amd")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sph.h"', "int main(void) {"]
    for cname, py in (("sph_params", sph.Params), ("sph_particles", sph.Particles),
                      ("sph_stats", sph.Stats)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, py in (("sph_params", sph.Params), ("sph_particles", sph.Particles),
                      ("sph_stats", sph.Stats)):
        assert got[(cname, "size")] == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_invalid_parameters_are_rejected_without_gpu():
    sph = pytest.importorskip("paper_2511_11425_amd")
    with pytest.raises(sph.SphError):
        sph.Context({"n_ngb": 5.0})           # below (4 pi/3) sigma of the cubic spline
    with pytest.raises(sph.SphError):
        sph.Context({"n_ngb": 64, "bucket": 48})
    with pytest.raises(sph.SphError):
        sph.Context({"n_ngb": 64}, set_offsets=[0, 10, 5])
