"""Host-side checks of the C ABI (no device calls)."""

import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rp_[a-zA-Z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("rp_create", "rp_destroy", "rp_synchronize", "rp_last_error", "rp_pair_density",
              "rp_weights", "rp_chi0_accumulate", "rp_screen_W", "rp_wannier_W"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2001_02351_amd as rp
    if not os.path.exists(rp.library_path()):
        rp.build()
    lib = ctypes.CDLL(rp.library_path())
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(rp.EXPORTED) == _declared()


def test_cell_marshalling():
    import paper_2001_02351_amd as rp
    lat = np.array([[7.0, 0.1, 0.0], [0.0, 7.5, 0.2], [0.3, 0.0, 8.0]])
    c = rp.make_cell(lat, (16, 18, 20), (4, 3, 2))
    assert ctypes.sizeof(c) == 9 * 8 + 6 * 4
    assert [[c.lat[i][j] for j in range(3)] for i in range(3)] == lat.tolist()
    assert list(c.fft) == [16, 18, 20] and list(c.kmesh) == [4, 3, 2]


def test_problem_struct_layout_matches_the_header(tmp_path):
    """The ctypes rp_problem has the size and field offsets of the C struct
    (compiled from include/rp.h with the host compiler)."""
    import shutil
    import subprocess

    import paper_2001_02351_amd as rp
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        import pytest
        pytest.skip("no host C compiler")
    fields = [f[0] for f in rp.rp_problem._fields_]
    src = ['#include <stddef.h>', '#include <stdio.h>', '#include "rp.h"', "int main(void) {",
           '  printf("%zu\\n", sizeof(rp_problem));']
    src += [f'  printf("%zu\\n", offsetof(rp_problem, {f}));' for f in fields]
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(rp.rp_problem)
    assert out[1:] == [getattr(rp.rp_problem, f).offset for f in fields]


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2001_02351_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f
