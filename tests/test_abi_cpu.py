"""Host-side checks of the C ABI (no device calls)."""

import ctypes
import os
import re

import numpy as np
import pytest

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


@pytest.mark.parametrize("name", ["rp_problem", "rp_tune_entry"])
def test_struct_layout_matches_the_header(tmp_path, name):
    """The ctypes structs have the size and field offsets of the C structs
    (compiled from include/rp.h with the host compiler)."""
    import shutil
    import subprocess

    import paper_2001_02351_amd as rp
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    cls = getattr(rp, name)
    fields = [f[0] for f in cls._fields_]
    src = ['#include <stddef.h>', '#include <stdio.h>', '#include "rp.h"', "int main(void) {",
           f'  printf("%zu\\n", sizeof({name}));']
    src += [f'  printf("%zu\\n", offsetof({name}, {f}));' for f in fields]
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(cls)
    assert out[1:] == [getattr(cls, f).offset for f in fields]


def test_tuning_table_loading(tmp_path):
    import json

    import paper_2001_02351_amd as rp
    from paper_2001_02351_amd import _rp
    good = {"entries": [dict(ng_max=512, grid_max=27, chi_nw=1, chi_fill=0, fft_lines=8, chi_kernel=1)]}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(good))
    assert _rp.load_tuning(str(f)) == good["entries"]
    f.write_text(json.dumps({"entries": [dict(ng_max=512, grid_max=27)]}))
    with pytest.raises(ValueError):
        _rp.load_tuning(str(f))
    if os.path.exists(_rp.DEFAULT_TUNING):      # the committed table is well formed
        for e in _rp.load_tuning(_rp.DEFAULT_TUNING):
            assert e["chi_nw"] in (0, 1, 2) and -1 <= e["chi_fill"] and 0 <= e["fft_lines"] <= 64
            assert e["chi_kernel"] in (0, 1)
    assert rp.rp_tune_entry is _rp.rp_tune_entry


def test_autotune_class_problems_are_alias_free():
    """The tuner's synthetic inputs satisfy the pair kernel's alias-free
    condition N > 2 mmax + max |m + G0| on every class."""
    from paper_2001_02351_amd import autotune
    for edge in autotune.GRID_BUCKETS:
        for ng in autotune.NG_BUCKETS:
            p = autotune._ClassProblem(edge=edge, ng=ng, nocc=2, nemp=4)
            assert p.gsph.shape == (ng, 3) and len({tuple(g) for g in p.gsph.tolist()}) == ng
            for a in range(3):
                up = p.gsph[:, a].max() + (1 if p.iq[a] > 0 else 0)
                gmax = max(abs(int(p.gsph[:, a].min())), int(up))
                assert edge > 2 * int(p.mmax[a]) + gmax


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2001_02351_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f


def test_cell_average_host_routine_matches_the_oracle():
    """rp_coulomb_cell_average is host code (no device): the library's
    composite Gauss-Legendre value against the oracle's adaptive quadrature,
    cubic and triclinic cells, and the error path for a degenerate cell."""
    import paper_2001_02351_amd as rp
    from oracle import qsum
    for lat, kmesh in ((np.eye(3) * 7.26, (8, 8, 8)), (np.eye(3) * 5.0, (2, 3, 4)),
                       (np.array([[6.0, 0.8, 0.0], [0.5, 7.0, 0.0], [0.3, -0.4, 6.5]]), (3, 2, 4))):
        got = rp.rp_coulomb_cell_average(rp.make_cell(lat, (8, 8, 8), kmesh))
        want = qsum.cell_average(lat, kmesh)
        assert abs(got - want) < 1e-12 * want, (kmesh, got, want)
    with pytest.raises(rp.RpError):
        rp.rp_coulomb_cell_average(rp.make_cell(np.zeros((3, 3)), (8, 8, 8), (2, 2, 2)))


def test_pair_grid_is_the_smallest_alias_free_lane_grid():
    """rp_pair_grid (host code): the grid that steps a2-a4 run on holds the
    sphere products alias-free (N > 2 mmax + max |m + G0| per axis), takes
    N2 = N3 from the lane kernels' lengths of the precision and N1 from
    2^a 3^b 5^c, is never larger than the cell's grid, and is the cell's grid
    where no lane length fits."""
    import paper_2001_02351_amd as rp
    from synth.gen import A_SRVO3_BOHR, qpoint_gvectors
    lat = np.eye(3) * A_SRVO3_BOHR
    g, _ = qpoint_gvectors(lat, (8, 8, 8), (1, 0, 0), 1500, 10.0)
    cell = rp.make_cell(lat, (48, 48, 48), (8, 8, 8))
    for prec in (rp.RP_FP64, rp.RP_SPLIT_BF16):
        assert rp.rp_pair_grid(cell, (1, 0, 0), (12, 12, 12), g, prec) == (32, 32, 32)
    # m in [-7, 6] on axis 1 and q's G0 = 1 there: 2*12 + 7 = 31 < 32 on every axis;
    # one more unit of mmax on axis 1 needs N > 33 there: 36 for both of N2 = N3
    assert rp.rp_pair_grid(cell, (1, 0, 0), (12, 13, 12), g, rp.RP_SPLIT_BF16) == (32, 36, 36)
    assert rp.rp_pair_grid(cell, (1, 0, 0), (13, 12, 12), g, rp.RP_SPLIT_BF16) == (36, 32, 32)
    # bound 2*11 + 3 = 25: FP32 lines of 27, FP64 lines of 32 (no 25, 27, 30 in FP64); N1 = 27
    cube = np.array([(i, j, k) for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)], np.int32)
    c0 = rp.make_cell(lat, (48, 48, 48), (2, 2, 2))
    assert rp.rp_pair_grid(c0, (0, 0, 0), (11, 11, 11), cube, rp.RP_SPLIT_BF16) == (27, 27, 27)
    assert rp.rp_pair_grid(c0, (0, 0, 0), (11, 11, 11), cube, rp.RP_FP64) == (27, 32, 32)
    # never above the cell's grid; N2 != N3 keeps the cell's grid
    for fft, want in (((30, 30, 30), (27, 27, 27)), ((27, 27, 27), (27, 27, 27)), ((32, 30, 30), (27, 27, 27)),
                      ((48, 48, 40), (48, 48, 40))):
        got = rp.rp_pair_grid(rp.make_cell(lat, fft, (2, 2, 2)), (0, 0, 0), (11, 11, 11), cube, rp.RP_SPLIT_BF16)
        assert got == want, (fft, got)
    with pytest.raises(rp.RpError) as e:
        rp.rp_pair_grid(rp.make_cell(lat, (24, 24, 24), (2, 2, 2)), (0, 0, 0), (11, 11, 11), cube, rp.RP_FP64)
    assert e.value.status == 4                      # RP_E_ALIAS: the cell's own grid folds


def test_binding_checks_tensor_dtype_and_size():
    """The binding refuses a tensor of the wrong dtype or with fewer elements
    than the call reads or writes, before anything reaches the library."""
    torch = pytest.importorskip("torch")
    from paper_2001_02351_amd import _rp
    t = torch.zeros(10, dtype=torch.float64)
    _rp._need(t, "x", "f64", 10)
    _rp._need(None, "x", "f64", 10, optional=True)
    with pytest.raises(ValueError, match="elements"):
        _rp._need(t, "x", "f64", 11)
    with pytest.raises(ValueError, match="expected"):
        _rp._need(t.float(), "x", "f64", 4)
    with pytest.raises(ValueError, match="expected"):
        _rp._need(t, "x", "i32", 4)
    with pytest.raises(ValueError, match="required"):
        _rp._need(None, "x", "f64", 1)
    cell = _rp.make_cell(np.eye(3), (4, 5, 6), (2, 3, 4))
    assert _rp._nk(cell) == 24 and _rp._nr(cell) == 120
    assert _rp._pairs(0, 3, 3, 7, 1, 4) == 36
