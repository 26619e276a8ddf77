"""The oracle's C routines under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle.c is built a second time with -fsanitize=address,undefined (any
undefined-behaviour report fatal) and loaded by a child Python process with
the sanitizer runtimes preloaded.  The child runs every C entry point on a
small problem (k + q map, u-grids and pair densities by the direct and the
separable transforms and by the plane-wave convolution, the batched u-grids
and pair densities of the path, the divided differences and vertex
integrals, the weights with the cRPA T, chi0, the inversion, eps^-1 and W,
the Wannier densities and W_ij); it must end cleanly, with no sanitizer
report, and every result must equal the regular build's to 1e-12.  A second
test plants an off-by-one overflow in a scratch copy of oracle.c and expects
the report, so that a run without the sanitizers cannot pass unnoticed.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
import numpy as np
sys.path.insert(0, sys.argv[2])
import oracle
from synth import make_problem
p = make_problem(name="san", a_bohr=7.26, fft=(12, 12, 12), kmesh=(2, 2, 2), iq=(1, 0, 1), nocc=3, nemp=4,
                 gpsi=2.2, ng=19, freq_eV=np.array([0.0, 3.0, 9.0]), delta_eV=0.1, nwan=2, crpa=True, seed=5)
out = {}
kp, g0 = oracle.kq(p.kmesh, p.iq)
out["kp"], out["g0"] = kp, g0
k, kk = 3, kp[3]
na, nb = p.npw[kk], p.npw[k]
for method in ("direct", "separable"):
    ua = oracle.u_grid(p.fft, p.miller[kk, :na], p.coef[kk, 4, :na], method)
    ub = oracle.u_grid(p.fft, p.miller[k, :nb], p.coef[k, 1, :nb], method)
    out["u_" + method] = ua
    out["M_" + method] = oracle.pair_density(p.fft, ua, ub, g0[k], p.gsph, method)
out["M_conv"] = oracle.pair_conv(p.miller[kk, :na], p.coef[kk, 4, :na], p.miller[k, :nb], p.coef[k, 1, :nb],
                                 g0[k], p.gsph)
out["dd4"] = np.array([oracle.dd4(2.0 + 0.1j, [0.3, 0.5, 0.5, 1.1, 1.7])])
out["vertex"] = np.array([oracle.vertex_integral(1.2 + 0.05j, [0.1, 0.4, 0.9, 1.6], i) for i in range(4)])
out["tetra"] = np.array([oracle.tetra_scalar(1.2 + 0.05j, [0.1, 0.4, 0.9, 1.6])])
inv = np.eye(5) + 0.1 * np.arange(25).reshape(5, 5) / 25.0
out["invert"] = oracle.invert(inv.astype(np.complex128))
run = oracle.run_path(p)
for key, val in run.items():
    out["path_" + key] = val
np.savez(sys.argv[1], **out)
'''


def test_oracle_c_under_sanitizers(tmp_path):
    san = obuild.build_sanitized(str(tmp_path / "liboracle_san.so"))
    res_san, res_ref = tmp_path / "san.npz", tmp_path / "ref.npz"
    script = tmp_path / "child.py"
    script.write_text(CHILD)
    env = dict(os.environ, RP_ORACLE_LIB=san, LD_PRELOAD=obuild.sanitizer_preload(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, str(script), str(res_san), ROOT], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    env_ref = {k: v for k, v in os.environ.items() if k not in ("RP_ORACLE_LIB", "LD_PRELOAD")}
    r = subprocess.run([sys.executable, str(script), str(res_ref), ROOT], env=env_ref, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    a, b = np.load(res_san), np.load(res_ref)
    assert sorted(a.files) == sorted(b.files)
    for key in b.files:
        x, y = a[key], b[key]
        scale = max(1.0, float(np.abs(y).max()))
        assert np.abs(x - y).max() <= 1e-12 * scale, key
    assert np.abs(b["path_Wij"]).max() > 0 and np.abs(b["path_chi"]).max() > 0


def test_sanitized_run_reports_a_planted_overflow(tmp_path):
    """The checking run is live: a scratch copy of oracle.c whose inversion
    clears one element past its output (an off-by-one loop bound), built and
    loaded the same way, ends with AddressSanitizer's heap-buffer-overflow
    report."""
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    good = "    for (long i = 0; i < (long)n * n; i++) Ainv[i] = 0;"
    assert good in src
    bad = tmp_path / "oracle_planted.c"
    bad.write_text(src.replace(good, good.replace("i < (long)n * n", "i <= (long)n * n"), 1))
    lib = str(tmp_path / "liboracle_planted.so")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", str(bad), "-o", lib, "-lm"])
    env = dict(os.environ, RP_ORACLE_LIB=lib, LD_PRELOAD=obuild.sanitizer_preload(),
               ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="1")
    code = (f"import sys; sys.path.insert(0, {ROOT!r}); import numpy as np, oracle; "
            "oracle.invert(np.eye(20, dtype=complex)); print('no report')")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stdout + r.stderr[-2000:]
