"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (relative Frobenius norm per frequency for chi and eps^-1, per
element for W_ij, as the precision forms require):
  FP64 path        1e-10
  split-BF16 chi   1e-5
Pair densities and weights are compared at 1e-12 (both sides are FP64 and
differ only in summation order).
"""

import numpy as np
import pytest

import oracle
from synth import make_problem, parity_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    """The larger of the relative Frobenius norm of a - b and the largest
    element-wise deviation over the largest |b|."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    return max(np.linalg.norm(d) / np.linalg.norm(b), d.max() / np.abs(b).max())


def _rel_per_freq(a, b):
    return max(_rel(a[f], b[f]) for f in range(b.shape[0]))


@pytest.fixture(scope="module")
def rp():
    import paper_2001_02351_amd as rp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rp.load()
    return rp


@pytest.fixture(scope="module")
def ctx(rp):
    c = rp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c1():
    p = parity_workload()
    print("[oracle] parity-workload path", flush=True)
    ref = oracle.run_path(p)
    return p, ref


@pytest.fixture(scope="module")
def d1(c1, rp):
    from paper_2001_02351_amd.path import DeviceInputs
    return DeviceInputs(c1[0])


def test_pair_density_matches_oracle(ctx, c1, d1):
    from paper_2001_02351_amd import path
    p, ref = c1
    M = path.to_complex(path.pair_density(ctx, d1, 3, 6))
    npk = p.nocc * p.nemp
    assert _rel(M, ref["M"][3 * npk:6 * npk]) < 1e-12
    # ragged band and k ranges
    o, e, k = (1, 6), (9, 20), (60, 64)
    M2 = path.to_complex(path.pair_density(ctx, d1, *k, o=o, e=e))
    want = oracle.pair_densities(p, *o, *e, *k)
    assert M2.shape == want.shape
    assert _rel(M2, want) < 1e-12
    # FP32 grids (split-precision path)
    M3 = path.to_complex(path.pair_density(ctx, d1, *k, o=o, e=e, prec=1))
    assert _rel(M3, want) < 2e-6


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-6)])
def test_pair_density_on_a_smaller_alias_free_grid(ctx, rp, prec, tol):
    """A cell grid (40^3) far above what the sphere products need: steps
    a2-a4 run on the smaller grid rp_pair_grid reports and still give the
    oracle's densities on the cell's grid and the exact plane-wave form."""
    from paper_2001_02351_amd import path
    p = make_problem(name="oversampled", a_bohr=7.26, fft=(40, 40, 40), kmesh=(2, 2, 2), iq=(1, 0, 1), nocc=3,
                     nemp=4, gpsi=2.6, ng=27, freq_eV=np.array([0.0]), delta_eV=0.1, seed=5)
    d = path.DeviceInputs(p)
    grid = rp.rp_pair_grid(d.cell, p.iq, d.mmax, p.gsph, prec)
    print(f"[pair grid] prec={prec} cell 40^3 -> {grid}", flush=True)
    assert np.prod(grid) * 8 < np.prod(p.fft)
    M = path.to_complex(path.pair_density(ctx, d, 0, p.nk, prec=prec))
    want = oracle.pair_densities(p, 0, p.nocc, p.nocc, p.nocc + p.nemp, 0, p.nk)
    assert _rel(M, want) < tol
    kp, g0 = oracle.kq(p.kmesh, p.iq)
    for k in (0, 5):
        n, kk = int(p.npw[k]), int(kp[k])
        na = int(p.npw[kk])
        row = (k * p.nemp + 2) * p.nocc + 1              # empty band nocc + 2 at k+q, occupied band 1 at k
        exact = oracle.pair_conv(p.miller[kk, :na], p.coef[kk, p.nocc + 2, :na], p.miller[k, :n], p.coef[k, 1, :n],
                                 g0[k], p.gsph)
        assert np.max(np.abs(M[row] - exact)) < tol * np.abs(exact).max()


def test_weights_match_oracle(ctx, rp, c1, d1):
    from paper_2001_02351_amd import path
    p, ref = c1
    w = path.to_complex(path.weights(ctx, d1, 0, p.nk))
    assert np.max(np.abs(w - ref["w"])) < 1e-12 * np.abs(ref["w"]).max()
    ws = path.to_complex(path.weights(ctx, d1, 5, 9, mode=rp.RP_W_SAMPLING))
    want = oracle.prob_weights(p, 0, p.nocc, p.nocc, p.nband, 5, 9, mode=1)
    assert np.max(np.abs(ws - want)) < 1e-13 * np.abs(want).max()


def test_weights_crpa_and_imaginary_axis(ctx, rp):
    from paper_2001_02351_amd import path
    p = make_problem(name="t", a_bohr=7.26, fft=(12, 12, 12), kmesh=(3, 3, 2), iq=(1, 2, 1),
                     nocc=3, nemp=5, gpsi=2.4, ng=20, freq_eV=1j * np.array([0.0, 0.3, 2.0, 30.0]),
                     delta_eV=0.0, crpa=True, seed=17)
    d = path.DeviceInputs(p)
    w = path.to_complex(path.weights(ctx, d, 0, p.nk))
    want = oracle.prob_weights(p, 0, 3, 3, 8, 0, p.nk)
    assert np.max(np.abs(w - want)) < 1e-12 * np.abs(want).max()


def test_chi0_fp64_matches_oracle(ctx, rp, c1, d1):
    from paper_2001_02351_amd import path
    p, ref = c1
    chi = path.to_complex(path.chi0(ctx, d1, prec=rp.RP_FP64, kbatch=4))
    err = _rel_per_freq(chi, ref["chi"])
    print(f"chi fp64 rel err {err:.2e}")
    assert err < 1e-10


def test_chi0_batch_linearity(ctx, rp, c1, d1):
    """chi over [0,64) equals chi over [0,20) plus chi over [20,64) (band-pair
    block decomposition of Eq. chi)."""
    from paper_2001_02351_amd import path
    a = path.to_complex(path.chi0(ctx, d1, kbatch=7, k0=0, k1=20))
    b = path.to_complex(path.chi0(ctx, d1, kbatch=5, k0=20, k1=64))
    whole = path.to_complex(path.chi0(ctx, d1, kbatch=64))
    assert _rel_per_freq(a + b, whole) < 1e-13


def test_chi0_split_bf16_matches_oracle(ctx, rp, c1, d1):
    from paper_2001_02351_amd import path
    p, ref = c1
    chi = path.to_complex(path.chi0(ctx, d1, prec=rp.RP_SPLIT_BF16, kbatch=8))
    err = _rel_per_freq(chi, ref["chi"])
    print(f"chi split-bf16 rel err {err:.2e}")
    assert err < 1e-5


def test_screen_matches_oracle(ctx, rp, c1, d1):
    from paper_2001_02351_amd import path
    p, ref = c1
    chi_t = torch.from_numpy(np.ascontiguousarray(ref["chi"]).view(np.float64).reshape(
        ref["chi"].shape + (2,))).cuda()
    einv, W = path.screen(ctx, d1, chi_t)
    rp.rp_synchronize(ctx)
    assert _rel_per_freq(path.to_complex(einv), ref["eps_inv"]) < 1e-10
    assert _rel_per_freq(path.to_complex(W), ref["W"]) < 1e-10


def test_wannier_matches_oracle(ctx, rp, c1, d1):
    from paper_2001_02351_amd import path
    p, ref = c1
    einv = torch.from_numpy(np.ascontiguousarray(ref["eps_inv"]).view(np.float64).reshape(
        ref["eps_inv"].shape + (2,))).cuda()
    Wij = path.to_complex(path.wannier(ctx, d1, einv))
    assert np.max(np.abs(Wij - ref["Wij"]) / np.abs(ref["Wij"])) < 1e-10


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)])
def test_end_to_end(ctx, rp, c1, d1, prec, tol):
    from paper_2001_02351_amd import path
    p, ref = c1
    out = path.run_q(ctx, d1, prec=prec, kbatch=16)
    rp.rp_synchronize(ctx)
    e_chi = _rel_per_freq(path.to_complex(out["chi"]), ref["chi"])
    e_inv = _rel_per_freq(path.to_complex(out["eps_inv"]), ref["eps_inv"])
    Wij = path.to_complex(out["Wij"])
    e_w = np.max(np.abs(Wij - ref["Wij"]) / np.abs(ref["Wij"]))
    print(f"prec {prec}: chi {e_chi:.2e} eps_inv {e_inv:.2e} W_ij {e_w:.2e}")
    assert e_chi < tol and e_inv < tol and e_w < tol


def test_abi_errors(ctx, rp, c1, d1):
    from paper_2001_02351_amd import path
    p, _ = c1
    d = d1
    # large enough for every call below (the binding refuses a tensor smaller
    # than the pair ranges ask for before the library checks the ranges)
    M = torch.empty(((p.nocc + 2) * (p.nemp + 2), p.ng, 2), dtype=torch.float64, device="cuda")
    small = rp.make_cell(p.lat, (10, 10, 10), p.kmesh)
    with pytest.raises(rp.RpError) as e:
        rp.rp_pair_density(ctx, small, p.iq, d.nband, p.miller.shape[1], p.npw, d.mmax, d.miller,
                           d.coef, 0, p.nocc, p.nocc, p.nband, 0, 1, p.ng, p.gsph, 0, M)
    assert e.value.status == 4            # RP_E_ALIAS
    odd = rp.make_cell(p.lat, (16, 16, 14), p.kmesh)
    with pytest.raises(rp.RpError) as e:
        rp.rp_pair_density(ctx, odd, p.iq, d.nband, p.miller.shape[1], p.npw, d.mmax, d.miller,
                           d.coef, 0, p.nocc, p.nocc, p.nband, 0, 1, p.ng, p.gsph, 0, M)
    assert e.value.status == 8            # RP_E_UNSUPPORTED (factor 7)
    with pytest.raises(rp.RpError) as e:
        rp.rp_pair_density(ctx, d.cell, p.iq, d.nband, p.miller.shape[1], p.npw, d.mmax, d.miller,
                           d.coef, 0, p.nocc + 1, p.nocc, p.nband + 2, 0, 1, p.ng, p.gsph, 0, M)
    assert e.value.status == 2            # RP_E_SHAPE
    chi = torch.zeros((1, 4, 4, 2), dtype=torch.float64, device="cuda")
    g_with_zero = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.int32)
    with pytest.raises(rp.RpError) as e:
        rp.rp_screen_W(ctx, d.cell, (0, 0, 0), 4, g_with_zero, 1, chi, None, None)
    assert e.value.status == 3            # RP_E_RANGE: |q+G| = 0
    big = torch.empty((1, 6145, 6145, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(rp.RpError) as e:
        rp.rp_screen_W(ctx, d.cell, p.iq, 6145, np.ones((6145, 3), np.int32), 1, big, None, None)
    assert e.value.status == 8            # RP_E_UNSUPPORTED: N_G above the inversion's LDS plan
    del big
    # the binding refuses an undersized tensor before the library sees it
    with pytest.raises(ValueError, match="elements"):
        rp.rp_screen_W(ctx, d.cell, p.iq, 6145, np.ones((6145, 3), np.int32), 1, chi, None, None)
    with pytest.raises(rp.RpError) as e:
        rp.rp_weights(ctx, d.cell, p.iq, d.nband, d.energy, None, 0, 1, 1, 2, 0, 1, 1, [0.0],
                      -0.1, 0, torch.empty((1, 1, 2), dtype=torch.float64, device="cuda"))
    assert e.value.status == 3            # delta < 0


def test_singular_dielectric_matrix_is_reported(ctx, rp, c1, d1):
    """chi = v^-1 on the diagonal makes eps = 0 up to rounding: the pivot
    falls below the singularity floor and surfaces as RP_E_SINGULAR from
    rp_synchronize; a NaN in chi surfaces as RP_E_RANGE."""
    p, _ = c1
    g = p.gsph[1:5]
    b = 2 * np.pi * np.linalg.inv(p.lat).T
    qg = np.linalg.norm((np.array(p.iq) / np.array(p.kmesh) + g) @ b, axis=1)
    v = 4 * np.pi / abs(np.linalg.det(p.lat)) / qg ** 2
    chi = np.zeros((1, 4, 4), complex)
    chi[0][np.diag_indices(4)] = 1.0 / v
    chi_t = torch.from_numpy(chi.view(np.float64).reshape(1, 4, 4, 2)).cuda()
    out = torch.empty_like(chi_t)
    rp.rp_screen_W(ctx, d1.cell, p.iq, 4, g, 1, chi_t, out, None)
    with pytest.raises(rp.RpError) as e:
        rp.rp_synchronize(ctx)
    assert e.value.status == 7
    rp.rp_synchronize(ctx)                # the flag is cleared once reported
    chi[0, 1, 2] = np.nan
    chi[0][np.diag_indices(4)] = 0.0
    chi_t = torch.from_numpy(chi.view(np.float64).reshape(1, 4, 4, 2)).cuda()
    rp.rp_screen_W(ctx, d1.cell, p.iq, 4, g, 1, chi_t, out, None)
    with pytest.raises(rp.RpError) as e:
        rp.rp_synchronize(ctx)
    assert e.value.status == 3
