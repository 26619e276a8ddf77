"""The large-supercell shape: 96^3 grid, Gamma-only k mesh, q = 0 (G = 0
dropped), 600 + 1200 bands, N_G = 6000, sampling weights (N_k = 1), 20 Wannier
orbitals.  Checked where the oracle can follow, and by properties that hold at
any size where it cannot:

* pair densities of 8 x 16 bands (FP64 and FP32 grids) against the oracle,
* chi of those pairs at N_G = 6000 (two frequencies) on a sampled block,
* chi of 16 800 pairs (two FP32 slices of the split contraction) at N_G = 6000
  on sampled rows and columns against the oracle,
* eps^-1 at N_G = 6000 of a synthetic chi: the residual eps eps^-1 - I, and W
  against its definition v^1/2 eps^-1 v^1/2 (v^1/2 computed here),
* W_ij of the 20 orbitals (first 600 G of the sphere, empty tail) against the
  oracle.
"""

import math

import numpy as np
import pytest

import oracle
from synth import supercell_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HARTREE_EV = 27.211386245988


def _rel(a, b):
    """The larger of the relative Frobenius norm of a - b and the largest
    element-wise deviation over the largest |b|."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    return max(np.linalg.norm(d) / np.linalg.norm(b), d.max() / np.abs(b).max())


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
def sc():
    print("[supercell] generating the 96^3 / Gamma / 1800-band workload", flush=True)
    return supercell_workload()


@pytest.fixture(scope="module")
def dsc(sc, rp):
    from paper_2001_02351_amd.path import DeviceInputs
    return DeviceInputs(sc)


O, E = (0, 8), (600, 616)


@pytest.fixture(scope="module")
def oracle_pairs(sc):
    print("[supercell] oracle pair densities (128 pairs) and sampling weights", flush=True)
    return oracle.pair_densities(sc, *O, *E, 0, 1), oracle.prob_weights(sc, *O, *E, 0, 1)


def test_supercell_pair_densities(ctx, rp, sc, dsc, oracle_pairs):
    from paper_2001_02351_amd import path
    M, _ = oracle_pairs
    for prec, tol in ((rp.RP_FP64, 1e-12), (rp.RP_SPLIT_BF16, 2e-6)):
        got = path.to_complex(path.pair_density(ctx, dsc, 0, 1, o=O, e=E, prec=prec))
        err = _rel(got, M)
        print(f"[supercell] M prec={prec}: rel err {err:.2e}", flush=True)
        assert err < tol


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)])
def test_supercell_chi_block(ctx, rp, sc, dsc, oracle_pairs, prec, tol):
    from paper_2001_02351_amd import path
    M, w = oracle_pairs
    nf = 2
    Md = path.pair_density(ctx, dsc, 0, 1, o=O, e=E, prec=prec)
    chi = torch.empty((nf, dsc.ng, dsc.ng, 2), dtype=torch.float64, device="cuda")
    rp.rp_chi0_accumulate(ctx, dsc.cell, sc.iq, dsc.nband, dsc.energy, dsc.T, *O, *E, 0, 1, dsc.ng, Md,
                          nf, sc.freq_eV[:nf], sc.delta_eV, path.weight_mode(sc), prec, 0, chi)
    rng = np.random.default_rng(7)
    cols = np.unique(np.concatenate([rng.choice(sc.ng, 48, replace=False), [0, sc.ng - 1]]))
    idx = torch.from_numpy(cols).cuda()
    got = path.to_complex(chi.index_select(1, idx).index_select(2, idx))
    want = oracle.chi0(M[:, cols], w[:nf])
    err = max(_rel(got[f], want[f]) for f in range(nf))
    print(f"[supercell] chi block prec={prec}: rel err {err:.2e}", flush=True)
    assert err < tol


SLICED = (0, 600), (600, 628)   # 16 800 pairs: 525 pair steps, two FP32 slices of the split contraction


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)])
def test_supercell_sliced_chi_block(ctx, rp, sc, dsc, prec, tol):
    """A block of 600 x 28 bands (16 800 pairs, more than one 512-step FP32
    slice of the split contraction, so it is cut into two slices summed in
    FP64) at N_G = 6000 and two frequencies, against the oracle's Eq. chi of
    the same pairs on sampled rows and columns (slab |m3| <= 1 of the sphere,
    spread over the row tiles), per frequency: relative Frobenius norm and
    largest element-wise deviation over the largest |chi|."""
    from paper_2001_02351_amd import path
    from dataclasses import replace
    O2, E2 = SLICED
    nf = 2
    rng = np.random.default_rng(17)
    slab = np.where(np.abs(sc.gsph[:, 2]) <= 1)[0]
    cols = []
    for t in range(0, sc.ng, 512):
        cand = slab[(slab >= t) & (slab < t + 512)]
        if len(cand):
            cols.append(int(rng.choice(cand)))
    cols = np.unique(np.concatenate([cols, rng.choice(np.setdiff1d(slab, cols), 40 - len(cols), replace=False)]))
    print(f"[supercell] oracle pair densities of 16 800 pairs on {len(cols)} columns", flush=True)
    M = oracle.pair_densities(replace(sc, gsph=np.ascontiguousarray(sc.gsph[cols])), *O2, *E2, 0, 1)
    w = oracle.prob_weights(sc, *O2, *E2, 0, 1)[:nf]
    want = oracle.chi0(M, w)
    npair = (O2[1] - O2[0]) * (E2[1] - E2[0])
    Md = torch.empty((npair, dsc.ng, 2), dtype=torch.float64, device="cuda")
    path.pair_density(ctx, dsc, 0, 1, o=O2, e=E2, out=Md, prec=prec)
    chi = torch.empty((nf, dsc.ng, dsc.ng, 2), dtype=torch.float64, device="cuda")
    rp.rp_chi0_accumulate(ctx, dsc.cell, sc.iq, dsc.nband, dsc.energy, dsc.T, *O2, *E2, 0, 1, dsc.ng, Md,
                          nf, sc.freq_eV[:nf], sc.delta_eV, path.weight_mode(sc), prec, 0, chi)
    idx = torch.from_numpy(cols).cuda()
    got = path.to_complex(chi.index_select(1, idx).index_select(2, idx))
    err = max(_rel(got[f], want[f]) for f in range(nf))
    print(f"[supercell] sliced chi block prec={prec}: rel err {err:.2e}", flush=True)
    assert err < tol


def _vsqrt(p):
    """sqrt(4 pi / Omega) / |q + G| for the problem's sphere (written out here)."""
    rec = 2.0 * math.pi * np.linalg.inv(p.lat).T
    q = np.array(p.iq, float) / np.array(p.kmesh, float)
    qg = (p.gsph + q) @ rec
    return math.sqrt(4.0 * math.pi / abs(np.linalg.det(p.lat))) / np.linalg.norm(qg, axis=1)


def test_supercell_screen(ctx, rp, sc, dsc):
    p = sc
    ng = p.ng
    rng = np.random.default_rng(3)
    A = (rng.standard_normal((ng, 120)) + 1j * rng.standard_normal((ng, 120))) * 0.02
    chi = -(A @ A.conj().T)[None]
    chi_t = torch.from_numpy(np.ascontiguousarray(chi).view(np.float64).reshape(chi.shape + (2,))).cuda()
    e_t = torch.empty_like(chi_t)
    W_t = torch.empty_like(chi_t)
    print("[supercell] eps^-1 of one 6000 x 6000 dielectric matrix", flush=True)
    rp.rp_screen_W(ctx, dsc.cell, p.iq, ng, p.gsph, 1, chi_t, e_t, W_t)
    rp.rp_synchronize(ctx)
    vs = torch.from_numpy(_vsqrt(p)).cuda()
    c = torch.view_as_complex(chi_t[0])
    eps = torch.eye(ng, dtype=torch.complex128, device="cuda") - vs[:, None] * c * vs[None, :]
    einv = torch.view_as_complex(e_t[0])
    res = eps @ einv - torch.eye(ng, dtype=torch.complex128, device="cuda")
    r = float(torch.linalg.norm(res) / math.sqrt(ng))
    print(f"[supercell] ||eps eps^-1 - I||_F / sqrt(N_G) = {r:.2e}", flush=True)
    assert r < 1e-12
    Wd = HARTREE_EV * vs[:, None] * einv * vs[None, :]
    W = torch.view_as_complex(W_t[0])
    assert float(torch.linalg.norm(W - Wd) / torch.linalg.norm(Wd)) < 1e-14


def test_supercell_wannier(ctx, rp, sc, dsc):
    p = sc
    ngs = 600
    gs = np.ascontiguousarray(p.gsph[:ngs])
    rng = np.random.default_rng(4)
    A = (rng.standard_normal((ngs, 40)) + 1j * rng.standard_normal((ngs, 40))) * 0.05
    chi = -(A @ A.conj().T)[None]
    _, einv, _ = oracle.screen(p.lat, p.kmesh, p.iq, gs, chi)
    print("[supercell] oracle Wannier densities (20 orbitals, 96^3, 600 G)", flush=True)
    rho_e = oracle.wannier_rho(p.lat, p.fft, p.kmesh, p.iq, p.phi, p.centre_frac, gs)
    rho_t = np.zeros((p.nwan, 0), np.complex128)
    want = oracle.wannier_W(p.lat, p.kmesh, rho_e, rho_t, einv)
    e_t = torch.from_numpy(np.ascontiguousarray(einv).view(np.float64).reshape(einv.shape + (2,))).cuda()
    Wij = torch.empty((1, p.nwan, p.nwan, 2), dtype=torch.float64, device="cuda")
    rp.rp_wannier_W(ctx, dsc.cell, p.iq, p.nwan, dsc.phi, p.centre_frac, ngs, gs, 0,
                    np.zeros((0, 3), np.int32), 1, e_t, Wij)
    from paper_2001_02351_amd import path
    got = path.to_complex(Wij)
    err = np.max(np.abs(got - want) / np.abs(want))
    print(f"[supercell] W_ij max elementwise rel err {err:.2e}", flush=True)
    assert err < 1e-10
