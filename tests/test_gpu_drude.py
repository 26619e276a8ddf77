"""GPU parity of the intraband (Drude) head term (Eqs. eps00, plasma,
momentum) against the oracle (oracle/drude.py): the plasma tensor of a metal
with and without the cRPA factor, and eps^-1 at q -> 0 with the term on the
real and the imaginary axis, including the frequencies where it is
infinite."""

import dataclasses
import math

import numpy as np
import pytest

from oracle import drude, head

torch = pytest.importorskip("torch")


def _rel(a, b):
    """The larger of the relative Frobenius norm of a - b and the largest
    element-wise deviation over the largest |b|."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    return max(np.linalg.norm(d) / np.linalg.norm(b), d.max() / np.abs(b).max())
pytestmark = pytest.mark.gpu

HA = drude.HARTREE_EV


@pytest.fixture(scope="module")
def rp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_02351_amd as rp
    rp.load()
    return rp


@pytest.fixture(scope="module")
def ctx(rp):
    c = rp.Context(0)
    yield c
    c.close()


def _metal():
    from synth import make_problem
    p = make_problem(name="drude", a_bohr=7.26, fft=(12, 12, 12), kmesh=(4, 3, 3), iq=(0, 0, 0), nocc=3, nemp=3,
                     gpsi=2.4, ng=19, freq_eV=np.array([0.0]), delta_eV=0.1, seed=23)
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in p.kmesh], indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(5)
    c = np.sort(rng.uniform(-3.0, 3.0, 6))
    t = rng.uniform(0.5, 1.5, (6, 3))
    E = np.stack([c[n] - np.sum(t[n] * np.cos(2 * math.pi * kf + n), axis=1) for n in range(6)], 1)
    T = rng.uniform(0.0, 1.0, E.shape)
    return dataclasses.replace(p, energy_eV=np.ascontiguousarray(E), T=np.ascontiguousarray(T))


@pytest.mark.parametrize("crpa", [False, True])
def test_plasma_tensor_matches_oracle(rp, ctx, crpa):
    from paper_2001_02351_amd import path
    p = _metal()
    d = path.DeviceInputs(p)
    ef, b0, b1 = 0.2, 1, 6
    got = rp.rp_plasma_frequency(ctx, d.cell, d.nband, p.miller.shape[1], p.npw, d.miller, d.coef, d.energy,
                                 d.T if crpa else None, b0, b1, ef)
    want = drude.plasma_tensor(p, b0, b1, ef, T=p.T if crpa else None) * HA * HA
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"[drude] plasma tensor crpa={crpa}: diag {np.diag(got)} eV^2, rel {err:.1e}", flush=True)
    assert np.abs(want).max() > 0.1
    assert err < 1e-10
    # E_F below every band: no Fermi surface
    z = rp.rp_plasma_frequency(ctx, d.cell, d.nband, p.miller.shape[1], p.npw, d.miller, d.coef, d.energy, None, 0,
                               6, -50.0)
    assert np.all(z == 0.0)


def _chi(ng, nfreq, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nfreq):
        a = rng.normal(size=(ng, ng)) + 1j * rng.normal(size=(ng, ng))
        h = -(a @ a.conj().T) * (0.02 / ng)
        out.append(h + 0.002j * np.eye(ng))
    return np.stack(out)


@pytest.mark.parametrize("axis", ["real", "imaginary"])
def test_drude_head_matches_oracle(rp, ctx, axis):
    lat = np.eye(3) * 7.26
    cell = rp.make_cell(lat, (12, 12, 12), (4, 4, 4))
    gsph = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1], [1, 1, 0],
                     [1, -1, 0], [0, 1, 1], [1, 0, 1]], np.int32)
    ng = len(gsph)
    if axis == "real":
        freq, delta = np.array([0.0, 0.5, 2.0, 6.0, 15.0], np.complex128), 0.1
    else:
        freq, delta = 1j * np.array([0.0, 0.3, 2.0, 9.0]), 0.0
    nf = len(freq)
    chi = _chi(ng, nf, 7)
    wq = 9.5                                    # eV^2
    chi_d = torch.from_numpy(chi.view(np.float64).reshape(nf, ng, ng, 2).copy()).cuda()
    einv = torch.empty_like(chi_d)
    opt = torch.empty((nf, 5), dtype=torch.float64, device="cuda")
    rp.rp_set_drude(ctx, wq, delta)
    try:
        rp.rp_screen_head(ctx, cell, ng, gsph, nf, freq, chi_d, einv, opt)
        rp.rp_synchronize(ctx)
    finally:
        rp.rp_set_drude(ctx, 0.0, 0.0)
    a = einv.cpu().numpy()
    got = a[..., 0] + 1j * a[..., 1]
    _, want = drude.drude_head(lat, gsph, chi, freq, delta, wq / HA ** 2, np.linalg.inv)
    err = max(_rel(got[f], want[f]) for f in range(nf))
    print(f"[drude] head {axis}: eps^-1 rel {err:.1e}; eps^-1_00 {got[:, 0, 0]}", flush=True)
    assert err < 1e-12
    assert np.all(got[0, 0, :] == 0) and np.all(got[0, :, 0] == 0)      # w = 0: infinite head
    o = opt.cpu().numpy()
    assert o[0, 2] == 0.0 and o[0, 4] == 1.0 and np.all(np.isnan(o[0, [0, 1, 3]]))
    ref = head.optics(want[1:, 0, 0], freq[1:])
    for j, key in enumerate(("eps_M", None, "eels", "sigma", "refl")):
        if key is None:
            continue
        w = ref[key].real if key == "eps_M" else ref[key]
        assert np.allclose(o[1:, j], w, rtol=1e-10, atol=1e-13), key
    assert np.allclose(o[1:, 1], ref["eps_M"].imag, rtol=1e-10, atol=1e-13)
    # the term removed: the head oracle without it
    rp.rp_screen_head(ctx, cell, ng, gsph, nf, freq, chi_d, einv, None)
    rp.rp_synchronize(ctx)
    a = einv.cpu().numpy()
    _, plain = head.screen_head(lat, gsph, chi, np.linalg.inv)
    assert np.max(np.abs(a[..., 0] + 1j * a[..., 1] - plain)) < 1e-12 * np.abs(plain).max()


def test_drude_arguments(rp, ctx):
    with pytest.raises(rp.RpError):
        rp.rp_set_drude(ctx, float("nan"), 0.1)
    with pytest.raises(rp.RpError):
        rp.rp_set_drude(ctx, 1.0, -0.1)
    rp.rp_set_drude(ctx, 0.0, 0.0)


def test_metal_head_chain_matches_oracle(rp, ctx):
    """A metal at q -> 0 end to end in FP64: pair densities at iq = 0 with
    G = 0 first, the head densities along qhat in that column (intraband
    pairs zero), Fermi-cut weights over overlapping band ranges, the
    contraction, the plasma tensor of the same bands, and eps^-1 with the
    intraband term along qhat, against the oracle's chain."""
    import oracle
    from oracle import metal
    from paper_2001_02351_amd import path
    from synth import make_problem
    p = make_problem(name="metal_head", a_bohr=7.26, fft=(12, 12, 12), kmesh=(2, 2, 2), iq=(0, 0, 0), nocc=3, nemp=3,
                     gpsi=2.2, ng=26, freq_eV=np.array([0.0, 1.0, 4.0]), delta_eV=0.1, seed=29)
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in p.kmesh], indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(8)
    c = np.sort(rng.uniform(-3.0, 3.0, 6))
    t = rng.uniform(0.5, 1.5, (6, 3))
    E = np.stack([c[n] - np.sum(t[n] * np.cos(2 * math.pi * kf + n), axis=1) for n in range(6)], 1)
    p = dataclasses.replace(p, energy_eV=np.ascontiguousarray(E))
    gaug = np.ascontiguousarray(np.concatenate([np.zeros((1, 3), np.int32), np.asarray(p.gsph, np.int32)]))
    ng, nk, nf = len(gaug), p.nk, len(p.freq_eV)
    ef, o, e = 0.2, (0, 4), (2, 6)
    qhat = np.array([1.0, 0.5, 0.2]) / np.linalg.norm([1.0, 0.5, 0.2])
    d = path.DeviceInputs(p)
    npw_max = p.miller.shape[1]
    M = torch.empty((nk * 4 * 4, ng, 2), dtype=torch.float64, device="cuda")
    rp.rp_pair_density(ctx, d.cell, p.iq, d.nband, npw_max, p.npw, d.mmax, d.miller, d.coef, *o, *e, 0, nk, ng, gaug,
                       rp.RP_FP64, M)
    rp.rp_head_density(ctx, d.cell, d.nband, npw_max, p.npw, d.miller, d.coef, d.energy, *o, *e, 0, nk, qhat, ng, 0,
                       M)
    chi = torch.empty((nf, ng, ng, 2), dtype=torch.float64, device="cuda")
    einv = torch.empty_like(chi)
    rp.rp_set_fermi_level(ctx, ef)
    try:
        rp.rp_chi0_accumulate(ctx, d.cell, p.iq, d.nband, d.energy, None, *o, *e, 0, nk, ng, M, nf, p.freq_eV,
                              p.delta_eV, rp.RP_W_TETRA_METAL, rp.RP_FP64, 0, chi)
        Om = rp.rp_plasma_frequency(ctx, d.cell, d.nband, npw_max, p.npw, d.miller, d.coef, d.energy, None, 0, 6, ef)
        wq = float(qhat @ Om @ qhat)
        rp.rp_set_drude(ctx, wq, p.delta_eV)
        rp.rp_screen_head(ctx, d.cell, ng, gaug, nf, p.freq_eV, chi, einv, None)
        rp.rp_synchronize(ctx)
    finally:
        rp.rp_set_drude(ctx, 0.0, 0.0)
        rp.rp_set_fermi_level(ctx, float("nan"))
    got_chi, got = path.to_complex(chi), path.to_complex(einv)
    Mo = oracle.pair_densities(dataclasses.replace(p, gsph=gaug), *o, *e, 0, nk)
    Mo[:, 0] = head.head_density(p, *o, *e, 0, nk, qhat)
    wo = metal.weights_metal(p.kmesh, p.iq, E, None, *o, *e, 0, nk, p.freq_eV, p.delta_eV, ef)
    chi_o = oracle.chi0(Mo, wo)
    wq_o = float(qhat @ drude.plasma_tensor(p, 0, 6, ef) @ qhat)
    _, einv_o = drude.drude_head(p.lat, gaug, chi_o, p.freq_eV, p.delta_eV, wq_o, np.linalg.inv)
    e_chi = max(_rel(got_chi[f], chi_o[f]) for f in range(nf))
    e_inv = max(_rel(got[f], einv_o[f]) for f in range(nf))
    print(f"[drude] metal head chain: wq {wq:.4f} eV^2, chi rel {e_chi:.1e}, eps^-1 rel {e_inv:.1e}", flush=True)
    assert wq > 0 and abs(wq - wq_o * HA * HA) < 1e-10 * wq
    assert e_chi < 1e-10 and e_inv < 1e-10
    assert np.all(got[0, 0, :] == 0) and np.all(got[0, :, 0] == 0)     # w = 0 with delta > 0: infinite head
