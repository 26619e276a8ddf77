"""GPU parity of the metallic tetrahedron weights (RP_W_TETRA_METAL: the
Fermi level cuts the tetrahedra) against the oracle (oracle/metal.py), and
chi of a metal with overlapping occupied and empty band ranges."""

import math

import numpy as np
import pytest

import oracle
from oracle import metal

torch = pytest.importorskip("torch")


def _rel(a, b):
    """The larger of the relative Frobenius norm of a - b and the largest
    element-wise deviation over the largest |b|."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    return max(np.linalg.norm(d) / np.linalg.norm(b), d.max() / np.abs(b).max())
pytestmark = pytest.mark.gpu


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


def _bands(kmesh, nband, seed=0):
    """Cosine bands with random centres and widths; several cross E_F = 0."""
    rng = np.random.default_rng(seed)
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in kmesh], indexing="ij"), -1).reshape(-1, 3)
    c = np.sort(rng.uniform(-3.0, 3.0, nband))
    t = rng.uniform(0.5, 1.5, (nband, 3))
    return np.stack([c[n] - np.sum(t[n] * np.cos(2 * math.pi * kf + n), axis=1) for n in range(nband)], 1)


def _weights(rp, ctx, kmesh, iq, E, o, e, freq, delta, mode):
    nk = int(np.prod(kmesh))
    cell = rp.make_cell(np.eye(3) * 7.0, (8, 8, 8), kmesh)
    npair = nk * (e[1] - e[0]) * (o[1] - o[0])
    w = torch.empty((len(freq), npair, 2), dtype=torch.float64, device="cuda")
    Ed = torch.from_numpy(np.ascontiguousarray(E)).cuda()
    rp.rp_weights(ctx, cell, iq, E.shape[1], Ed, None, *o, *e, 0, nk, len(freq), freq, delta, mode, w)
    rp.rp_synchronize(ctx)
    a = w.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


@pytest.mark.parametrize("imag", [False, True])
def test_metal_weights_match_oracle(rp, ctx, imag):
    kmesh, iq = (3, 3, 2), (1, 0, 1)
    E = _bands(kmesh, 5)
    ef = 0.1
    freq = 1j * np.array([0.0, 0.8, 4.0]) if imag else np.array([0.0, 1.5, 6.0])
    delta = 0.0 if imag else 0.1
    o, e = (0, 3), (1, 4)          # overlapping ranges: bands 1 and 2 can be either
    rp.rp_set_fermi_level(ctx, ef)
    got = _weights(rp, ctx, kmesh, iq, E, o, e, freq, delta, rp.RP_W_TETRA_METAL)
    want = metal.weights_metal(kmesh, iq, E, None, *o, *e, 0, 18, freq, delta, ef)
    err = np.max(np.abs(got - want)) / np.abs(want).max()
    cut = np.mean(np.abs(want) > 0)
    print(f"[metal] imag={imag}: max |diff| / max = {err:.1e}; nonzero weights {cut:.2f}", flush=True)
    assert err < 1e-11
    assert 0.1 < cut < 0.95      # the Fermi level bites: some pairs vanish, some do not


def test_metal_mode_in_a_gap_is_the_insulating_mode(rp, ctx):
    kmesh, iq = (3, 2, 2), (1, 1, 0)
    rng = np.random.default_rng(1)
    E = np.concatenate([np.sort(rng.uniform(-6, -1, (12, 2)), 1), np.sort(rng.uniform(1, 9, (12, 3)), 1)], 1)
    freq = np.array([0.0, 2.5])
    rp.rp_set_fermi_level(ctx, 0.0)
    a = _weights(rp, ctx, kmesh, iq, E, (0, 2), (2, 5), freq, 0.1, rp.RP_W_TETRA_METAL)
    b = _weights(rp, ctx, kmesh, iq, E, (0, 2), (2, 5), freq, 0.1, rp.RP_W_TETRA)
    assert np.array_equal(a, b)


def test_metal_chi_matches_oracle(rp, ctx):
    """chi (FP64) of a metal: pair densities of synthetic wave functions,
    metallic band energies, overlapping band ranges."""
    from paper_2001_02351_amd import path
    from synth import make_problem
    import dataclasses
    p = make_problem(name="metal", a_bohr=7.26, fft=(12, 12, 12), kmesh=(2, 2, 2), iq=(1, 0, 0), nocc=3, nemp=3,
                     gpsi=2.2, ng=27, freq_eV=np.array([0.0, 3.0]), delta_eV=0.1, seed=17)
    E = _bands(p.kmesh, 6, seed=4)
    p = dataclasses.replace(p, energy_eV=np.ascontiguousarray(E))
    ef = 0.2
    o, e = (0, 4), (2, 6)
    d = path.DeviceInputs(p)
    rp.rp_set_fermi_level(ctx, ef)
    M = path.pair_density(ctx, d, 0, p.nk, o=o, e=e, prec=rp.RP_FP64)
    chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device="cuda")
    rp.rp_chi0_accumulate(ctx, d.cell, p.iq, d.nband, d.energy, d.T, *o, *e, 0, p.nk, d.ng, M, d.nfreq,
                          p.freq_eV, p.delta_eV, rp.RP_W_TETRA_METAL, rp.RP_FP64, 0, chi)
    rp.rp_synchronize(ctx)
    got = path.to_complex(chi)
    Mo = oracle.pair_densities(p, *o, *e, 0, p.nk)
    wo = metal.weights_metal(p.kmesh, p.iq, E, None, *o, *e, 0, p.nk, p.freq_eV, p.delta_eV, ef)
    want = oracle.chi0(Mo, wo)
    err = max(_rel(got[f], want[f]) for f in range(d.nfreq))
    print(f"[metal] chi rel {err:.1e}", flush=True)
    assert err < 1e-10


def test_metal_mode_needs_a_fermi_level(rp, ctx):
    rp.rp_set_fermi_level(ctx, float("nan"))
    with pytest.raises(rp.RpError) as e:
        _weights(rp, ctx, (2, 2, 2), (1, 0, 0), _bands((2, 2, 2), 3), (0, 2), (1, 3), np.array([1.0]), 0.1,
                 rp.RP_W_TETRA_METAL)
    assert e.value.status == 3
