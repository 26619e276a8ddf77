"""The q -> 0 head, wings and optics on the GPU against the oracle
(oracle/head.py): head densities, chi with the head row and column, eps^-1
with head and wings, and eps_M, EELS, conductivity and reflectance.
FP64 to 1e-10 (head densities 1e-12), split-BF16 chi and eps^-1 to 1e-5; the
optical quantities (functions of the single element eps^-1_00) per quantity
relative to the magnitude of what it is made of, to the same bars.
"""

import copy

import numpy as np
import pytest

import oracle
from oracle import head as ohead
from synth import make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

QHAT = (0.6, -0.48, 0.64)


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
    c = rp.Context(0, tuning=None)
    yield c
    c.close()


def _problem(imag):
    freq = 1j * np.array([0.0, 0.5, 3.0]) if imag else np.array([0.0, 2.0, 7.5, 15.0])
    return make_problem(name="q0", a_bohr=7.26, fft=(16, 16, 16), kmesh=(2, 2, 2), iq=(0, 0, 0), nocc=4,
                        nemp=12, gpsi=2.4, ng=40, freq_eV=freq, delta_eV=0.0 if imag else 0.1, seed=31)


def _oracle(p):
    q = copy.copy(p)
    gaug = np.concatenate([np.zeros((1, 3), np.int32), p.gsph]).astype(np.int32)
    q.gsph = gaug
    M = oracle.pair_densities(q, 0, p.nocc, p.nocc, p.nband, 0, p.nk)
    h = ohead.head_density(p, 0, p.nocc, p.nocc, p.nband, 0, p.nk, QHAT)
    M[:, 0] = h
    w = oracle.prob_weights(p, 0, p.nocc, p.nocc, p.nband, 0, p.nk)
    chi = oracle.chi0(M, w)
    _, einv = ohead.screen_head(p.lat, gaug, chi, oracle.invert)
    return dict(h=h, chi=chi, einv=einv, optics=ohead.optics(einv[:, 0, 0], p.freq_eV))


@pytest.mark.parametrize("imag", [False, True])
def test_head_chain_matches_oracle(ctx, rp, imag):
    from paper_2001_02351_amd import path
    p = _problem(imag)
    ref = _oracle(p)
    d = path.DeviceInputs(p)
    for prec, tol in ((rp.RP_FP64, 1e-10), (rp.RP_SPLIT_BF16, 1e-5)):
        chi, gaug = path.chi0_head(ctx, d, QHAT, prec=prec, kbatch=3)
        einv, opt = path.screen_head(ctx, d, chi, gaug)
        rp.rp_synchronize(ctx)
        c, e = path.to_complex(chi), path.to_complex(einv)
        o = opt.cpu().numpy()
        e_chi = max(_rel(c[f], ref["chi"][f]) for f in range(d.nfreq))
        e_inv = max(_rel(e[f], ref["einv"][f]) for f in range(d.nfreq))
        want = np.stack([ref["optics"]["eps_M"].real, ref["optics"]["eps_M"].imag, ref["optics"]["eels"],
                         ref["optics"]["sigma"], ref["optics"]["refl"]], axis=1)
        # per quantity, relative to the largest magnitude of what it is made
        # of: |eps_M| for eps_M, |eps^-1_00| for L, (|w|/4 pi)|eps_M| for sigma
        # (which vanishes with w on the imaginary axis), R for R; parts that are
        # zero up to rounding (Im eps_M on the imaginary axis) are so measured
        em = np.abs(ref["optics"]["eps_M"]).max()
        w = np.abs(np.real(p.freq_eV)) / ohead.HARTREE_EV
        ssc = (w / (4 * np.pi) * np.abs(ref["optics"]["eps_M"])).max()
        scale = np.array([em, em, np.abs(ref["einv"][:, 0, 0]).max(), ssc if ssc > 0 else 1.0,
                          np.abs(want[:, 4]).max()])
        e_opt = np.max(np.abs(o - want).max(axis=0) / scale)
        print(f"[head] imag={imag} prec={prec}: chi {e_chi:.1e}, eps^-1 {e_inv:.1e}, optics {e_opt:.1e}",
              flush=True)
        assert e_chi < tol and e_inv < tol and e_opt < tol
        if imag:      # static screening on the imaginary axis: eps_M >= 1
            assert np.all(o[:, 0] >= 1.0)


def test_head_density_matches_oracle(ctx, rp):
    from paper_2001_02351_amd import path
    p = _problem(False)
    d = path.DeviceInputs(p)
    h = ohead.head_density(p, 1, 3, 5, 13, 2, 7, QHAT)
    ng = 5
    M = torch.zeros((len(h), ng, 2), dtype=torch.float64, device="cuda")
    rp.rp_head_density(ctx, d.cell, d.nband, p.miller.shape[1], p.npw, d.miller, d.coef, d.energy, 1, 3, 5, 13,
                       2, 7, QHAT, ng, 3, M)
    got = path.to_complex(M)
    assert np.max(np.abs(got[:, 3] - h)) < 1e-12 * np.abs(h).max()
    assert np.all(got[:, [0, 1, 2, 4]] == 0)       # only column col is written


def test_head_abi_errors(ctx, rp):
    from paper_2001_02351_amd import path
    p = _problem(False)
    d = path.DeviceInputs(p)
    M = torch.zeros((4, 5, 2), dtype=torch.float64, device="cuda")
    args = (ctx, d.cell, d.nband, p.miller.shape[1], p.npw, d.miller, d.coef, d.energy, 0, 1, 4, 8, 0, 1)
    with pytest.raises(rp.RpError) as e:
        rp.rp_head_density(*args, (0.0, 0.0, 0.0), 5, 0, M)
    assert e.value.status == 3
    with pytest.raises(rp.RpError) as e:
        rp.rp_head_density(*args, QHAT, 5, 5, M)
    assert e.value.status == 2
    chi = torch.zeros((1, 2, 2, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(rp.RpError) as e:
        rp.rp_screen_head(ctx, d.cell, 2, np.array([[1, 0, 0], [0, 0, 0]], np.int32), 1, [0.0], chi, None, None)
    assert e.value.status == 3
