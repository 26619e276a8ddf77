"""Pins of the oracle's q -> 0 head, wings and optics (oracle/head.py), each
against something other than the oracle itself:

* transition moments of two-plane-wave states (closed form),
* the k.p limit on true eigenstates of a model Hamiltonian (numpy eigh):
  <psi_a,k+q| e^{iq.r} |psi_b,k> / |q| -> qhat . p_ab / (E_a - E_b) (phase
  included, states at k+q in the gauge continuous with those at k),
* eps^-1_00 and eps_M against the Schur complement (numpy.linalg.solve),
* the optical formulas on a transparent and on an absorbing dielectric
  (textbook Fresnel reflectance, zero conductivity without absorption),
* the sign of the static head on the imaginary axis (eps_00 >= 1).
"""

import math

import numpy as np
import pytest

import oracle
from oracle import head


def _cell(a=7.26):
    return np.eye(3) * a


def test_momentum_of_two_plane_wave_states():
    lat = _cell()
    rec = head.reciprocal(lat)
    miller = np.array([[0, 0, 0], [1, -1, 2], [0, 2, 0]])
    kfrac = np.array([0.25, 0.0, 0.5])
    s = 1.0 / math.sqrt(2.0)
    ca = np.array([[s, s, 0.0]], complex)               # (G1 + G2)/sqrt2
    cb = np.array([[s, -s, 0.0], [0.0, 0.0, 1j]])        # (G1 - G2)/sqrt2, i G3
    p = head.momentum_k(rec, kfrac, miller, ca, cb)
    kg = (kfrac + miller) @ rec
    np.testing.assert_allclose(p[:, 0, 0], (kg[0] - kg[1]) / 2, atol=1e-15)
    np.testing.assert_allclose(p[:, 0, 1], 0.0, atol=1e-15)
    paa = head.momentum_k(rec, kfrac, miller, ca, ca)[:, 0, 0]
    np.testing.assert_allclose(paa, (kg[0] + kg[1]) / 2, atol=1e-15)


def test_head_density_is_the_kp_limit_on_model_eigenstates():
    """H_k = |k+G|^2/2 + V(G-G') on a small basis: the overlap of eigenstates
    at k+q and k (the G = 0 pair density) over |q| tends to the head density."""
    rng = np.random.default_rng(3)
    lat = _cell(6.0)
    rec = head.reciprocal(lat)
    r = 2
    ax = np.arange(-r, r + 1)
    miller = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    miller = miller[(miller ** 2).sum(1) <= 5]
    n = len(miller)
    vq = {}
    d = miller[:, None, :] - miller[None, :, :]
    V = np.zeros((n, n), complex)
    for i in range(n):
        for j in range(n):
            key = tuple(d[i, j])
            if key == (0, 0, 0) or sum(abs(x) for x in key) > 2:
                continue
            if key not in vq:
                v = 0.3 * (rng.standard_normal() + 1j * rng.standard_normal())
                vq[key], vq[tuple(-x for x in key)] = v, np.conj(v)
            V[i, j] = vq[key]

    def eig(kfrac):
        kg = (kfrac + miller) @ rec
        e, c = np.linalg.eigh(np.diag(0.5 * (kg ** 2).sum(1)) + V)
        return e, c.T                                    # rows = bands

    kfrac = np.array([0.13, 0.27, -0.08])
    qhat = np.array([0.6, -0.48, 0.64])
    e0, c0 = eig(kfrac)
    occ, emp = [0, 1], [4, 5, 6]
    p = head.momentum_k(rec, kfrac, miller, c0[emp], c0[occ])
    h = np.tensordot(qhat, p, axes=(0, 0)) / (e0[emp][:, None] - e0[occ][None, :])
    for qmag, tol in ((1e-4, 2e-3), (1e-5, 2e-4)):
        qfrac = qmag * qhat @ np.linalg.inv(rec)          # Cartesian q -> fractional
        _, cq = eig(kfrac + qfrac)
        # gauge of the states at k+q continuous with those at k
        ph = np.einsum("ag,ag->a", cq.conj(), c0)
        cq = cq * (ph / np.abs(ph))[:, None]
        ov = cq[emp].conj() @ c0[occ].T                   # <psi_a,k+q| e^{iqr} |psi_b,k>
        err = np.max(np.abs(ov / qmag - h) / np.abs(h).max())
        assert err < tol, (qmag, err)


def test_head_eps_inverse_is_the_schur_complement():
    rng = np.random.default_rng(5)
    lat = _cell()
    g = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0]])
    A = rng.standard_normal((5, 9)) + 1j * rng.standard_normal((5, 9))
    chi = -(A @ A.conj().T)[None] * 0.05
    eps, einv = head.screen_head(lat, g, chi, oracle.invert)
    vs = head.vsqrt_head(lat, g)
    assert vs[0] == pytest.approx(math.sqrt(4 * math.pi / abs(np.linalg.det(lat))), rel=1e-15)
    e = eps[0]
    schur = e[0, 0] - e[0, 1:] @ np.linalg.solve(e[1:, 1:], e[1:, 0])
    assert abs(1.0 / einv[0, 0, 0] - schur) < 1e-12 * abs(schur)
    # head only: eps_M = eps_00
    _, einv1 = head.screen_head(lat, g[:1], chi[:, :1, :1], oracle.invert)
    assert abs(1.0 / einv1[0, 0, 0] - eps[0, 0, 0]) < 1e-14
    with pytest.raises(ValueError):
        head.screen_head(lat, g[1:], chi[:, 1:, 1:], oracle.invert)


def test_optics_formulas():
    n = 2.5
    o = head.optics(np.array([1.0 / n ** 2]), np.array([1.0]))
    assert o["refl"][0] == pytest.approx(((n - 1) / (n + 1)) ** 2, rel=1e-14)
    assert o["sigma"][0] == 0.0 and o["eels"][0] == 0.0
    em = 3.0 + 2.0j
    w_ev = 5.0
    o = head.optics(np.array([1.0 / em]), np.array([w_ev]))
    N = np.sqrt(em)
    assert o["refl"][0] == pytest.approx(abs((N - 1) / (N + 1)) ** 2, rel=1e-14)
    assert o["sigma"][0] == pytest.approx(w_ev / head.HARTREE_EV / (4 * math.pi) * 2.0, rel=1e-14)
    assert o["eels"][0] == pytest.approx((1.0 / em).imag * -1.0, rel=1e-14)


def test_static_head_on_the_imaginary_axis_screens():
    """Real negative weights on the imaginary axis make chi~ negative
    semidefinite: eps_00 >= 1 and 0 < eps^-1_00 <= 1 (eps_M >= 1)."""
    from synth import make_problem
    p = make_problem(name="h", a_bohr=7.26, fft=(12, 12, 12), kmesh=(2, 2, 2), iq=(0, 0, 0), nocc=3,
                     nemp=5, gpsi=2.4, ng=14, freq_eV=1j * np.array([0.0, 1.0]), delta_eV=0.0, seed=9)
    h = head.head_density(p, 0, 3, 3, 8, 0, p.nk, (1.0, 0.0, 0.0))
    w = oracle.prob_weights(p, 0, 3, 3, 8, 0, p.nk)
    assert np.all(w.real < 0) and np.abs(w.imag).max() < 1e-11 * np.abs(w).max()
    M = oracle.pair_densities(p, 0, 3, 3, 8, 0, p.nk)
    Ma = np.concatenate([h[:, None], M], axis=1)
    chi = oracle.chi0(Ma, w.real.astype(complex))
    g = np.concatenate([[[0, 0, 0]], p.gsph])
    eps, einv = head.screen_head(p.lat, g, chi, oracle.invert)
    assert np.all(eps[:, 0, 0].real >= 1.0)
    assert np.all((einv[:, 0, 0].real > 0) & (einv[:, 0, 0].real <= 1.0 + 1e-14))
