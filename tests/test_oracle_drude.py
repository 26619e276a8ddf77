"""Pins of the intraband (Drude) oracle (oracle/drude.py; Eqs. eps00, plasma,
momentum): the Fermi-surface corner weights against the derivative of the
occupied corner integrals of the metal oracle's clipping (convex hulls), the
mesh sum against the derivative of the occupied fraction, the free-electron
gas (Omega = 4 pi n), single plane waves, the cRPA and gap limits, and the
Drude dielectric function."""

import math

import numpy as np
import pytest

from oracle import drude, metal

HA = drude.HARTREE_EV


def _occupied_corner_integrals(e, E):
    """O_v(E) = (1/|T|) int_T lambda_v theta(E - e) from the metal oracle's
    tiling of {e < E} (an always-empty upper band)."""
    big = np.full(4, abs(np.asarray(e)).max() + abs(E) + 1.0)
    kind, tets = metal.region_tetrahedra(e, big, E)
    if kind == "full":
        return np.full(4, 0.25)
    if kind == "empty":
        return np.zeros(4)
    return sum(ratio * P.mean(axis=0) for P, ratio in tets)


@pytest.mark.parametrize("seed", range(6))
def test_section_weights_are_the_derivative_of_the_occupied_integrals(seed):
    rng = np.random.default_rng(seed)
    e = rng.uniform(-1.0, 1.0, 4)
    s = np.sort(e)
    h = 1e-6
    for E in (0.5 * (s[0] + s[1]), 0.3 * s[1] + 0.7 * s[2], 0.5 * (s[2] + s[3])):   # the three cases
        fd = (_occupied_corner_integrals(e, E + h) - _occupied_corner_integrals(e, E - h)) / (2 * h)
        got = drude.section_weights(e, E)
        assert np.max(np.abs(got - fd)) < 1e-6 * max(1.0, np.abs(fd).max()), (E, got, fd)
    assert np.all(drude.section_weights(e, s[0] - 0.1) == 0.0)
    assert np.all(drude.section_weights(e, s[3] + 0.1) == 0.0)


def test_mesh_weights_sum_to_the_density_of_states():
    """sum_k D(k) = d/dE_F of the occupied fraction (metal oracle), for a
    cosine band on a 4 x 3 x 3 mesh."""
    kmesh = (4, 3, 3)
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in kmesh], indexing="ij"), -1).reshape(-1, 3)
    band = 0.4 - np.sum(np.array([0.7, 1.1, 0.9]) * np.cos(2 * math.pi * kf + 0.3), axis=1)
    for EF in (-0.5, 0.2, 0.9):
        D = drude.fermi_weights(kmesh, band, EF)
        h = 1e-5
        fd = (metal.occupied_fraction(kmesh, band, EF + h) - metal.occupied_fraction(kmesh, band, EF - h)) / (2 * h)
        assert abs(D.sum() / HA - fd) < 1e-6 * fd, (EF, D.sum() / HA, fd)   # D per hartree, fd per eV


def test_free_electron_gas():
    """A free-electron band E = |k|^2/2 with the Fermi sphere inside the zone:
    Omega^{mu nu} -> 4 pi n delta_mu_nu as the mesh is refined (the linear
    tetrahedra around the cells' (1,1,1) diagonals leave equal off-diagonal
    terms of the same order as the diagonal error)."""
    a = 10.0
    lat = np.eye(3) * a
    b = 2 * math.pi / a
    kF = 0.3 * b
    n = 2.0 * (4.0 * math.pi / 3.0) * kF ** 3 / (2 * math.pi) ** 3
    want = 4.0 * math.pi * n
    errs = []
    for K in (8, 16):
        kf = np.stack(np.meshgrid(*[np.arange(K) / K] * 3, indexing="ij"), -1).reshape(-1, 3)
        kc = ((kf + 0.5) % 1.0 - 0.5) * b
        band = 0.5 * np.sum(kc * kc, axis=1) * HA
        D = drude.fermi_weights((K, K, K), band, 0.5 * kF * kF * HA)
        Om = drude.plasma_from(lat, kc[:, None, :], D[:, None]) / want
        print(f"[drude] free electrons {K}^3: diagonal {np.diag(Om)}, off-diagonal {Om[0, 1]:.2e}", flush=True)
        assert np.allclose(np.diag(Om), Om[0, 0], rtol=1e-12)          # the three axes alike
        errs.append(max(abs(Om[0, 0] - 1.0), abs(Om[0, 1])))
    assert errs[1] < 0.02 and errs[1] < 0.5 * errs[0], errs


def test_momentum_of_plane_waves():
    lat = np.diag([6.0, 7.0, 8.0])
    rec = 2 * math.pi * np.linalg.inv(lat).T
    k = np.array([0.25, -0.125, 0.5])
    miller = np.array([[0, 0, 0], [1, -2, 3], [-1, 0, 2]])
    coef = np.zeros((2, 3), np.complex128)
    coef[0, 1] = np.exp(0.7j)
    c = np.array([0.6, 0.8j])
    coef[1, [0, 2]] = c
    p = drude.momentum_diag(lat, k, miller, coef)
    assert np.allclose(p[0], (k + miller[1]) @ rec, atol=1e-14)
    assert np.allclose(p[1], 0.36 * (k @ rec) + 0.64 * ((k + miller[2]) @ rec), atol=1e-14)


def test_crpa_and_gap_limits():
    kmesh = (3, 3, 2)
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in kmesh], indexing="ij"), -1).reshape(-1, 3)
    band = -np.sum(np.cos(2 * math.pi * kf), axis=1)
    D = drude.fermi_weights(kmesh, band, 0.1)
    p = np.random.default_rng(3).normal(size=(kf.shape[0], 1, 3))
    lat = np.eye(3) * 7.0
    assert np.abs(drude.plasma_from(lat, p, D[:, None])).max() > 0
    assert np.all(drude.plasma_from(lat, p, D[:, None], T=np.ones((kf.shape[0], 1))) == 0.0)
    assert np.all(drude.fermi_weights(kmesh, band, 5.0) == 0.0)      # E_F above the band


def _inv(m):
    return np.linalg.inv(m)


def test_drude_dielectric_function():
    """With no interband chi the head is the Drude form: eps_M = 1/eps^-1_00 =
    1 - wq / (w (w + i delta)); the imaginary axis gives 1 + wq / (nu (nu +
    delta)); w = 0 gives a zero head row and column of eps^-1 and the body's
    inverse, which is the limit of small w."""
    lat = np.eye(3) * 7.0
    gsph = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0]])
    rng = np.random.default_rng(0)
    ng = len(gsph)
    wq = 0.04                                   # hartree^2
    freq = np.array([1.0, 3.0, 7.5])
    chi0 = np.zeros((3, ng, ng), np.complex128)
    _, einv = drude.drude_head(lat, gsph, chi0, freq, 0.1, wq, _inv)
    w = freq / HA
    dl = 0.1 / HA
    assert np.allclose(1.0 / einv[:, 0, 0], 1.0 - wq / (w * (w + 1j * dl)), rtol=1e-13)
    _, einv = drude.drude_head(lat, gsph, chi0[:2], 1j * np.array([0.5, 2.0]), 0.0, wq, _inv)
    nu = np.array([0.5, 2.0]) / HA
    assert np.allclose(1.0 / einv[:, 0, 0], 1.0 + wq / (nu * nu), rtol=1e-13)
    # a random interband chi: w -> 0 approaches the w = 0 limit
    a = rng.normal(size=(ng, ng)) + 1j * rng.normal(size=(ng, ng))
    chi = np.stack([-(a @ a.conj().T) * 0.01] * 2)
    eps, e0 = drude.drude_head(lat, gsph, chi, np.array([0.0, 1e-7]), 0.1, wq, _inv)
    assert np.isinf(eps[0, 0, 0].real)
    assert np.all(e0[0, 0, :] == 0) and np.all(e0[0, :, 0] == 0)
    assert np.allclose(e0[0, 1:, 1:], np.linalg.inv(eps[1, 1:, 1:]), rtol=1e-13)
    assert np.max(np.abs(e0[1] - e0[0])) < 1e-8
    # no intraband term: the head oracle's eps^-1
    from oracle import head
    _, ref = head.screen_head(lat, gsph, chi, _inv)
    _, got = drude.drude_head(lat, gsph, chi, np.array([0.0, 1e-7]), 0.1, 0.0, _inv)
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-15)
