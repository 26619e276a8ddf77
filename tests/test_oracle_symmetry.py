"""Pins of the symmetry-unfolding oracle (oracle/symmetry.py; Eqs.
red-wavefunction, k-and-kirr, G-and-Girr, coef-G, symeps) on a synthetic
crystal that has the symmetry: a local potential averaged over the four
operations of a 4_1 screw axis, its bands diagonalized independently at
every k of the mesh (synth/symmetric.py)."""

import dataclasses

import numpy as np
import pytest

import oracle
from oracle import symmetry as osym
from synth.gen import mesh_fractions
from synth.symmetric import star_table, symmetric_problem, with_gvectors


@pytest.fixture(scope="module")
def model():
    p, ops = symmetric_problem()
    return p, ops, star_table(p.kmesh, ops), mesh_fractions(p.kmesh)


def _chi(p):
    nb = p.nocc + p.nemp
    M = oracle.pair_densities(p, 0, p.nocc, p.nocc, nb, 0, p.nk)
    w = oracle.prob_weights(p, 0, p.nocc, p.nocc, nb, 0, p.nk, mode=1)
    return oracle.chi0(M, w)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_model_has_the_symmetry(model):
    """Energies at every mesh point equal those at its irreducible
    representative; the orbit table covers the mesh with integer rewinds."""
    p, ops, tab, kf = model
    assert len({i for i, _, _ in tab}) < p.nk          # some points are images
    for k, (i, g, d) in enumerate(tab):
        S = osym.op_S(ops[g][0])
        assert np.allclose(kf[k], S @ kf[i] + d, atol=1e-12)
        assert np.max(np.abs(p.energy_eV[k] - p.energy_eV[i])) < 1e-11


def test_unfolded_bands_reproduce_chi(model):
    """Coefficients unfolded from the irreducible points (Eq. coef-G) give the
    same chi as the bands diagonalized at every k (gauge-invariant), at two
    q-points."""
    p, ops, tab, kf = model
    coef = np.zeros_like(p.coef)
    energy = np.empty_like(p.energy_eV)
    for k, (i, g, d) in enumerate(tab):
        W, t = ops[g]
        n, ni = int(p.npw[k]), int(p.npw[i])
        coef[k, :, :n] = osym.unfold_coef(W, t, kf[i], p.miller[i, :ni], p.coef[i, :, :ni], kf[k], p.miller[k, :n])
        energy[k] = p.energy_eV[i]
    pu = dataclasses.replace(p, coef=coef, energy_eV=energy)
    assert not np.allclose(coef, p.coef)               # a different gauge ...
    for iq in ((1, 0, 0), (1, 2, 1)):
        a, b = _chi(with_gvectors(pu, iq)), _chi(with_gvectors(p, iq))
        assert _rel(a, b) < 1e-10, iq                  # ... the same chi


def test_chi_rotation_sign(model):
    """chi at q = S q* + Delta computed from the bands equals chi(q*) moved
    by Eq. symeps onto the rotated G list, with the phase e^{+i(G - G').T}
    that Eq. chi's M conj(M) order and Eq. red-wavefunction's operator give;
    the printed e^{-i(G - G').T} fails for the quarter turns of the 4_1
    screw (t = 1/4)."""
    p, ops, _, _ = model
    qs = np.array([1, 0, 1])
    qf = qs / np.array(p.kmesh)
    ps = with_gvectors(p, tuple(qs))
    chis = _chi(ps)
    for W, t in ops:
        S = osym.op_S(W)
        iq = tuple(int(round(x * K)) % K for x, K in zip(S @ qf, p.kmesh))
        qg = np.array(iq) / np.array(p.kmesh)
        d = osym.rewind(W, qf, qg)
        pg = dataclasses.replace(with_gvectors(p, iq), gsph=np.ascontiguousarray((ps.gsph @ S.T - d).astype(np.int32)))
        direct = _chi(pg)
        assert _rel(osym.unfold_matrix(W, t, qf, ps.gsph, chis, qg, pg.gsph), direct) < 1e-10
        printed = osym.unfold_matrix(W, -np.asarray(t), qf, ps.gsph, chis, qg, pg.gsph)
        if abs(t[2] % 0.5) > 1e-12:
            assert _rel(printed, direct) > 1e-2


def test_unfolding_composes(model):
    """Unfolding by g1 and then by g2 equals unfolding by g2 o g1 =
    (W2 W1, W2 t1 + t2) up to one global phase per band."""
    p, ops, _, kf = model
    k0 = 5
    n0 = int(p.npw[k0])
    (W1, t1), (W2, t2) = ops[1], ops[3]
    S1, S2 = osym.op_S(W1), osym.op_S(W2)
    k1 = np.mod(S1 @ kf[k0], 1.0)
    m1 = (p.miller[k0, :n0] @ S1.T - osym.rewind(W1, kf[k0], k1)).astype(np.int64)
    c1 = osym.unfold_coef(W1, t1, kf[k0], p.miller[k0, :n0], p.coef[k0, :, :n0], k1, m1)
    k2 = np.mod(S2 @ k1, 1.0)
    m2 = (m1 @ S2.T - osym.rewind(W2, k1, k2)).astype(np.int64)
    two = osym.unfold_coef(W2, t2, k1, m1, c1, k2, m2)
    one = osym.unfold_coef(W2 @ W1, W2 @ t1 + t2, kf[k0], p.miller[k0, :n0], p.coef[k0, :, :n0], k2, m2)
    for b in range(one.shape[0]):
        ov = np.vdot(one[b], two[b])
        assert abs(abs(ov) - 1.0) < 1e-12
        assert np.max(np.abs(two[b] - ov * one[b])) < 1e-12
