"""Pins of the metallic tetrahedron oracle (oracle/metal.py): the insulating
limit, the half-filled cosine band, additivity of complementary regions, a
brute-force quadrature of the clipped vertex integral, and absorption."""

import math

import numpy as np
import pytest

import oracle
from oracle import metal

HA = metal.HARTREE_EV


def test_gap_gives_the_insulating_weights():
    """E_F in a gap of every k: the cut never bites, the weights equal the
    insulating oracle's (C)."""
    rng = np.random.default_rng(1)
    kmesh, iq = (3, 2, 2), (1, 1, 0)
    nk = 12
    E = np.concatenate([np.sort(rng.uniform(-6, -1, (nk, 2)), 1), np.sort(rng.uniform(1, 9, (nk, 3)), 1)], 1)
    freq = np.array([0.0, 2.5, 7.0])
    w0 = oracle.weights(kmesh, iq, E, None, 0, 2, 2, 5, 0, nk, freq, 0.1, 0)
    wm = metal.weights_metal(kmesh, iq, E, None, 0, 2, 2, 5, 0, nk, freq, 0.1, 0.0)
    assert np.max(np.abs(wm - w0)) < 1e-12 * np.abs(w0).max()


@pytest.mark.parametrize("kmesh", [(4, 4, 4), (6, 4, 2), (2, 2, 2)])
def test_half_filled_cosine_band(kmesh):
    """E(k) = -sum_a cos(2 pi k_a) at E_F = 0 on an even mesh: k -> k + (1/2,
    1/2, 1/2) maps the mesh onto itself and E onto -E, so the interpolated
    occupied fraction is exactly 1/2; it is 0 below the band and 1 above."""
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in kmesh], indexing="ij"), -1).reshape(-1, 3)
    E = -np.sum(np.cos(2 * math.pi * kf), axis=1)
    assert abs(metal.occupied_fraction(kmesh, E, 0.0) - 0.5) < 1e-13
    assert metal.occupied_fraction(kmesh, E, -3.5) == 0.0
    assert abs(metal.occupied_fraction(kmesh, E, 3.5) - 1.0) < 1e-13
    assert metal.occupied_fraction(kmesh, E, -0.4) < metal.occupied_fraction(kmesh, E, 0.3)


def test_complementary_regions_add_up():
    """For random cut tetrahedra: {Eb < EF < Ea} + {Eb > EF, Ea > EF} =
    {Ea > EF}, and {Ea > EF} + {Ea < EF} = the whole tetrahedron."""
    rng = np.random.default_rng(5)
    big = 1e3
    for _ in range(40):
        Eb, Ea = rng.uniform(-1, 1, 4), rng.uniform(-1, 1, 4) + 0.3
        EF = rng.uniform(-0.3, 0.6)
        e = rng.uniform(0.1, 1.0, 4)
        z = complex(rng.uniform(-1, 2), rng.uniform(0.01, 0.3))
        v = int(rng.integers(4))
        cut = metal.clipped_vertex_integral(z, e, Eb, Ea, EF, v)
        # reflecting an energy about E_F flips its constraint alone
        rest = metal.clipped_vertex_integral(z, e, 2 * EF - Eb, Ea, EF, v)          # Eb > EF < Ea
        upper = metal.clipped_vertex_integral(z, e, np.full(4, -big), Ea, EF, v)     # Ea > EF
        lower = metal.clipped_vertex_integral(z, e, np.full(4, -big), 2 * EF - Ea, EF, v)   # Ea < EF
        full = oracle.vertex_integral(z, e, v)
        assert abs(cut + rest - upper) < 1e-11 * abs(full)
        assert abs(upper + lower - full) < 1e-11 * abs(full)


def test_clipped_integral_brute_force():
    """(1/|T|) int_R lambda_v / (z - e) on a cut tetrahedron against a
    midpoint sum over a fine barycentric grid (indicator of R)."""
    rng = np.random.default_rng(9)
    n = 160
    g = (np.arange(n) + 0.5) / n
    Y = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    Y = Y[Y.sum(1) < 1.0]
    mu = np.column_stack([1 - Y.sum(1), Y])
    done = 0
    while done < 3:
        Eb, Ea = rng.uniform(-1, 1, 4), rng.uniform(-0.5, 1.5, 4)
        EF = 0.1
        e = rng.uniform(0.2, 1.5, 4)
        z = complex(0.7, 0.3)
        v = int(rng.integers(4))
        inside = (mu @ Eb < EF) & (mu @ Ea > EF)
        if not 0.05 < inside.mean() < 0.95:
            continue                                  # not a genuine cut: draw again
        done += 1
        brute = np.sum(np.where(inside, mu[:, v] / (z - mu @ e), 0.0)) / len(mu)
        got = metal.clipped_vertex_integral(z, e, Eb, Ea, EF, v)
        assert abs(got - brute) < 2e-2 * abs(brute)


def test_metal_absorbs():
    """A band crossing E_F on a 3x3x2 mesh: Im w < 0 for real omega > 0 and
    delta > 0 (absorption), intraband pairs (a = b) included."""
    kmesh, iq = (3, 3, 2), (1, 0, 0)
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in kmesh], indexing="ij"), -1).reshape(-1, 3)
    band = -np.sum(np.cos(2 * math.pi * kf), axis=1)
    E = np.column_stack([band - 4.0, band, band + 4.5])
    w = metal.weights_metal(kmesh, iq, E, None, 0, 2, 1, 3, 0, 18, np.array([0.5, 3.0]), 0.1, 0.2)
    assert np.all(w.imag < 0)
