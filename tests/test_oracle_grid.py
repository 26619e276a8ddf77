"""Pins of the frequency-grid oracle (oracle/grid.py, Eq. grid): the four
boundary conditions the paper states, monotonicity, the defaults, and the
library's host routine against the oracle."""

import math

import numpy as np
import pytest

from oracle import grid


@pytest.mark.parametrize("emax,dw,nomega,nmax", [(30.0, 0.05, 70, None), (12.5, 0.05, 70, None),
                                                  (30.0, 0.2, 40, 30), (2.0, 0.05, 70, None)])
def test_boundary_conditions(emax, dw, nomega, nmax):
    w = grid.frequency_grid(emax, dw, nomega, nmax)
    nm = (9 * nomega) // 10 if nmax is None else nmax
    assert w.shape == (nomega,)
    assert w[0] == 0.0                                          # (i)
    assert abs(w[1] - dw) < 1e-12 * dw                          # (ii)
    assert abs(w[nm - 1] - emax) < 1e-11 * emax                 # (iii)
    assert abs(w[-1] - 3 * emax) < 1e-12 * emax                 # (iv)
    assert np.all(np.diff(w) > 0)
    # the first branch is geometric: successive spacings share one ratio s
    d = np.diff(w[:nm])
    s = grid.solve_s(emax, dw, nm)
    assert np.allclose(d[1:] / d[:-1], s, rtol=1e-9, atol=0)
    # the second branch is geometric with ratio 3^(1/(N_Omega - N_max))
    tail = w[nm - 1:]
    assert np.allclose(tail[1:] / tail[:-1], 3 ** (1 / (nomega - nm)), rtol=1e-12, atol=0)


def test_defaults_and_the_printed_sign():
    """N_Omega = 70, N_max = 63 by default; the equation as printed (with +)
    has no root s > 1 (its left side exceeds 1 for every s > 1), so condition
    (iii) fixes the sign."""
    w = grid.frequency_grid(30.0)
    assert len(w) == 70 and abs(w[62] - 30.0) < 1e-10
    r = 30.0 / 0.05
    for s in (1.0001, 1.01, 1.1, 2.0):
        assert s ** 62 + r * (s - 1) > 1


def test_equal_spacing_limit():
    """E_max / d_omega = N_max - 1: s = 1 and the first branch is linear."""
    w = grid.frequency_grid(3.1, 0.05, 70, 63)
    assert np.allclose(w[:63], 0.05 * np.arange(63), rtol=0, atol=1e-12)


def test_library_routine_matches_the_oracle():
    """rp_frequency_grid is host code: the library's grid against the
    oracle's, element by element, and its argument checks."""
    import paper_2001_02351_amd as rp
    for emax, dw, nomega, nmax in ((30.0, 0.05, 70, 0), (12.5, 0.05, 70, 0), (30.0, 0.2, 40, 30),
                                   (2.0, 0.05, 70, 0), (3.1, 0.05, 70, 63)):
        got = rp.rp_frequency_grid(emax, dw, nomega, nmax)
        want = grid.frequency_grid(emax, dw, nomega, nmax or None)
        assert np.max(np.abs(got - want)) <= 1e-12 * want.max(), (emax, dw, nomega, nmax)
    for bad in ((0.0, 0.05, 70, 0), (30.0, -0.1, 70, 0), (30.0, 0.05, 2, 0), (30.0, 0.05, 70, 70),
                (30.0, 0.05, 70, 1), (math.nan, 0.05, 70, 0)):
        with pytest.raises(rp.RpError):
            rp.rp_frequency_grid(*bad)
