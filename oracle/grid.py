"""Oracle for the logarithmic frequency grid of the polarization function
(section "Frequency grid", Eq. grid).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain Python/numpy in
FP64; scipy's bracketing root finder serves as a library step.

Reading (also listed in the design notes): the paper states four boundary
conditions, omega_1 = 0, omega_2 = d_omega, omega_{N_max} = E_max and
omega_{N_Omega} = 3 E_max, and prints the equation for s as
s^{N_max - 1} + (E_max / d_omega)(s - 1) = 1.  With the first branch of Eq.
grid, condition (iii) reads (d_omega / (s - 1))(s^{N_max - 1} - 1) = E_max,
i.e. s^{N_max - 1} - (E_max / d_omega)(s - 1) = 1: the printed "+" is read as
"-" (with "+" there is no root s > 0 other than the trivial s = 1 when
E_max > 0).  s = 1 always solves that equation and is excluded; the grid
needs the other root.  The second branch starts at i = N_max + 1.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import optimize


def solve_s(emax: float, dw: float, nmax: int) -> float:
    """The root s != 1 of s^(nmax-1) - (emax/dw)(s - 1) - 1 = 0."""
    r = emax / dw
    n = nmax - 1
    if abs(r - n) < 1e-12 * max(1.0, r):
        return 1.0                       # equal spacing: the limit s -> 1

    def f(s):
        return s ** n - r * (s - 1.0) - 1.0

    if r > n:                            # the grid spacing grows: s > 1
        lo, hi = 1.0 + 1e-12, 2.0
        while f(hi) <= 0.0:
            hi *= 2.0
        # move lo off the trivial root: f < 0 just above 1 when r > n
        lo = 1.0 + 1e-9
        while f(lo) >= 0.0:
            lo = 1.0 + (lo - 1.0) * 10.0
        return optimize.brentq(f, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    if r <= 1.0:
        raise ValueError("E_max must exceed d_omega")
    lo, hi = 0.0, 1.0 - 1e-9             # r < n: s in (0, 1); f(0) = r - 1 > 0, f < 0 just below 1
    while f(hi) >= 0.0:
        hi = 1.0 - (1.0 - hi) / 10.0
    return optimize.brentq(f, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)


def frequency_grid(emax: float, dw: float = 0.05, nomega: int = 70, nmax: int | None = None) -> np.ndarray:
    """omega_i, i = 1 .. N_Omega (eV), by the two branches of Eq. grid:
    (dw / (s - 1)) (exp((i - 1) ln s) - 1) up to N_max, then
    E_max exp(ln 3 (i - N_max) / (N_Omega - N_max)).  Default N_max = 9 N_Omega / 10
    (integer division)."""
    if nmax is None:
        nmax = (9 * nomega) // 10
    s = solve_s(emax, dw, nmax)
    out = np.empty(nomega)
    for i in range(1, nomega + 1):
        if i <= nmax:
            out[i - 1] = dw * (i - 1) if s == 1.0 else dw / (s - 1.0) * (math.exp((i - 1) * math.log(s)) - 1.0)
        else:
            out[i - 1] = emax * math.exp(math.log(3.0) * (i - nmax) / (nomega - nmax))
    return out
