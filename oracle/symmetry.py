"""Oracle for the symmetry unfolding of wave-function coefficients and of
G-indexed matrices such as eps^-1 (section "Symmetry", Eqs.
red-wavefunction, wavefunction, k-and-kirr, G-and-Girr, coef-G,
G-and-Gstar, symeps).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy.

Conventions.  An operation is x -> W x + t on fractional real-space
coordinates (W integer, t fractional); on fractional reciprocal coordinates
it acts as S = W^{-T}, so S^{-1} = W^T.  A reducible k is S k* + Delta
(Delta integer, the rewind vector); its plane-wave vectors are
G = S G* - Delta, so G* = S^{-1} (G + Delta) = W^T (m + Delta) for Miller
indices m, and (G + Delta) . T = 2 pi (m + Delta) . t.

Reading (also listed in the design notes): Eq. symeps prints the phase
e^{-i(G - G').T}.  With Eq. red-wavefunction's operator (psi_k(r) =
psi_k*(R^{-1}(r - T))) and Eq. chi's order M(G) conj(M(G')), the pair
densities at the image point pick up e^{+i(q + G).T} and chi (and eps^-1)
transform with e^{+i(G - G').T}; the pinned test that rotates a directly
computed chi(q*) onto chi(q) fixes this sign, and `unfold_matrix` takes it.
"""

from __future__ import annotations

import math

import numpy as np


def op_S(W) -> np.ndarray:
    """S = W^{-T} (integer)."""
    return np.rint(np.linalg.inv(np.asarray(W, np.float64)).T).astype(np.int64)


def rewind(W, kfrac_irr, kfrac) -> np.ndarray:
    """Delta = k - S k*, required to be an integer vector."""
    d = np.asarray(kfrac, np.float64) - op_S(W) @ np.asarray(kfrac_irr, np.float64)
    if np.max(np.abs(d - np.rint(d))) > 1e-9:
        raise ValueError("k is not the image of k* under the operation")
    return np.rint(d).astype(np.int64)


def unfold_coef(W, t, kfrac_irr, miller_irr, coef_irr, kfrac, miller) -> np.ndarray:
    """C_G(k) = C_{S^{-1}(G + Delta)}(k*) e^{-i (G + Delta).T} (Eq. coef-G in
    the S form) for the target Miller list `miller` at k; coef_irr [nband][npw*]
    on miller_irr.  A target vector whose source is missing is an error."""
    W = np.asarray(W, np.int64)
    delta = rewind(W, kfrac_irr, kfrac)
    where = {tuple(int(x) for x in m): i for i, m in enumerate(np.asarray(miller_irr).reshape(-1, 3))}
    m = np.asarray(miller, np.int64).reshape(-1, 3)
    src = (m + delta) @ W                      # rows: (W^T (m + Delta))^T
    idx = np.array([where[tuple(int(x) for x in s)] for s in src], np.int64)
    ph = np.exp(-2j * math.pi * ((m + delta) @ np.asarray(t, np.float64)))
    return np.asarray(coef_irr, np.complex128)[:, idx] * ph[None, :]


def unfold_matrix(W, t, qfrac_irr, gsph_irr, mat_irr, qfrac, gsph) -> np.ndarray:
    """X_{G,G'}(q) = X_{S^{-1}(G+Delta), S^{-1}(G'+Delta)}(q*) e^{+i(G - G').T}
    for X = chi or eps^-1 ([nfreq][ng*][ng*] on gsph_irr) onto the list gsph at
    q = S q* + Delta (the sign as pinned; see the module docstring)."""
    W = np.asarray(W, np.int64)
    delta = rewind(W, qfrac_irr, qfrac)
    where = {tuple(int(x) for x in m): i for i, m in enumerate(np.asarray(gsph_irr).reshape(-1, 3))}
    m = np.asarray(gsph, np.int64).reshape(-1, 3)
    src = (m + delta) @ W
    idx = np.array([where[tuple(int(x) for x in s)] for s in src], np.int64)
    ph = np.exp(2j * math.pi * (m @ np.asarray(t, np.float64)))
    X = np.asarray(mat_irr, np.complex128)[:, idx][:, :, idx]
    return X * ph[None, :, None] * ph.conj()[None, None, :]
