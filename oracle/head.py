"""Oracle for the q -> 0 head and wings of the dielectric matrix and the
optical quantities derived from it (section "Response function with random
phase approximation", Eqs. eps00, eps00-cRPA, momentum, epsilonM, eels,
optical-conductivity, reflectance).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in FP64,
each function the definition it names.

Readings (also listed in the design notes):
* Head density.  For q -> 0 the G = 0 pair density of an empty band a and an
  occupied band b at the same k is, to first order in q (k.p perturbation of
  the periodic parts), M_ab(q, 0) = q . p_ab(k) / (E_a(k) - E_b(k)) with the
  transition moment p_ab = <psi_a| -i grad |psi_b> of Eq. momentum (the
  non-local pseudopotential term dropped, as the paper does).  The head
  density is h_ab = qhat . p_ab / (E_a - E_b): M(q, 0) / |q|.
* Head and wings of eps.  With h in place of the G = 0 pair density, the
  contraction of Eq. chi gives chi~_00 = lim chi_00 / q^2 and
  chi~_0G = lim chi_0G / q, and eps = 1 - v^1/2 chi v^1/2 keeps its form with
  v^1/2_0 = sqrt(4 pi / Omega) (the factors of q cancel).  This is Eq.
  eps00-cRPA with "d^2 chi_00 / dq^2" read as the coefficient of q^2 in
  chi_00 (the limit chi_00 / q^2).  No intraband (Drude) term: the synthetic
  spectra are gapped, so the plasma frequency of Eq. plasma is zero.
* Reflectance.  Eq. reflectance prints the modulus of the Fresnel amplitude
  (1 - sqrt(eps^-1_00)) / (1 + sqrt(eps^-1_00)) = (sqrt(eps_M) - 1) /
  (sqrt(eps_M) + 1); the reflectance is its squared modulus.
"""

from __future__ import annotations

import math

import numpy as np

HARTREE_EV = 27.211386245988


def reciprocal(lat) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(np.asarray(lat, np.float64)).T


def momentum_k(rec, kfrac, miller, coef_a, coef_b) -> np.ndarray:
    """p[mu][a][b] = sum_G conj(C_Ga) (k + G)_mu C_Gb (Cartesian, bohr^-1):
    <psi_a| -i grad |psi_b> for plane-wave expansions sharing one G list
    (Eq. momentum without the non-local term)."""
    kg = (np.asarray(kfrac, np.float64)[None, :] + np.asarray(miller, np.float64)) @ rec
    ca = np.asarray(coef_a, np.complex128)
    cb = np.asarray(coef_b, np.complex128)
    return np.stack([(ca.conj() * kg[None, :, mu]) @ cb.T for mu in range(3)])


def head_density(prob, o0, o1, e0, e1, k0, k1, qhat) -> np.ndarray:
    """h[(k, a, b)] = qhat . p_ab(k) / (E_a(k) - E_b(k)) (energies in
    hartree) for occupied b in [o0, o1), empty a in [e0, e1), k in [k0, k1);
    the pair layout of the pair densities (b fastest).  Where the band ranges
    overlap (a metal), the intraband pairs a = b get h = 0: at q -> 0 they
    belong to the intraband (Drude) term of Eq. eps00, not to the head
    density."""
    rec = reciprocal(prob.lat)
    qhat = np.asarray(qhat, np.float64)
    qhat = qhat / np.linalg.norm(qhat)
    kmesh = np.asarray(prob.kmesh)
    out = np.empty((k1 - k0, e1 - e0, o1 - o0), np.complex128)
    for k in range(k0, k1):
        n = int(prob.npw[k])
        idx = np.array([k // (kmesh[1] * kmesh[2]), (k // kmesh[2]) % kmesh[1], k % kmesh[2]])
        kfrac = idx / kmesh
        p = momentum_k(rec, kfrac, prob.miller[k, :n], prob.coef[k, e0:e1, :n], prob.coef[k, o0:o1, :n])
        pq = np.tensordot(qhat, p, axes=(0, 0))            # [a][b]
        de = (prob.energy_eV[k, e0:e1][:, None] - prob.energy_eV[k, o0:o1][None, :]) / HARTREE_EV
        same = (np.arange(e0, e1)[:, None] == np.arange(o0, o1)[None, :])
        out[k - k0] = np.where(same, 0.0, pq / np.where(same, 1.0, de))
    return out.reshape(-1)


def vsqrt_head(lat, gsph) -> np.ndarray:
    """sqrt(4 pi / Omega) / |G| for G != 0 and sqrt(4 pi / Omega) for G = 0
    (q -> 0 with the q factors of the head and wings taken out)."""
    lat = np.asarray(lat, np.float64)
    omega = abs(np.linalg.det(lat))
    g = np.asarray(gsph, np.float64) @ reciprocal(lat)
    n = np.linalg.norm(g, axis=1)
    v = np.full(n.shape, math.sqrt(4.0 * math.pi / omega))
    nz = n > 0
    v[nz] /= n[nz]
    return v


def screen_head(lat, gsph, chi, invert) -> tuple:
    """eps = I - v^1/2 chi v^1/2 at q -> 0 (gsph[0] = G = 0, chi with the head
    density in its G = 0 row and column) and eps^-1 by `invert` (the oracle's
    Gauss-Jordan inverse)."""
    gsph = np.asarray(gsph)
    if np.any(gsph[0] != 0) or np.any(np.all(gsph[1:] == 0, axis=1)):
        raise ValueError("gsph must hold G = 0 first and only there")
    vs = vsqrt_head(lat, gsph)
    chi = np.asarray(chi, np.complex128)
    eps = np.eye(chi.shape[1])[None] - vs[None, :, None] * chi * vs[None, None, :]
    einv = np.stack([invert(e) for e in eps])
    return eps, einv


def optics(einv00, freq_eV) -> dict:
    """Eqs. epsilonM, eels, optical-conductivity, reflectance from eps^-1_00:
    eps_M = 1/eps^-1_00, L = -Im eps^-1_00, Re sigma = (w/4 pi) Im eps_M (w in
    hartree, sigma in atomic units), R = |(sqrt(eps_M) - 1)/(sqrt(eps_M) + 1)|^2
    (principal square root)."""
    einv00 = np.asarray(einv00, np.complex128)
    w = np.real(np.asarray(freq_eV, np.complex128)) / HARTREE_EV
    eps_m = 1.0 / einv00
    s = np.sqrt(eps_m)
    return dict(eps_M=eps_m, eels=-einv00.imag, sigma=w / (4.0 * math.pi) * eps_m.imag,
                refl=np.abs((s - 1.0) / (s + 1.0)) ** 2)
