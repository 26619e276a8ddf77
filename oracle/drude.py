"""Oracle for the intraband (Drude) term of the q -> 0 head (section "Response
function with random phase approximation", Eqs. eps00, plasma, momentum).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Python/numpy in FP64.

Readings (also listed in the design notes):

* Eq. plasma prints the Fermi-surface sum without the Coulomb and spin
  factors of the intraband term.  The term that enters Eq. eps00 is taken as
      Omega^{mu nu} = (4 pi / Omega) (2 / N_k) sum_k sum_a (1 - T_ak^2)
                      p^mu_aak p^nu_aak delta(E_ak - E_F)
  in hartree^2 (atomic units; the 2 is the spin sum that Eq. chi's weights
  carry), and its projection on the direction of q replaces the square of
  the printed plasma frequency:
      eps_00(w) -> eps_00(w) - qhat.Omega.qhat / (w (w + i delta)).
  A free-electron gas gives Omega^{xx} = 4 pi n.
* The Fermi-surface delta is integrated with the linear tetrahedra of the
  weights (6 per mesh cell around its (0,0,0)-(1,1,1) diagonal):
      (1/N_k) sum_k f(k) delta(E_k - E_F) = sum_k f(k) D(k),
      D(k) = (1/(6 N_k)) sum over the 24 tetrahedra T around k of D_v^T,
  with D_v^T = (1/|T|) int_T lambda_v delta(e - E_F) d^3k for k's corner v
  and the linear interpolant e.  On a plane section of T the delta turns a
  volume integral into a surface integral: int_T f delta(e - E) dV =
  int_{e = E} f dA / |grad e|.
* Where w (w + i delta) = 0 (w = 0 with or without broadening, or nu = 0 on
  the imaginary axis) the term is infinite: eps^-1 then has a zero head row
  and column and its body is the inverse of eps's body (the limit of the
  Schur complement as eps_00 grows without bound).
"""

from __future__ import annotations

import math

import numpy as np

from . import head as _head
from .metal import _tetrahedra

HARTREE_EV = 27.211386245988

# corners of the reference tetrahedron in y-space: V0 = 0, V1..V3 unit vectors
_CORNERS = np.vstack([np.zeros(3), np.eye(3)])


def _lambda(y) -> np.ndarray:
    """Barycentric coordinates (lambda_0..lambda_3) of a point y."""
    y = np.asarray(y, np.float64)
    return np.array([1.0 - y.sum(), y[0], y[1], y[2]])


def section_weights(e, E) -> np.ndarray:
    """D_v = (1/|T|) int_T lambda_v delta(e(k) - E) d^3k, v = 0..3, for the
    linear interpolant of the corner energies e (hartree), per unit energy.
    The section {e = E} is a triangle or a quadrilateral whose corners lie on
    the edges that E separates; it is fanned into triangles, over each of
    which the mean of the linear lambda_v is the mean of its corner values."""
    e = np.asarray(e, np.float64)
    grad = e[1:] - e[0]                       # e(y) = e0 + grad . y
    gn = np.linalg.norm(grad)
    if gn == 0.0:
        return np.zeros(4)
    pts = []
    for i in range(4):
        for j in range(i + 1, 4):
            if (e[i] - E) * (e[j] - E) < 0.0:
                t = (E - e[i]) / (e[j] - e[i])
                pts.append(_CORNERS[i] + t * (_CORNERS[j] - _CORNERS[i]))
    if len(pts) < 3:
        return np.zeros(4)
    P = np.array(pts)
    c = P.mean(axis=0)
    # order the section's corners by angle in its plane (normal = grad)
    n = grad / gn
    u = P[0] - c
    u /= np.linalg.norm(u)
    v = np.cross(n, u)
    ang = np.arctan2((P - c) @ v, (P - c) @ u)
    P = P[np.argsort(ang)]
    D = np.zeros(4)
    for k in range(1, len(P) - 1):
        tri = (P[0], P[k], P[k + 1])
        area = 0.5 * np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0]))
        D += area * np.mean([_lambda(p) for p in tri], axis=0)
    return 6.0 * D / gn                       # |T| = 1/6 in y-space


def fermi_weights(kmesh, band_eV, EF_eV) -> np.ndarray:
    """D(k) (1/hartree) of one band on the Gamma-centred mesh, k in C order,
    so that sum_k f(k) D(k) = (1/N_k) sum_k f(k) delta(E_k - E_F)."""
    kmesh = np.asarray(kmesh, int)
    nk = int(np.prod(kmesh))
    E = np.asarray(band_eV, np.float64) / HARTREE_EV
    EF = EF_eV / HARTREE_EV
    D = np.zeros(nk)

    def idx(m):
        r = np.mod(m, kmesh)
        return (r[0] * kmesh[1] + r[1]) * kmesh[2] + r[2]

    for n in np.ndindex(*kmesh):
        for cr in _tetrahedra():
            m = np.array(n) + cr
            ks = [idx(mm) for mm in m]
            w = section_weights(E[ks], EF)
            for v in range(4):
                D[ks[v]] += w[v]
    return D / (6.0 * nk)


def momentum_diag(lat, kfrac, miller, coef) -> np.ndarray:
    """p[a][mu] = <psi_a| -i grad |psi_a> = sum_G |C_Ga|^2 (k + G)_mu
    (Eq. momentum, local part), Cartesian, bohr^-1."""
    p = _head.momentum_k(_head.reciprocal(lat), kfrac, miller, coef, coef)
    return np.real(np.einsum("maa->am", p))


def plasma_from(lat, p, D, T=None) -> np.ndarray:
    """Omega^{mu nu} (hartree^2) from p[k][a][mu], D[k][a] (1/hartree) and T[k][a]."""
    p = np.asarray(p, np.float64)
    D = np.asarray(D, np.float64)
    fac = 1.0 if T is None else 1.0 - np.asarray(T, np.float64) ** 2
    vol = abs(np.linalg.det(np.asarray(lat, np.float64)))
    return (4.0 * math.pi / vol) * 2.0 * np.einsum("ka,kam,kan->mn", fac * D, p, p)


def plasma_tensor(prob, b0, b1, EF_eV, T=None) -> np.ndarray:
    """Omega^{mu nu} (hartree^2) of bands [b0, b1) of a plane-wave problem."""
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in prob.kmesh], indexing="ij"), -1).reshape(-1, 3)
    p = np.stack([momentum_diag(prob.lat, kf[k], prob.miller[k, :prob.npw[k]], prob.coef[k, b0:b1, :prob.npw[k]])
                  for k in range(prob.nk)])
    D = np.stack([fermi_weights(prob.kmesh, prob.energy_eV[:, b], EF_eV) for b in range(b0, b1)], axis=1)
    Tb = None if T is None else np.asarray(T)[:, b0:b1]
    return plasma_from(prob.lat, p, D, Tb)


def drude_head(lat, gsph, chi, freq_eV, delta_eV, wq, invert) -> tuple:
    """eps and eps^-1 at q -> 0 with the intraband term wq = qhat.Omega.qhat
    (hartree^2) subtracted from the head: eps_00 -= wq / (w (w + i delta)),
    w = freq / hartree (complex; i nu on the imaginary axis).  Where
    w (w + i delta) = 0 the head is infinite: eps^-1 is returned with a zero
    head row and column and the inverse of eps's body, and eps with its head
    set to inf."""
    vs = _head.vsqrt_head(lat, gsph)
    chi = np.asarray(chi, np.complex128)
    eps = np.eye(chi.shape[1])[None] - vs[None, :, None] * chi * vs[None, None, :]
    w = np.asarray(freq_eV, np.complex128) / HARTREE_EV
    dl = delta_eV / HARTREE_EV
    einv = np.empty_like(eps)
    for f in range(eps.shape[0]):
        den = w[f] * (w[f] + 1j * dl)
        if den == 0.0 and wq != 0.0:
            einv[f] = 0.0
            einv[f, 1:, 1:] = invert(eps[f, 1:, 1:])
            eps[f, 0, 0] = np.inf
        else:
            eps[f, 0, 0] -= wq / den if wq != 0.0 else 0.0
            einv[f] = invert(eps[f])
    return eps, einv
