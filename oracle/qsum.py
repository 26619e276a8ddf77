"""Oracle for the q-mesh sums of the interaction parameters: screened direct
U, bare direct V, screened exchange J and bare exchange X between Wannier
orbitals i in the home cell and j in cell R (section "Interaction
parameters", Eqs. W, Wq, matrix_U, rhoiqG, matrix_V, matrix_J, matrix_X).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in FP64;
numpy's FFT and scipy's adaptive quadrature serve as library steps.

Readings (also listed in the design notes):
* Orbitals.  phi_i is given on the real-space grid of one cell, folded into
  it, and stands for a function localized within half a cell of its centre
  c_i: phi_i0(r) = phi_i(r) where r is the image nearest c_i, else 0, and
  phi_jR(r) = phi_j0(r - R).
* Densities.  With the Bloch sums of the orbitals, the sum over k in Eq.
  rhoiqG and in the exchange density reduces to a real-space integral:
  rho_ijRq(G) = ntilde_ijR(q+G) / |q+G| with
  ntilde_ijR(Q) = int phi_i0(r) phi_jR(r) e^{iQ.r} dr, evaluated on the grid
  as (Omega/N_r) sum over the images rt of the grid points nearest the
  midpoint (c_i + c_j + R)/2.  The direct density is rho_iq = rho_ii0q (Eq.
  rhoiqG read with i on both sides).
* The bare exchange X sums over the same G set as the bare direct V (the
  eps sphere and the tail up to the wave-function cutoff), i.e. X is J with
  eps^-1 = delta as V is U with eps^-1 = delta.
* q = 0.  The G = 0 density diverges as 1/|q|.  Following the usual
  treatment of the Coulomb singularity (the prescription the paper cites), the
  q = 0 term of the mesh average (1/N_q) sum_q F(q) is replaced by the
  average of F over the q-cell around Gamma, with F ~ f(0)/|q|^2 there: the
  head term becomes A eps^-1_00 ntilde_a(0) conj(ntilde_b(0)) with
  A = (N_q Omega / (2 pi)^3) int_cell d^3q / |q|^2, the mean of 1/|q|^2 over
  the cell {sum_a x_a b_a / N_a : x in [-1/2, 1/2)^3}.  The wings (odd in q
  to leading order) average to zero and are dropped; the body G, G' != 0 is
  taken at q = 0 with the head-including eps^-1.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import integrate

HARTREE_EV = 27.211386245988


def reciprocal(lat) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(np.asarray(lat, np.float64)).T


def _inside(d) -> np.ndarray:
    """True where each fractional component lies in [-1/2, 1/2)."""
    return np.all((d >= -0.5) & (d < 0.5), axis=-1)


def exchange_ntilde(lat, fft, kmesh, iq, phi, centre_frac, R, glist) -> np.ndarray:
    """ntilde[r][i][j][g] = ntilde_ijR(q + G_g) for R = R[r] (integer lattice
    vectors), i, j over the orbitals: the transform of the overlap density
    phi_i0 phi_jR on the window of images nearest the pair's midpoint."""
    lat = np.asarray(lat, np.float64)
    N = np.asarray(fft, int)
    nr = int(np.prod(N))
    vol = abs(np.linalg.det(lat))
    qf = np.asarray(iq, np.float64) / np.asarray(kmesh, np.float64)
    phi = np.asarray(phi, np.float64).reshape(len(phi), nr)
    cen = np.asarray(centre_frac, np.float64)
    R = np.asarray(R, np.int64).reshape(-1, 3)
    glist = np.asarray(glist, np.int64).reshape(-1, 3)
    grid = np.stack(np.meshgrid(*[np.arange(n) / n for n in N], indexing="ij"), -1).reshape(nr, 3)
    nw = len(cen)
    out = np.empty((len(R), nw, nw, len(glist)), np.complex128)
    idx = tuple((glist % N).T)
    for r, Rv in enumerate(R):
        for i in range(nw):
            for j in range(nw):
                m = 0.5 * (cen[i] + cen[j] + Rv)
                d = grid - m
                d -= np.floor(d + 0.5)
                rt = m + d                                   # image nearest the midpoint
                w = np.where(_inside(rt - cen[i]) & _inside(rt - Rv - cen[j]), phi[i] * phi[j], 0.0)
                f = w * np.exp(2j * math.pi * (rt @ qf))     # e^{iq.rt}
                # sum_r f(r) e^{iG.r}: e^{iG.rt} = e^{iG.r} on grid points
                F = np.fft.ifftn(f.reshape(tuple(N))) * nr
                out[r, i, j] = F[idx] * (vol / nr)
    return out


def qg_norm(lat, kmesh, iq, glist) -> np.ndarray:
    """|q + G| in bohr^-1 for each G of glist."""
    qf = np.asarray(iq, np.float64) / np.asarray(kmesh, np.float64)
    Q = (qf[None, :] + np.asarray(glist, np.float64).reshape(-1, 3)) @ reciprocal(lat)
    return np.linalg.norm(Q, axis=1)


def cell_average(lat, kmesh) -> float:
    """A = (N_q Omega / (2 pi)^3) int_cell d^3q / |q|^2 over the cell spanned
    by b_a / N_a around Gamma.  The cell is cut into six pyramids with apex at
    Gamma, one per face; on the pyramid over a face at distance h from Gamma,
    q = t p (p on the face, t in [0, 1]) gives d^3q / |q|^2 = h dt dA / |p|^2,
    so each pyramid contributes h int_face dA / |p|^2 (adaptive 2-D
    quadrature)."""
    lat = np.asarray(lat, np.float64)
    nq = int(np.prod(kmesh))
    vol = abs(np.linalg.det(lat))
    e = reciprocal(lat) / np.asarray(kmesh, np.float64)[:, None]   # cell edges
    total = 0.0
    for a in range(3):
        u, v = e[(a + 1) % 3], e[(a + 2) % 3]
        n = np.cross(u, v)
        area = np.linalg.norm(n)
        n /= area
        for s in (0.5, -0.5):
            c = s * e[a]                                  # face centre
            h = abs(c @ n)

            def f(y, x, c=c, u=u, v=v):
                p = c + x * u + y * v
                return 1.0 / (p @ p)

            val, _ = integrate.dblquad(f, -0.5, 0.5, -0.5, 0.5, epsabs=1e-14, epsrel=1e-13)
            total += h * val * area
    return nq * vol / (2.0 * math.pi) ** 3 * total


def qterm(lat, kmesh, iq, n_u, n_x, ng, eps_inv, R, glist, head_avg=None) -> dict:
    """One q-point's term of Eqs. matrix_U, matrix_V, matrix_J, matrix_X (eV).

    n_u [nwan][nG], n_x [nR][nwan][nwan][nG]: ntilde of the direct and the
    exchange densities on glist, whose first ng entries index eps_inv
    ([nfreq][ng][ng]) and the rest form the bare tail.  At q = 0, glist[0]
    must be G = 0 and head_avg the cell average A; that entry then enters only
    through the head term.
      U[f][r][i][j] = e^{-iq.R} pre [ sum_{GG'} rho_i eps^-1 conj(rho_j) + tail + head ]
      V[r][i][j]    = e^{-iq.R} pre [ sum_G rho_i conj(rho_j) + head with eps^-1_00 = 1 ]
      J[f][r][i][j] = pre [ sum_{GG'} rho_v eps^-1 conj(rho_v) + tail + head ], v = (r, i, j)
      X[r][i][j]    = pre [ sum_G |rho_v|^2 + head with eps^-1_00 = 1 ]
    with pre = HA 4 pi / (Omega N_q) and rho = ntilde / |q + G|."""
    lat = np.asarray(lat, np.float64)
    glist = np.asarray(glist).reshape(-1, 3)
    nq = int(np.prod(kmesh))
    vol = abs(np.linalg.det(lat))
    pre = HARTREE_EV * 4.0 * math.pi / (vol * nq)
    qn = qg_norm(lat, kmesh, iq, glist)
    head = bool(np.all(np.asarray(iq) % np.asarray(kmesh) == 0))
    if head:
        if np.any(glist[0] != 0) or head_avg is None:
            raise ValueError("q = 0 needs G = 0 first in glist and the cell average")
    elif np.any(qn == 0):
        raise ValueError("|q + G| = 0 away from q = 0")
    inv = np.where(qn > 0, 1.0 / np.where(qn > 0, qn, 1.0), 0.0)
    ru = np.asarray(n_u, np.complex128) * inv            # G = 0 at q = 0 -> 0
    rx = np.asarray(n_x, np.complex128) * inv
    E = np.asarray(eps_inv, np.complex128)
    nf = E.shape[0]
    qf = np.asarray(iq, np.float64) / np.asarray(kmesh, np.float64)
    R = np.asarray(R, np.float64).reshape(-1, 3)
    phase = np.exp(-2j * math.pi * (R @ qf))             # e^{-iq.R}
    nw = ru.shape[0]
    re, rt = ru[:, :ng], ru[:, ng:]
    xe, xt = rx[..., :ng], rx[..., ng:]
    U = np.empty((nf, len(R), nw, nw), np.complex128)
    J = np.empty((nf, len(R), nw, nw), np.complex128)
    tail_u = rt @ rt.conj().T
    tail_x = np.sum(np.abs(xt) ** 2, axis=-1)
    bare_u = re @ re.conj().T + tail_u
    bare_x = np.sum(np.abs(xe) ** 2, axis=-1) + tail_x
    hu = np.zeros((nw, nw), np.complex128)
    hx = np.zeros(rx.shape[:3])
    if head:
        n0 = np.asarray(n_u, np.complex128)[:, 0]
        hu = head_avg * np.outer(n0, n0.conj())
        hx = head_avg * np.abs(np.asarray(n_x, np.complex128)[..., 0]) ** 2
    for f in range(nf):
        body_u = re @ E[f] @ re.conj().T
        sw_u = body_u + tail_u + E[f][0, 0] * hu
        # sum_{G,G'} rho_v(G) eps^-1_GG' conj(rho_v(G')) for every v, as one
        # matrix product over G' and a sum over G
        xv = xe.reshape(-1, ng)
        body_x = np.sum(xv.T * (E[f] @ xv.conj().T), axis=0).reshape(xe.shape[:3])
        sw_x = body_x + tail_x + E[f][0, 0] * hx
        for r in range(len(R)):
            U[f, r] = phase[r] * pre * sw_u
        J[f] = pre * sw_x
    V = pre * phase[:, None, None] * (bare_u + hu)[None]
    X = pre * (bare_x + hx).astype(np.complex128)
    return dict(U=U, V=V, J=J, X=X)
