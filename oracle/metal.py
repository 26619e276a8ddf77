"""Oracle for the generalized-tetrahedron weights of a metal: the Fermi level
cuts the tetrahedra (section "Response function with random phase
approximation", Eqs. Xakqbk, tetrahedron; the generalized tetrahedron
technique the paper cites).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Python/numpy in FP64;
scipy's convex hull serves as a library step; the vertex integrals are the
pinned ones of the C oracle.

Reading (also listed in the design notes): for a pair of a band a at k+q and
a band b at k, the tetrahedron integral of Eq. tetrahedron runs over the
part of each tetrahedron where the linear interpolants satisfy
E_b(k) < E_F < E_a(k+q) (b occupied, a empty); with both conditions true at
all four corners this is the whole tetrahedron and the weight is the
insulating one.  On a region R of the tetrahedron T with k's vertex v:
  I_v^R(z) = (1/|T|) int_R lambda_v / (z - e) d^3k
           = sum over tetrahedra S tiling R of (|S|/|T|) sum_j lambda_v(s_j) I_j^S(z)
(s_j the corners of S, I_j^S the vertex integral of S on e(s_j)), since
lambda_v is linear.  The oracle finds R's vertices (points where three of
the six bounding planes meet and all constraints hold) and tiles R by a fan
from its centroid over the facets of its convex hull.
"""

from __future__ import annotations

import itertools

import numpy as np
from scipy.spatial import ConvexHull, QhullError

from . import vertex_integral

HARTREE_EV = 27.211386245988


def region_tetrahedra(Eb, Ea, EF):
    """Tetrahedra tiling {mu in T : mu.Eb < EF < mu.Ea} as barycentric corner
    matrices (4 x 4, rows = corners), with their volume ratios |S|/|T|.
    Returns ("full", None), ("empty", None) or ("cut", [(P, ratio), ...])."""
    Eb, Ea = np.asarray(Eb, np.float64), np.asarray(Ea, np.float64)
    if np.all(Eb < EF) and np.all(Ea > EF):
        return "full", None
    if np.all(Eb >= EF) or np.all(Ea <= EF):
        return "empty", None
    # y = (mu_1, mu_2, mu_3), mu_0 = 1 - sum(y); constraints A y <= c
    A = np.array([[-1, 0, 0], [0, -1, 0], [0, 0, -1], [1, 1, 1],
                  Eb[1:] - Eb[0], -(Ea[1:] - Ea[0])], np.float64)
    c = np.array([0, 0, 0, 1, EF - Eb[0], Ea[0] - EF], np.float64)
    scale = max(1.0, np.abs(np.concatenate([Eb, Ea])).max(), abs(EF))
    verts = []
    for tri in itertools.combinations(range(6), 3):
        M = A[list(tri)]
        if abs(np.linalg.det(M)) < 1e-14 * max(1.0, np.abs(M).max()) ** 3:
            continue
        y = np.linalg.solve(M, c[list(tri)])
        if np.all(A @ y <= c + 1e-12 * scale):
            if not any(np.max(np.abs(y - v)) < 1e-12 for v in verts):
                verts.append(y)
    if len(verts) < 4:
        return "empty", None
    V = np.array(verts)
    try:
        hull = ConvexHull(V)
    except QhullError:
        return "empty", None                  # flat: no volume
    cen = V.mean(axis=0)
    out = []
    for tri in hull.simplices:
        Y = np.vstack([cen, V[tri]])
        ratio = abs(np.linalg.det(Y[1:] - Y[0]))   # |S| / |T| (|T| = 1/6 in y)
        if ratio == 0.0:
            continue
        P = np.column_stack([1.0 - Y.sum(axis=1), Y])
        out.append((P, ratio))
    return "cut", out


def clipped_vertex_integral(z: complex, e, Eb, Ea, EF: float, v: int) -> complex:
    """I_v^R(z) of the transition energies e (corner values, hartree) over
    R = {E_b < E_F < E_a} within the tetrahedron."""
    kind, tets = region_tetrahedra(Eb, Ea, EF)
    e = np.asarray(e, np.float64)
    if kind == "full":
        return vertex_integral(z, e, v)
    if kind == "empty":
        return 0.0
    s = 0.0
    for P, ratio in tets:
        eS = P @ e
        for j in range(4):
            if P[j, v] != 0.0:
                s += ratio * P[j, v] * vertex_integral(z, eS, j)
    return s


def _tetrahedra():
    """The 6 tetrahedra of a mesh cell around its (0,0,0)-(1,1,1) diagonal:
    corner paths that raise one axis at a time, for every axis order."""
    out = []
    for perm in itertools.permutations(range(3)):
        cr = [np.zeros(3, int)]
        for a in perm:
            nxt = cr[-1].copy()
            nxt[a] = 1
            cr.append(nxt)
        out.append(np.array(cr))
    return out


def weights_metal(kmesh, iq, energy_eV, T, o0, o1, e0, e1, k0, k1, freq_eV, delta_eV, EF_eV):
    """w[f][p] = (2/Nk)(1 - T T) x_p(omega_f) for the pairs (k, a, b) (b
    fastest) with x = (1/6) sum over the 24 tetrahedra around k of
    [I_v^R(z) + I_v^R(z')], z = omega + i delta, z' = -omega + i delta."""
    kmesh = np.asarray(kmesh, int)
    iq = np.asarray(iq, int)
    E = np.asarray(energy_eV, np.float64) / HARTREE_EV
    EF = EF_eV / HARTREE_EV
    nk = int(np.prod(kmesh))
    freq = np.asarray(freq_eV, np.complex128) / HARTREE_EV
    dl = delta_eV / HARTREE_EV
    nO, nE = o1 - o0, e1 - e0
    npair = (k1 - k0) * nE * nO
    w = np.zeros((len(freq), npair), np.complex128)
    tets = _tetrahedra()

    def idx(m):
        r = np.mod(m, kmesh)
        return (r[0] * kmesh[1] + r[1]) * kmesh[2] + r[2]

    for p in range(npair):
        b = o0 + p % nO
        a = e0 + (p // nO) % nE
        k = k0 + p // (nO * nE)
        n = np.array([k // (kmesh[1] * kmesh[2]), (k // kmesh[2]) % kmesh[1], k % kmesh[2]])
        corners = []
        for s in range(8):
            off = np.array([(s >> 2) & 1, (s >> 1) & 1, s & 1])
            for cr in tets:
                hit = np.where(np.all(cr == off, axis=1))[0]
                if len(hit) == 0:
                    continue
                m = n - off + cr
                Eb = np.array([E[idx(mm), b] for mm in m])
                Ea = np.array([E[idx(mm + iq), a] for mm in m])
                corners.append((Eb, Ea, int(hit[0])))
        kq = idx(n + iq)
        fac = 1.0 if T is None else 1.0 - T[kq, a] * T[k, b]
        for f, om in enumerate(freq):
            z, zp = om + 1j * dl, -om + 1j * dl
            x = sum(clipped_vertex_integral(z, Ea - Eb, Eb, Ea, EF, v) + clipped_vertex_integral(zp, Ea - Eb, Eb, Ea, EF, v)
                    for Eb, Ea, v in corners)
            w[f, p] = (2.0 / nk) * fac * x / 6.0
    return w


def occupied_fraction(kmesh, band_eV, EF_eV) -> float:
    """Fraction of the Brillouin zone where the linear interpolant of one band
    lies below E_F: sum over the 6 N_k tetrahedra of |T cap {E < E_F}| / |T|,
    divided by 6 N_k (the same clipping with an always-empty upper band)."""
    kmesh = np.asarray(kmesh, int)
    E = np.asarray(band_eV, np.float64)
    big = np.full(4, np.abs(E).max() + abs(EF_eV) + 1.0)
    tot = 0.0
    for n in np.ndindex(*kmesh):
        for cr in _tetrahedra():
            m = np.array(n) + cr
            r = np.mod(m, kmesh)
            Eb = E[(r[:, 0] * kmesh[1] + r[:, 1]) * kmesh[2] + r[:, 2]]
            kind, parts = region_tetrahedra(Eb, big, EF_eV)
            if kind == "full":
                tot += 1.0
            elif kind == "cut":
                tot += sum(ratio for _, ratio in parts)
    return tot / (6 * int(np.prod(kmesh)))
