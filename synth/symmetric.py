"""A synthetic crystal with a space-group symmetry, for the symmetry
unfolding of wave functions and of eps^-1.

Input generation only: a simple cubic cell, the four operations of a 4_1
screw axis along z (x -> W x + t in fractional coordinates), a local
potential averaged over them (so that V(W x + t) = V(x)), and the band data
of the plane-wave Hamiltonian H_GG'(k) = |k+G|^2/2 delta_GG' + V(G - G')
diagonalized independently at every point of the k mesh.  The bands at k
and at a symmetry image of k are then related by the operation (up to
phases within degenerate multiplets), which is what the unfolding must
reproduce.  The band cut between occupied and empty bands, and the last
band kept, sit at gaps of the whole mesh.
"""

from __future__ import annotations

import math
from dataclasses import replace

import numpy as np

from .gen import HARTREE_EV, Problem, mesh_fractions, qpoint_gvectors

# 4_1 screw along z: (x, y, z) -> (-y, x, z + 1/4), and its powers
_W1 = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.int64)
_T1 = np.array([0.0, 0.0, 0.25])


def screw_ops():
    """[(W, t)] for g^0 .. g^3 of the 4_1 screw, t reduced to [0, 1)."""
    ops = []
    W, t = np.eye(3, dtype=np.int64), np.zeros(3)
    for _ in range(4):
        ops.append((W.copy(), np.mod(t, 1.0)))
        W, t = _W1 @ W, _W1 @ t + _T1
    return ops


def _sphere(kfrac, rec, gmax):
    span = int(math.ceil(gmax / np.linalg.norm(rec, axis=1).min())) + 2
    ax = np.arange(-span, span + 1)
    m = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    kv = (m + kfrac) @ rec
    d2 = np.einsum("ij,ij->i", kv, kv)
    keep = d2 <= gmax * gmax * (1 + 1e-12)
    m, d2 = m[keep], d2[keep]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], np.round(d2 * 1e9)))
    return np.ascontiguousarray(m[order].astype(np.int32))


def _potential(ops, rng, nterm=6, vmax=2, amp=0.6):
    """Fourier coefficients {m: V_m} (hartree) of a real potential averaged
    over the operations: f(x) = sum_m f_m e^{2 pi i m.x} (f_{-m} = conj f_m),
    V(x) = (1/|ops|) sum_g f(W_g x + t_g), whose coefficient at W_g^T m is
    f_m e^{2 pi i m.t_g}."""
    f = {}
    for _ in range(nterm):
        m = tuple(int(x) for x in rng.integers(-vmax, vmax + 1, 3))
        if m == (0, 0, 0) or m in f:
            continue
        c = amp * (rng.standard_normal() + 1j * rng.standard_normal()) / math.sqrt(2)
        f[m] = c
        f[tuple(-x for x in m)] = np.conj(c)
    V = {}
    for m, c in f.items():
        for W, t in ops:
            mp = tuple(int(x) for x in W.T @ np.array(m))
            V[mp] = V.get(mp, 0.0) + c * np.exp(2j * math.pi * np.dot(m, t)) / len(ops)
    return V


def symmetric_problem(a_bohr=7.26, fft=(12, 12, 12), kmesh=(4, 4, 2), iq=(1, 0, 0), gpsi=2.2, nocc_min=3,
                      nband_min=9, ng=25, freq_eV=(0.0, 4.0, 12.0), delta_eV=0.1, seed=7, min_gap_eV=0.02):
    """(Problem on the full mesh with directly diagonalized bands, ops).
    nocc and nband are the first cuts at or above nocc_min / nband_min whose
    gap exceeds min_gap_eV at every k."""
    rng = np.random.default_rng(seed)
    ops = screw_ops()
    lat = np.eye(3) * a_bohr
    rec = 2.0 * math.pi * np.linalg.inv(lat).T
    V = _potential(ops, rng)
    kf = mesh_fractions(kmesh)
    spheres = [_sphere(k, rec, gpsi) for k in kf]
    npw = np.array([s.shape[0] for s in spheres], np.int32)
    nmax_pw = int(npw.max())
    evals, evecs = [], []
    for k, s in zip(kf, spheres):
        kv = (s + k) @ rec
        H = np.diag(0.5 * np.einsum("ij,ij->i", kv, kv)).astype(np.complex128)
        for i in range(len(s)):
            for j in range(len(s)):
                d = tuple(int(x) for x in s[i] - s[j])
                if d in V:
                    H[i, j] += V[d]
        e, u = np.linalg.eigh(H)
        evals.append(e)
        evecs.append(u)
    nmin = int(npw.min())
    E = np.stack([e[:nmin] for e in evals]) * HARTREE_EV

    def cut(lo):
        for c in range(lo, nmin - 1):
            if np.min(E[:, c] - E[:, c - 1]) > min_gap_eV:
                return c
        raise ValueError("no band gap across the mesh")

    nocc = cut(nocc_min)
    nband = cut(max(nband_min, nocc + 2))
    miller = np.zeros((len(kf), nmax_pw, 3), np.int32)
    coef = np.zeros((len(kf), nband, nmax_pw), np.complex128)
    for i, (s, u) in enumerate(zip(spheres, evecs)):
        miller[i, : len(s)] = s
        coef[i, :, : len(s)] = u[:, :nband].T
    gsph, gtail = qpoint_gvectors(lat, kmesh, iq, ng, gpsi)
    prob = Problem(name="screw41", lat=lat, fft=tuple(fft), kmesh=tuple(kmesh), iq=tuple(iq), nocc=nocc,
                   nemp=nband - nocc, npw=npw, miller=miller, coef=coef,
                   energy_eV=np.ascontiguousarray(E[:, :nband]), gsph=gsph, gtail=gtail,
                   freq_eV=np.asarray(freq_eV, np.complex128), delta_eV=float(delta_eV), gpsi=float(gpsi), seed=seed)
    return prob, ops


def mesh_index(kfrac, kmesh) -> int:
    n = [int(round(k * K)) % K for k, K in zip(kfrac, kmesh)]
    return (n[0] * kmesh[1] + n[1]) * kmesh[2] + n[2]


def star_table(kmesh, ops):
    """For every mesh point k: (irreducible representative k*, op index g,
    integer rewind Delta) with k = S_g k* + Delta, S_g = W_g^{-T}; the
    representative of an orbit is its lowest mesh index."""
    kf = mesh_fractions(kmesh)
    table = [None] * len(kf)
    for i, k in enumerate(kf):
        if table[i] is not None:
            continue
        for g, (W, _) in enumerate(ops):
            S = np.rint(np.linalg.inv(W).T).astype(np.int64)
            kk = S @ k
            j = mesh_index(kk, kmesh)
            if table[j] is None:
                delta = np.rint(kf[j] - kk).astype(np.int64)
                table[j] = (i, g, delta)
    return table


def with_gvectors(prob, iq):
    """The problem at another q-point of its mesh (its own G lists)."""
    gsph, gtail = qpoint_gvectors(prob.lat, prob.kmesh, iq, int(prob.gsph.shape[0]), prob.gpsi)
    return replace(prob, iq=tuple(int(x) for x in iq), gsph=gsph, gtail=gtail)
