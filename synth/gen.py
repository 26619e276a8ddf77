"""Seeded synthetic problems shaped like the paper's SrVO3 workload.

The paper's calculations (section "Typical outputs") use a simple cubic cell
with a = 3.8425 Angstrom, an 8x8x8 k mesh, a 100 Ry wavefunction cutoff and a
400 Ry density cutoff.  The DFT wavefunctions are not available, so the
arrays built here keep those shapes with random content:

* Bloch coefficients C_{G n}(k) of the plane-wave expansion (Eq. pak): per k a
  complex Gaussian [N_PW(k), n_band] block made orthonormal by Cholesky-QR
  applied twice (CholQR2), so that sum_G |C_{G n}|^2 = 1 for every band.
* Band energies: per k, sorted uniform draws in a valence window and a
  conduction window (a gapped spectrum).
* Plane-wave spheres S_psi(k) = {G : |k+G| <= G_psi} (Eq. pak cutoff) and the
  polarization sphere S_eps(q) = the first N_G vectors by |q+G|^2 (Eq. epsGG
  cutoff), ties broken by Miller index (m1, m2, m3) ascending.
* Wannier orbitals: normalized Gaussians exp(-alpha |r - R_i|^2) sampled on the
  real-space grid with the minimum-image convention around their centre.

Nothing in this module evaluates the method (no pair densities, weights,
polarization, dielectric matrix or projection).
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

HARTREE_EV = 27.211386245988      # CODATA 2018
BOHR_ANGSTROM = 0.529177210903    # CODATA 2018

A_SRVO3_BOHR = 3.8425 / BOHR_ANGSTROM  # paper's SrVO3 lattice constant


@dataclass
class Problem:
    """All host arrays of one q-point problem (C-contiguous numpy)."""

    name: str
    lat: np.ndarray            # [3,3] rows a1,a2,a3 in bohr
    fft: tuple                 # (N1,N2,N3) real-space grid
    kmesh: tuple               # (K1,K2,K3) Gamma-centred mesh, k = n/K
    iq: tuple                  # q = iq/K (mesh index)
    nocc: int
    nemp: int
    npw: np.ndarray            # int32 [Nk]
    miller: np.ndarray         # int32 [Nk, npw_max, 3] (rows beyond npw[k] are 0)
    coef: np.ndarray           # complex128 [Nk, nband, npw_max] (zero padded)
    energy_eV: np.ndarray      # float64 [Nk, nband]; bands 0..nocc-1 occupied
    gsph: np.ndarray           # int32 [ng,3]  Miller indices of S_eps(q)
    gtail: np.ndarray          # int32 [ntail,3] S_psi(q) \ S_eps(q)
    freq_eV: np.ndarray        # complex128 [nfreq] (real omega, or i*nu)
    delta_eV: float
    T: Optional[np.ndarray] = None        # float64 [Nk, nband] or None (RPA)
    phi: Optional[np.ndarray] = None      # float64 [nwan,N1,N2,N3]
    centre_frac: Optional[np.ndarray] = None  # float64 [nwan,3]
    alpha: Optional[np.ndarray] = None    # float64 [nwan] Gaussian exponents
    gpsi: float = 0.0                     # wavefunction sphere radius, 1/bohr
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def nk(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def nband(self) -> int:
        return self.nocc + self.nemp

    @property
    def npw_max(self) -> int:
        return int(self.miller.shape[1])

    @property
    def ng(self) -> int:
        return int(self.gsph.shape[0])

    @property
    def nfreq(self) -> int:
        return int(self.freq_eV.shape[0])

    @property
    def nwan(self) -> int:
        return 0 if self.phi is None else int(self.phi.shape[0])

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.lat)))

    def recip(self) -> np.ndarray:
        """Rows b1,b2,b3 with a_i . b_j = 2 pi delta_ij (1/bohr)."""
        return 2.0 * math.pi * np.linalg.inv(self.lat).T


def mesh_fractions(kmesh) -> np.ndarray:
    """Fractional k = n/K of the Gamma-centred mesh, n1 slowest (mesh order)."""
    k1, k2, k3 = kmesh
    n = np.stack(np.meshgrid(np.arange(k1), np.arange(k2), np.arange(k3),
                             indexing="ij"), axis=-1).reshape(-1, 3)
    return n / np.array(kmesh, dtype=np.float64)


def _sphere(recip: np.ndarray, kfrac: np.ndarray, gmax: Optional[float],
            count: Optional[int] = None) -> np.ndarray:
    """Miller indices with |k+G| <= gmax (or the first `count` by |k+G|),
    sorted by |k+G|^2, ties by (m1,m2,m3) ascending."""
    lens = np.linalg.norm(recip, axis=1)
    if count is not None:
        # radius that certainly contains `count` lattice points
        vol = abs(np.linalg.det(recip))
        r = (3.0 * count * vol / (4.0 * math.pi)) ** (1.0 / 3.0) + 2.0 * lens.max()
    else:
        r = gmax
    inv = np.linalg.inv(recip)
    span = np.ceil(r * np.linalg.norm(inv, axis=0)).astype(int) + 2
    axes = [np.arange(-s, s + 1) for s in span]
    m = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    kv = (m + kfrac[None, :]) @ recip
    d2 = np.einsum("ij,ij->i", kv, kv)
    # quantize the key so that symmetry-equivalent vectors tie exactly
    key = np.round(d2 * 1e9) / 1e9
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], key))
    m, d2 = m[order], d2[order]
    if count is not None:
        return np.ascontiguousarray(m[:count].astype(np.int32))
    return np.ascontiguousarray(m[d2 <= gmax * gmax * (1.0 + 1e-12)].astype(np.int32))


def _cholqr2(a: np.ndarray) -> np.ndarray:
    """Orthonormal columns spanning a (Cholesky-QR applied twice)."""
    for _ in range(2):
        s = a.conj().T @ a
        l = np.linalg.cholesky(s)
        a = a @ np.linalg.inv(l).conj().T
    return a


def _coef_block(args):
    seed_entropy, spawn_key, npw_k, nband = args
    ss = np.random.SeedSequence(entropy=seed_entropy, spawn_key=spawn_key)
    rng = np.random.default_rng(ss)
    a = (rng.standard_normal((npw_k, nband)) +
         1j * rng.standard_normal((npw_k, nband))) / math.sqrt(2.0)
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            q = _cholqr2(a)
    except ImportError:  # pragma: no cover
        q = _cholqr2(a)
    return np.ascontiguousarray(q.T)


def _gen_coefficients(coef_ss: np.random.SeedSequence, npw: np.ndarray,
                      nband: int, npw_max: int, workers: int) -> np.ndarray:
    nk = len(npw)
    children = coef_ss.spawn(nk)
    coef = np.zeros((nk, nband, npw_max), dtype=np.complex128)
    jobs = [(c.entropy, c.spawn_key, int(npw[i]), nband) for i, c in enumerate(children)]
    big = nk * nband * npw_max > 4_000_000
    if big and workers > 1:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
            for i, blk in enumerate(ex.map(_coef_block, jobs, chunksize=4)):
                coef[i, :, :blk.shape[1]] = blk
    else:
        for i, j in enumerate(jobs):
            blk = _coef_block(j)
            coef[i, :, :blk.shape[1]] = blk
    return coef


def _default_workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def gaussian_orbitals(lat: np.ndarray, fft, centre_frac: np.ndarray,
                      alpha: np.ndarray) -> np.ndarray:
    """phi_i(r_j) = exp(-alpha_i |r_j - R_i|^2), r_j - R_i taken as the
    minimum image (fractional difference wrapped to [-1/2, 1/2)), normalized
    so that (Omega/N_r) sum_j phi_i(r_j)^2 = 1."""
    n1, n2, n3 = fft
    vol = abs(np.linalg.det(lat))
    nr = n1 * n2 * n3
    f = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2,
                             np.arange(n3) / n3, indexing="ij"), axis=-1)
    out = np.empty((len(alpha), n1, n2, n3))
    for i in range(len(alpha)):
        d = f - centre_frac[i]
        d -= np.floor(d + 0.5)
        x = d @ lat
        p = np.exp(-alpha[i] * np.einsum("...i,...i->...", x, x))
        p /= math.sqrt(vol / nr * np.sum(p * p))
        out[i] = p
    return out


def qpoint_gvectors(lat, kmesh, iq, ng: int, gpsi: float):
    """(gsph, gtail) for q = iq/K: S_eps the first ng Miller indices by |q+G|
    (ties by (m1, m2, m3)), the tail those with |q+G| <= gpsi outside it.  At
    q = 0 the G = 0 vector has no Coulomb factor and is left out of both
    (S_eps then holds the ng shortest nonzero G)."""
    recip = 2.0 * math.pi * np.linalg.inv(np.asarray(lat, np.float64)).T
    qf = np.array(iq, dtype=np.float64) / np.array(kmesh, dtype=np.float64)
    gsph = _sphere(recip, qf, None, count=ng)
    full = _sphere(recip, qf, gpsi)
    in_eps = {tuple(m) for m in gsph.tolist()}
    gtail = np.array([m for m in full.tolist() if tuple(m) not in in_eps],
                     dtype=np.int32).reshape(-1, 3)
    if tuple(iq) == (0, 0, 0):
        gsph = _sphere(recip, qf, None, count=ng + 1)[1:]
        gtail = gtail[np.any(gtail != 0, axis=1)]
    return gsph, np.ascontiguousarray(gtail)


def at_qpoint(prob: "Problem", iq) -> "Problem":
    """The same system at another q-point of its mesh: the band data are
    shared, the G lists are those of q = iq/K (same N_G and wave-function
    cutoff)."""
    gsph, gtail = qpoint_gvectors(prob.lat, prob.kmesh, iq, int(prob.gsph.shape[0]), prob.gpsi)
    return replace(prob, iq=tuple(int(x) for x in iq), gsph=gsph, gtail=gtail)


def make_problem(*, name: str, a_bohr: float, fft, kmesh, iq, nocc: int, nemp: int,
                 gpsi: float, ng: int, freq_eV, delta_eV: float,
                 occ_window=(-8.0, -1.0), emp_window=(1.0, 20.0),
                 nwan: int = 0, alpha_range=(1.0, 2.0), crpa: bool = False,
                 seed: int = 0, workers: Optional[int] = None) -> Problem:
    """Build one cubic-cell problem from a seed (see module docstring)."""
    lat = np.eye(3) * a_bohr
    recip = 2.0 * math.pi * np.linalg.inv(lat).T
    kf = mesh_fractions(kmesh)
    nk = kf.shape[0]
    nband = nocc + nemp
    ss = np.random.SeedSequence(seed)
    coef_ss, en_ss, wan_ss = ss.spawn(3)

    spheres = [_sphere(recip, kf[i], gpsi) for i in range(nk)]
    npw = np.array([s.shape[0] for s in spheres], dtype=np.int32)
    npw_max = int(npw.max())
    if npw.min() < nband:
        raise ValueError("wavefunction sphere smaller than the band count")
    miller = np.zeros((nk, npw_max, 3), dtype=np.int32)
    for i, s in enumerate(spheres):
        miller[i, :s.shape[0]] = s
    coef = _gen_coefficients(coef_ss, npw, nband, npw_max,
                             workers if workers is not None else _default_workers())

    rng_e = np.random.default_rng(en_ss)
    energy = np.empty((nk, nband))
    for i in range(nk):
        energy[i, :nocc] = np.sort(rng_e.uniform(*occ_window, nocc))
        energy[i, nocc:] = np.sort(rng_e.uniform(*emp_window, nemp))

    gsph, gtail = qpoint_gvectors(lat, kmesh, iq, ng, gpsi)

    rng_w = np.random.default_rng(wan_ss)
    T = None
    if crpa:
        # transition probabilities sum_i |U_{n i}|^2 of a random 4x3 isometry
        # acting on the bands nocc-2 .. nocc+1 (Eq. tak form)
        T = np.zeros((nk, nband))
        for i in range(nk):
            u = rng_w.standard_normal((4, 3)) + 1j * rng_w.standard_normal((4, 3))
            u = _cholqr2(u)
            T[i, nocc - 2:nocc + 2] = np.sum(np.abs(u) ** 2, axis=1)
    phi = centre = alpha = None
    if nwan > 0:
        centre = rng_w.uniform(0.0, 1.0, (nwan, 3))
        alpha = rng_w.uniform(*alpha_range, nwan)
        phi = gaussian_orbitals(lat, fft, centre, alpha)

    return Problem(name=name, lat=lat, fft=tuple(int(x) for x in fft),
                   kmesh=tuple(int(x) for x in kmesh), iq=tuple(int(x) for x in iq),
                   nocc=nocc, nemp=nemp, npw=npw, miller=miller, coef=coef,
                   energy_eV=energy, gsph=gsph, gtail=gtail,
                   freq_eV=np.ascontiguousarray(np.asarray(freq_eV, dtype=np.complex128)),
                   delta_eV=float(delta_eV), T=T, phi=phi, centre_frac=centre,
                   alpha=alpha, gpsi=float(gpsi), seed=seed)


def parity_workload(seed: Optional[int] = None, workers: Optional[int] = None) -> Problem:
    """The small parity workload: 16^3 grid, 4^3 k mesh, q = (1/4, 0, 0),
    8 + 24 bands, N_G = 89, 10 real frequencies on [0, 20] eV, delta =
    0.1 eV, 3 Wannier Gaussians.  The oracle finishes it in seconds."""
    a = A_SRVO3_BOHR
    b = 2.0 * math.pi / a
    return make_problem(name="parity_16cube_4k_32bands", a_bohr=a, fft=(16, 16, 16),
                        kmesh=(4, 4, 4), iq=(1, 0, 0), nocc=8, nemp=24,
                        gpsi=4.153 * b, ng=89,
                        freq_eV=np.linspace(0.0, 20.0, 10), delta_eV=0.1,
                        nwan=3, alpha_range=(1.0, 2.0),
                        seed=1 if seed is None else seed, workers=workers)


def srvo3_workload(seed: Optional[int] = None, workers: Optional[int] = None) -> Problem:
    """The SrVO3-shaped q-point: cubic a = 3.8425 A, 48^3 grid, 8^3 k mesh,
    q = (1/8, 0, 0), 40 + 200 bands, 100 Ry wavefunction cutoff, N_G = 1500,
    20 real frequencies on [0, 20] eV, delta = 0.1 eV, 10 Wannier Gaussians
    (the measured workload)."""
    a = A_SRVO3_BOHR
    return make_problem(name="srvo3_48cube_8k_240bands", a_bohr=a, fft=(48, 48, 48),
                        kmesh=(8, 8, 8), iq=(1, 0, 0), nocc=40, nemp=200,
                        gpsi=math.sqrt(2.0 * 50.0), ng=1500,
                        freq_eV=np.linspace(0.0, 20.0, 20), delta_eV=0.1,
                        nwan=10, alpha_range=(1.1, 1.9),
                        seed=2 if seed is None else seed, workers=workers)


BATCH_EDGES = (24, 25, 27, 30, 32, 36, 40)


def batch_system(s: int, iq_index: int = 0, workers: Optional[int] = None) -> Problem:
    """System s (0 <= s < 24) of the batched uneven workload, at its
    iq_index-th q-point (0 <= iq_index < 4).  Drawn from seed 400 + s: cubic
    grid edge from BATCH_EDGES, cell edge scaled with it (a = a_SrVO3 edge/48),
    k-mesh edge in 2..6, 16..64 occupied + 48..256 empty bands, plane-wave
    spheres of about max(300, 1.25 n_band) vectors, N_G in 300..1200; the
    q-points are the first four non-Gamma mesh points in lexicographic order;
    16 imaginary frequencies i nu, nu in {0} and geomspace(0.1, 100, 15) eV,
    delta = 0, generalized tetrahedron."""
    if not 0 <= s < 24 or not 0 <= iq_index < 4:
        raise ValueError("system index in 0..23, q index in 0..3")
    rng = np.random.default_rng(400 + s)
    edge = int(rng.choice(BATCH_EDGES))
    kedge = int(rng.integers(2, 7))
    nocc = int(rng.integers(16, 65))
    nemp = int(rng.integers(48, 257))
    ng = int(rng.integers(300, 1201))
    a = A_SRVO3_BOHR * edge / 48.0
    b = 2.0 * math.pi / a
    npw_target = max(300, int(1.25 * (nocc + nemp)))
    gpsi = b * (3.0 * npw_target / (4.0 * math.pi)) ** (1.0 / 3.0)
    qs = [(i, j, k) for i in range(kedge) for j in range(kedge) for k in range(kedge)
          if (i, j, k) != (0, 0, 0)]
    nu = np.concatenate([[0.0], np.geomspace(0.1, 100.0, 15)])
    return make_problem(name=f"batch_system_{s}_q{iq_index}", a_bohr=a, fft=(edge, edge, edge),
                        kmesh=(kedge, kedge, kedge), iq=qs[iq_index], nocc=nocc, nemp=nemp,
                        gpsi=gpsi, ng=ng, freq_eV=1j * nu, delta_eV=0.0, nwan=0,
                        seed=400 + s, workers=workers)


def batch_system_qpoints(s: int, workers: Optional[int] = None) -> list:
    """The four q-points of batch system s as four problems that share one
    set of coefficient, Miller and energy arrays (only iq, the G sphere and
    its tail differ): the same inputs as batch_system(s, 0..3)."""
    import dataclasses
    p0 = batch_system(s, 0, workers=workers)
    kedge = p0.kmesh[0]
    qs = [(i, j, k) for i in range(kedge) for j in range(kedge) for k in range(kedge)
          if (i, j, k) != (0, 0, 0)][:4]
    recip = 2.0 * math.pi * np.linalg.inv(p0.lat).T
    out = [p0]
    for n, iq in enumerate(qs[1:], start=1):
        qf = np.array(iq, dtype=np.float64) / np.array(p0.kmesh, dtype=np.float64)
        gsph = _sphere(recip, qf, None, count=int(p0.gsph.shape[0]))
        full = _sphere(recip, qf, p0.gpsi)
        in_eps = {tuple(m) for m in gsph.tolist()}
        gtail = np.array([m for m in full.tolist() if tuple(m) not in in_eps],
                         dtype=np.int32).reshape(-1, 3)
        out.append(dataclasses.replace(p0, name=f"batch_system_{s}_q{n}", iq=tuple(iq), gsph=gsph,
                                       gtail=gtail))
    return out


def supercell_workload(nocc: int = 600, nemp: int = 1200, workers: Optional[int] = None) -> Problem:
    """A 4x4x4 supercell of the SrVO3-shaped cell (a = 29.045 bohr): 96^3
    grid, Gamma-only k mesh, q = 0 (G = 0 dropped), 600 + 1200 bands,
    plane-wave sphere of radius 8.31 (2 pi/a) (about 2 400 vectors),
    N_G = 6000, 16 real frequencies on [0, 20] eV, delta = 0.1 eV (sampling
    weights, N_k = 1), 20 Wannier Gaussians with alpha in [0.1, 0.45]."""
    a = 4.0 * A_SRVO3_BOHR
    b = 2.0 * math.pi / a
    return make_problem(name="supercell_96cube_gamma", a_bohr=a, fft=(96, 96, 96), kmesh=(1, 1, 1),
                        iq=(0, 0, 0), nocc=nocc, nemp=nemp, gpsi=8.31 * b, ng=6000,
                        freq_eV=np.linspace(0.0, 20.0, 16), delta_eV=0.1, nwan=20,
                        alpha_range=(0.1, 0.45), seed=5, workers=workers)
