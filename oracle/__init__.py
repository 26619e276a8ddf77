"""FP64 CPU oracle for the polarization / screened-interaction path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The product library never loads it.  The C
source (oracle.c) implements each step from the paper's equations; this module
marshals numpy arrays and strings the steps together in the paper's order:

  a1  k+q on the mesh                          (q-grid equals k-grid)
  a2  u_{nk}(r) from the plane-wave expansion   Eq. pak
  a3/a4 pair densities M by a direct DFT        Eq. ism
  a5  generalized-tetrahedron weights           Eqs. Xakqbk, tetrahedron, tak
  a6  chi0 = sum_p w_p M_p M_p^H                Eq. chi
  a7-a9 eps, eps^-1, W                          Eqs. epsGG, Wq
  a10 Wannier densities and W_ij                Eqs. matrix_U, rhoiqG
  q -> 0 head, wings and optics (oracle.head)  Eqs. eps00-cRPA, momentum, epsilonM,
                                               eels, optical-conductivity, reflectance
  q-mesh sums of U, V, J, X (oracle.qsum)      Eqs. W, Wq, matrix_U, rhoiqG, matrix_V,
                                               matrix_J, matrix_X
  frequency grid (oracle.grid)                 Eq. grid
  symmetry unfolding (oracle.symmetry)         Eqs. red-wavefunction, coef-G, symeps
  metallic tetrahedron weights (oracle.metal)  Eqs. Xakqbk, tetrahedron (Fermi-level cut)
  intraband (Drude) head term (oracle.drude)   Eqs. eps00, plasma, momentum

Parity status of each function is listed in its docstring.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .build import build as _build, library_path

HARTREE_EV = 27.211386245988

_lib = None


def lib():
    """The oracle's C library (liboracle.so, built on first use); the
    environment variable RP_ORACLE_LIB names another build of oracle.c to load
    instead (the sanitized build of build.build_sanitized)."""
    global _lib
    if _lib is None:
        path = os.environ.get("RP_ORACLE_LIB") or library_path()
        if not os.path.exists(path):
            _build()
        _lib = ctypes.CDLL(path)
        c = ctypes
        P = c.c_void_p
        _lib.or_kq.argtypes = [P, P, P, P]
        _lib.or_u_direct.argtypes = [P, c.c_int, P, P, P]
        _lib.or_u_separable.argtypes = [P, c.c_int, P, P, P]
        _lib.or_pair_direct.argtypes = [P, P, P, P, c.c_int, P, P]
        _lib.or_pair_separable.argtypes = [P, P, P, P, c.c_int, P, P]
        _lib.or_u_batch.argtypes = [P, c.c_int, c.c_int, P, P, c.c_long, P]
        _lib.or_pair_batch.argtypes = [P, c.c_int, P, c.c_int, P, P, c.c_int, P, P]
        _lib.or_pair_conv.argtypes = [c.c_int, P, P, c.c_int, P, P, P, c.c_int, P, P]
        _lib.or_weights.argtypes = [P, P, c.c_int, P, P, c.c_int, c.c_int, c.c_int, c.c_int,
                                    c.c_int, c.c_int, c.c_int, P, c.c_double, c.c_int, P]
        _lib.or_weights.restype = c.c_int
        _lib.or_chi0.argtypes = [c.c_long, c.c_int, P, c.c_int, P, P]
        _lib.or_invert.argtypes = [c.c_int, P, P]
        _lib.or_invert.restype = c.c_int
        _lib.or_screen.argtypes = [P, P, P, c.c_int, P, c.c_int, P, P, P, P]
        _lib.or_screen.restype = c.c_int
        _lib.or_wannier_rho.argtypes = [P, P, P, P, c.c_int, P, P, c.c_int, P, c.c_int, P]
        _lib.or_wannier_W.argtypes = [P, P, c.c_int, c.c_int, P, c.c_int, P, c.c_int, P, P]
        _lib.or_vertex_integral_py.argtypes = [P, P, c.c_int, P]
        _lib.or_tetra_scalar_py.argtypes = [P, P, P]
        _lib.or_dd4_py.argtypes = [P, P, P]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _c128(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


# ----------------------------------------------------------------- a1
def kq(kmesh, iq):
    """k' = (n+iq) mod K and G0 = (n+iq) div K for every mesh k.
    Pinned by tests/test_oracle.py::test_kq_map (brute force)."""
    kmesh, iq = _i32(kmesh), _i32(iq)
    nk = int(np.prod(kmesh))
    kp = np.empty(nk, np.int32)
    g0 = np.empty((nk, 3), np.int32)
    lib().or_kq(_p(kmesh), _p(iq), _p(kp), _p(g0))
    return kp, g0


# ----------------------------------------------------------------- a2
def u_grid(fft, miller, coef, method: str = "separable"):
    """u(r_j) = sum_G C_G e^{iG.r_j} on the grid (Eq. pak, periodic part).
    Pinned: direct == separable; single plane wave; closure and
    orthonormality pins of the pair densities built from it."""
    fft, miller, coef = _i32(fft), _i32(miller), _c128(coef)
    u = np.empty(tuple(int(x) for x in fft), np.complex128)
    f = lib().or_u_direct if method == "direct" else lib().or_u_separable
    f(_p(fft), int(miller.shape[0]), _p(miller), _p(coef), _p(u))
    return u


# ----------------------------------------------------------------- a3/a4
def pair_density(fft, ua, ub, g0, gsph, method: str = "separable"):
    """M(G) = (1/N_r) sum_j conj(ua_j) ub_j e^{i(G+G0).r_j} (Eq. ism on the grid).
    Pinned: orthonormality at q=0,G=0; closure on a complete box basis;
    equality with the plane-wave convolution; single plane waves."""
    fft, g0, gsph = _i32(fft), _i32(g0), _i32(gsph)
    ua, ub = _c128(ua), _c128(ub)
    M = np.empty(gsph.shape[0], np.complex128)
    f = lib().or_pair_direct if method == "direct" else lib().or_pair_separable
    f(_p(fft), _p(ua), _p(ub), _p(g0), int(gsph.shape[0]), _p(gsph), _p(M))
    return M


def pair_conv(miller_a, ca, miller_b, cb, g0, gsph):
    """Exact plane-wave form M(G) = sum_{G2} conj(C_a[G2+G+G0]) C_b[G2]."""
    miller_a, miller_b, g0, gsph = _i32(miller_a), _i32(miller_b), _i32(g0), _i32(gsph)
    ca, cb = _c128(ca), _c128(cb)
    M = np.empty(gsph.shape[0], np.complex128)
    lib().or_pair_conv(int(miller_a.shape[0]), _p(miller_a), _p(ca), int(miller_b.shape[0]),
                       _p(miller_b), _p(cb), _p(g0), int(gsph.shape[0]), _p(gsph), _p(M))
    return M


# ----------------------------------------------------------------- a5
def dd4(z: complex, nodes) -> complex:
    """Fourth-order divided difference of g(x) = (z-x)^3 ln(z-x)."""
    zz = np.array([z], np.complex128)
    x = _f64(nodes)
    out = np.empty(1, np.complex128)
    lib().or_dd4_py(_p(zz), _p(x), _p(out))
    return complex(out[0])


def vertex_integral(z: complex, e, i: int) -> complex:
    """I_i(z) = <lambda_i/(z-e)>_T for vertex energies e[4] (hartree).
    Pinned: flat limit, sum over vertices vs the scalar closed form,
    brute-force simplex quadrature, large-|z| moments."""
    zz = np.array([z], np.complex128)
    ee = _f64(e)
    out = np.empty(1, np.complex128)
    lib().or_vertex_integral_py(_p(zz), _p(ee), int(i), _p(out))
    return complex(out[0])


def tetra_scalar(z: complex, e) -> complex:
    """<1/(z-e)>_T by the scalar closed form (distinct energies)."""
    zz = np.array([z], np.complex128)
    ee = _f64(e)
    out = np.empty(1, np.complex128)
    lib().or_tetra_scalar_py(_p(zz), _p(ee), _p(out))
    return complex(out[0])


def weights(kmesh, iq, energy_eV, T, o0, o1, e0, e1, k0, k1, freq_eV, delta_eV,
            mode: int = 0):
    """w[f][p] = (2/Nk)(1 - T_{a,k+q} T_{b,k}) x_p(omega_f), pairs (k,a,b) b fastest.
    mode 0 = generalized tetrahedron, 1 = sampling.  Pinned as listed in
    tests/test_oracle.py (flat band, quadrature, symmetry, limits)."""
    kmesh, iq = _i32(kmesh), _i32(iq)
    E = _f64(energy_eV)
    Tp = None if T is None else _f64(T)
    freq = _c128(freq_eV)
    npair = (k1 - k0) * (e1 - e0) * (o1 - o0)
    w = np.empty((freq.shape[0], npair), np.complex128)
    rc = lib().or_weights(_p(kmesh), _p(iq), int(E.shape[1]), _p(E),
                          None if Tp is None else _p(Tp), o0, o1, e0, e1, k0, k1,
                          int(freq.shape[0]), _p(freq), float(delta_eV), int(mode), _p(w))
    if rc != 0:
        raise ValueError("bad weight arguments")
    return w


# ----------------------------------------------------------------- a6
def chi0(M, w):
    """chi[f][G][G'] = sum_p w[f][p] M[p][G] conj(M[p][G']) (Kahan-summed)."""
    M, w = _c128(M), _c128(w)
    npair, ng = M.shape
    nfreq = w.shape[0]
    chi = np.empty((nfreq, ng, ng), np.complex128)
    lib().or_chi0(int(npair), int(ng), _p(M), int(nfreq), _p(w), _p(chi))
    return chi


# ----------------------------------------------------------------- a7-a9
def invert(A):
    """Gauss-Jordan inverse with partial pivoting.  Pinned against
    numpy.linalg.inv and by the residual."""
    A = _c128(A)
    out = np.empty_like(A)
    rc = lib().or_invert(int(A.shape[0]), _p(A), _p(out))
    if rc != 0:
        raise np.linalg.LinAlgError("singular matrix")
    return out


def screen(lat, kmesh, iq, gsph, chi):
    """eps = I - v^1/2 chi v^1/2, eps^-1 and W = v^1/2 eps^-1 v^1/2 (eV)."""
    lat, kmesh, iq, gsph, chi = _f64(lat), _i32(kmesh), _i32(iq), _i32(gsph), _c128(chi)
    nfreq, ng = chi.shape[0], chi.shape[1]
    eps = np.empty_like(chi)
    einv = np.empty_like(chi)
    W = np.empty_like(chi)
    rc = lib().or_screen(_p(lat), _p(kmesh), _p(iq), int(ng), _p(gsph), int(nfreq), _p(chi),
                         _p(eps), _p(einv), _p(W))
    if rc != 0:
        raise np.linalg.LinAlgError("singular dielectric matrix")
    return eps, einv, W


# ----------------------------------------------------------------- a10
def wannier_rho(lat, fft, kmesh, iq, phi, centre_frac, glist, direct: bool = False):
    """rho_i(G) = ntilde_i(q+G)/|q+G|, ntilde_i(Q) = (Omega/N_r) sum_j phi_i^2 e^{iQ.rt}.
    Pinned against the analytic Gaussian transform on resolved grids."""
    lat, fft, kmesh, iq = _f64(lat), _i32(fft), _i32(kmesh), _i32(iq)
    phi, cf, gl = _f64(phi), _f64(centre_frac), _i32(glist)
    nwan = phi.shape[0]
    rho = np.empty((nwan, gl.shape[0]), np.complex128)
    lib().or_wannier_rho(_p(lat), _p(fft), _p(kmesh), _p(iq), int(nwan), _p(phi), _p(cf),
                         int(gl.shape[0]), _p(gl), int(bool(direct)), _p(rho))
    return rho


def wannier_W(lat, kmesh, rho_eps, rho_tail, eps_inv):
    """W_ij(w) = (4pi/(Omega Nq)) [rho eps^-1 rho^H + rho_t rho_t^H] in eV."""
    lat, kmesh = _f64(lat), _i32(kmesh)
    re, rt, ei = _c128(rho_eps), _c128(rho_tail), _c128(eps_inv)
    nwan, ng = re.shape
    nfreq = ei.shape[0]
    W = np.empty((nfreq, nwan, nwan), np.complex128)
    lib().or_wannier_W(_p(lat), _p(kmesh), int(nwan), int(ng), _p(re), int(rt.shape[1]),
                       _p(rt), int(nfreq), _p(ei), _p(W))
    return W


# ----------------------------------------------------------------- the path
def u_grids(fft, miller, coef_rows):
    """u-grids of several bands that share one Miller list (rows of coef)."""
    fft, miller = _i32(fft), _i32(miller)
    c = _c128(coef_rows)
    nb, npw = c.shape
    u = np.empty((nb,) + tuple(int(x) for x in fft), np.complex128)
    lib().or_u_batch(_p(fft), int(nb), int(npw), _p(miller), _p(c), int(npw), _p(u))
    return u


def pair_batch(fft, ua, ub, g0, gsph):
    """M[a][b][G] for all grids ua (empty, at k+q) and ub (occupied, at k)."""
    fft, g0, gsph = _i32(fft), _i32(g0), _i32(gsph)
    ua, ub = _c128(ua), _c128(ub)
    M = np.empty((ua.shape[0], ub.shape[0], gsph.shape[0]), np.complex128)
    lib().or_pair_batch(_p(fft), int(ua.shape[0]), _p(ua), int(ub.shape[0]), _p(ub), _p(g0),
                        int(gsph.shape[0]), _p(gsph), _p(M))
    return M


def pair_densities(prob, o0, o1, e0, e1, k0, k1):
    """M[(k,a,b)][G] for occupied b in [o0,o1) at k, empty a in [e0,e1) at
    k+q, k in [k0,k1); the layout of the device library's output."""
    kp, g0 = kq(prob.kmesh, prob.iq)
    out = np.empty(((k1 - k0), (e1 - e0), (o1 - o0), prob.ng), np.complex128)
    for k in range(k0, k1):
        n = prob.npw[k]
        ub = u_grids(prob.fft, prob.miller[k, :n], prob.coef[k, o0:o1, :n])
        kk = int(kp[k])
        na = prob.npw[kk]
        ua = u_grids(prob.fft, prob.miller[kk, :na], prob.coef[kk, e0:e1, :na])
        out[k - k0] = pair_batch(prob.fft, ua, ub, g0[k], prob.gsph)
    return out.reshape(-1, prob.ng)


def prob_weights(prob, o0, o1, e0, e1, k0, k1, mode: Optional[int] = None):
    m = (1 if prob.nk == 1 else 0) if mode is None else mode
    return weights(prob.kmesh, prob.iq, prob.energy_eV, prob.T, o0, o1, e0, e1, k0, k1,
                   prob.freq_eV, prob.delta_eV, m)


def run_path(prob, k0: int = 0, k1: Optional[int] = None, mode: Optional[int] = None):
    """All steps a1..a10 for one q-point over k in [k0,k1) (all bands).
    Returns a dict with M, w, chi, eps_inv, W, rho_eps, rho_tail, Wij."""
    k1 = prob.nk if k1 is None else k1
    o0, o1, e0, e1 = 0, prob.nocc, prob.nocc, prob.nband
    M = pair_densities(prob, o0, o1, e0, e1, k0, k1)
    w = prob_weights(prob, o0, o1, e0, e1, k0, k1, mode)
    chi = chi0(M, w)
    _, einv, W = screen(prob.lat, prob.kmesh, prob.iq, prob.gsph, chi)
    out = dict(M=M, w=w, chi=chi, eps_inv=einv, W=W)
    if prob.phi is not None:
        rho_e = wannier_rho(prob.lat, prob.fft, prob.kmesh, prob.iq, prob.phi,
                            prob.centre_frac, prob.gsph)
        rho_t = wannier_rho(prob.lat, prob.fft, prob.kmesh, prob.iq, prob.phi,
                            prob.centre_frac, prob.gtail)
        out.update(rho_eps=rho_e, rho_tail=rho_t,
                   Wij=wannier_W(prob.lat, prob.kmesh, rho_e, rho_t, einv))
    return out


def threads_used() -> int:
    """OpenMP threads the oracle runs with (OMP_NUM_THREADS, else the
    affinity set)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


from . import head  # noqa: E402,F401  (q -> 0 head, wings and optics)
