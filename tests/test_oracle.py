"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses an
independent route (numpy FFT, numpy.linalg, closed forms, quadrature,
identities of the definitions) chosen so that a dropped term, a wrong sign,
a wrong index or a transposed operand in the oracle fails at least one.
"""

import itertools
import math

import numpy as np
import pytest

import oracle
from synth import HARTREE_EV, make_problem
from synth.gen import gaussian_orbitals

RNG = np.random.default_rng(12345)


def _rand_c(shape, rng=RNG):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def _box_reps(n):
    """Miller representatives of an n^3 grid in [-n/2, n/2)."""
    r = np.arange(-(n // 2), n - n // 2)
    return np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)


def _numpy_u(fft, miller, coef):
    """u(j) = sum_G C_G exp(+2 pi i m.j/N) via numpy's inverse FFT."""
    box = np.zeros(fft, np.complex128)
    np.add.at(box, (miller[:, 0] % fft[0], miller[:, 1] % fft[1], miller[:, 2] % fft[2]), coef)
    return np.fft.ifftn(box) * np.prod(fft)


# ------------------------------------------------------------------ a1
def test_kq_map_brute_force():
    kmesh, iq = (3, 4, 2), (2, 3, 1)
    kp, g0 = oracle.kq(kmesh, iq)
    K = np.array(kmesh)
    for k in range(np.prod(kmesh)):
        n = np.array(np.unravel_index(k, kmesh))
        n2 = np.array(np.unravel_index(kp[k], kmesh))
        assert np.all(n + np.array(iq) == n2 + K * g0[k])
        assert np.all((n2 >= 0) & (n2 < K))


# ------------------------------------------------------------------ a2
def test_u_grid_matches_numpy_fft_and_direct_sum():
    fft = (6, 5, 4)
    miller = np.array([[0, 0, 0], [1, -2, 1], [-1, 1, 0], [2, 0, -1], [0, 2, 1]], np.int32)
    coef = _rand_c(len(miller))
    ref = _numpy_u(fft, miller, coef)
    for method in ("direct", "separable"):
        u = oracle.u_grid(fft, miller, coef, method)
        assert np.max(np.abs(u - ref)) < 1e-13


# ------------------------------------------------------------------ a3/a4
def test_pair_single_plane_waves_are_kronecker():
    """psi_a = e^{i(k'+Ga)r}, psi_b = e^{i(k+Gb)r} => M(G) = [Ga = Gb + G + G0]."""
    fft = (12, 12, 12)
    gsph = _box_reps(7)
    Ga, Gb, g0 = np.array([1, -2, 0]), np.array([0, 1, 1]), np.array([1, 0, 0])
    ua = _numpy_u(fft, Ga[None].astype(np.int32), np.array([1.0 + 0j]))
    ub = _numpy_u(fft, Gb[None].astype(np.int32), np.array([1.0 + 0j]))
    for method in ("direct", "separable"):
        M = oracle.pair_density(fft, ua, ub, g0, gsph, method)
        want = np.all(gsph == (Ga - Gb - g0)[None], axis=1).astype(float)
        assert want.sum() == 1
        assert np.max(np.abs(M - want)) < 1e-14


def test_pair_orthonormality_q0_G0():
    """At q = 0 and G = 0, M_nm = <n,k|m,k> = delta_nm (Eq. ism with
    orthonormal Bloch functions)."""
    p = make_problem(name="t", a_bohr=7.26, fft=(12, 12, 12), kmesh=(2, 2, 2), iq=(0, 0, 0),
                     nocc=3, nemp=3, gpsi=2.2, ng=4, freq_eV=[0.0], delta_eV=0.1, seed=7)
    k = 3
    npw = p.npw[k]
    u = [oracle.u_grid(p.fft, p.miller[k, :npw], p.coef[k, n, :npw]) for n in range(6)]
    g = np.zeros((1, 3), np.int32)
    M = np.array([[oracle.pair_density(p.fft, u[n], u[m], [0, 0, 0], g)[0] for m in range(6)]
                  for n in range(6)])
    assert np.max(np.abs(M - np.eye(6))) < 1e-14


def test_pair_closure_complete_box_basis():
    """With all N_r bands of a unitary basis on a 4^3 box, sum over the
    occupied index: sum_m M_nm(G) conj(M_nm(G')) = (1/N_r) sum_j |u_n(j)|^2
    e^{i(G-G').r_j} (completeness; the umklapp G0 cancels)."""
    fft = (4, 4, 4)
    reps = _box_reps(4)
    nr = 64
    q1, _ = np.linalg.qr(_rand_c((nr, nr)))
    q2, _ = np.linalg.qr(_rand_c((nr, nr)))
    g0 = np.array([1, 0, 0])
    gs = np.array([[0, 0, 0], [1, 0, 0], [-1, 1, 0], [0, -1, 1]], np.int32)
    n = 5
    ua = _numpy_u(fft, reps, q1[:, n])
    ubs = [_numpy_u(fft, reps, q2[:, m]) for m in range(nr)]
    M = np.array([oracle.pair_density(fft, ua, ub, g0, gs) for ub in ubs])  # [m][G]
    lhs = M.T @ M.conj()
    dens = np.abs(ua) ** 2
    j = np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1)
    rhs = np.empty_like(lhs)
    for a, G in enumerate(gs):
        for b, Gp in enumerate(gs):
            ph = np.exp(2j * np.pi * (j @ (G - Gp)) / 4)
            rhs[a, b] = np.sum(dens * ph) / nr
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_pair_grid_route_equals_plane_wave_convolution():
    """Alias-free grid (2 n_psi + n_eps + 1 < N): the FFT route equals the
    exact convolution sum_{G2} conj(C_a[G2+G+G0]) C_b[G2] (Eq. ism)."""
    p = make_problem(name="t", a_bohr=7.26, fft=(16, 16, 16), kmesh=(2, 2, 2), iq=(1, 0, 1),
                     nocc=2, nemp=2, gpsi=3.0, ng=27, freq_eV=[0.0], delta_eV=0.1, seed=3)
    kp, g0 = oracle.kq(p.kmesh, p.iq)
    assert np.abs(p.miller).max() * 2 + np.abs(p.gsph).max() + 1 < 16
    for k in (0, 5):
        kk = kp[k]
        na, nb = p.npw[kk], p.npw[k]
        for a, b in ((2, 0), (3, 1)):
            ua = oracle.u_grid(p.fft, p.miller[kk, :na], p.coef[kk, a, :na])
            ub = oracle.u_grid(p.fft, p.miller[k, :nb], p.coef[k, b, :nb])
            Mc = oracle.pair_conv(p.miller[kk, :na], p.coef[kk, a, :na],
                                  p.miller[k, :nb], p.coef[k, b, :nb], g0[k], p.gsph)
            for method in ("separable", "direct"):
                Mg = oracle.pair_density(p.fft, ua, ub, g0[k], p.gsph, method)
                assert np.max(np.abs(Mg - Mc)) < 1e-13
            assert np.max(np.abs(Mc)) > 1e-3


def test_pair_densities_path_assembly_matches_plane_wave_form():
    """oracle.pair_densities (the layout the library writes: pairs (k, a, b)
    with b fastest, a empty at k' = k + q on the mesh, b occupied at k, the
    umklapp G0 shifting the gather) against the plane-wave convolution of Eq.
    ism, with k' and G0 worked out here from the mesh arithmetic, for pairs
    at k-points with and without umklapp.  A k <-> k' swap, a conj on the
    wrong side, a wrong G0 or a wrong pair index fails it."""
    kmesh, iq = (3, 2, 2), (2, 1, 0)
    p = make_problem(name="t", a_bohr=7.26, fft=(16, 16, 16), kmesh=kmesh, iq=iq,
                     nocc=3, nemp=3, gpsi=3.0, ng=27, freq_eV=[0.0], delta_eV=0.1, seed=9)
    assert np.abs(p.miller).max() * 2 + np.abs(p.gsph).max() + 2 < 16
    o0, o1, e0, e1, k0, k1 = 1, 3, 3, 6, 2, 8
    M = oracle.pair_densities(p, o0, o1, e0, e1, k0, k1)
    assert M.shape == ((k1 - k0) * (e1 - e0) * (o1 - o0), p.ng)
    K = np.array(kmesh)
    umklapp = 0
    checked = 0
    for k in range(k0, k1):
        n = np.array(np.unravel_index(k, kmesh))
        s = n + np.array(iq)
        kk = int(np.ravel_multi_index(tuple(s % K), kmesh))
        g0 = s // K
        umklapp += int(np.any(g0 != 0))
        for a, b in ((e0, o0), (e1 - 1, o1 - 1), (e0 + 1, o0 + 1)):
            row = ((k - k0) * (e1 - e0) + (a - e0)) * (o1 - o0) + (b - o0)
            na, nb = p.npw[kk], p.npw[k]
            want = oracle.pair_conv(p.miller[kk, :na], p.coef[kk, a, :na],
                                    p.miller[k, :nb], p.coef[k, b, :nb], g0, p.gsph)
            assert np.max(np.abs(M[row] - want)) < 1e-13, (k, a, b)
            assert np.max(np.abs(want)) > 1e-3
            checked += 1
    assert umklapp >= 2 and checked >= 9
    # the swapped assignment (empty band at k, occupied at k') is a different
    # array: the check above would see it
    k = k0
    n = np.array(np.unravel_index(k, kmesh))
    kk = int(np.ravel_multi_index(tuple((n + np.array(iq)) % K), kmesh))
    wrong = oracle.pair_conv(p.miller[k, :p.npw[k]], p.coef[k, e0, :p.npw[k]],
                             p.miller[kk, :p.npw[kk]], p.coef[kk, o0, :p.npw[kk]],
                             (n + np.array(iq)) // K, p.gsph)
    assert np.max(np.abs(M[0] - wrong)) > 1e-3


def test_pair_density_matches_numpy_fft():
    fft = (8, 6, 10)
    ua, ub = _rand_c(fft), _rand_c(fft)
    g0 = np.array([0, 1, -1])
    gs = np.array([[0, 0, 0], [1, 2, -3], [-2, 0, 4], [3, -2, 1]], np.int32)
    # (1/N) sum_j f_j e^{+2 pi i m.j/N} = ifftn(f)[m mod N]
    ref = np.fft.ifftn(np.conj(ua) * ub)
    m = (gs + g0) % np.array(fft)
    want = ref[m[:, 0], m[:, 1], m[:, 2]]
    for method in ("direct", "separable"):
        assert np.max(np.abs(oracle.pair_density(fft, ua, ub, g0, gs, method) - want)) < 1e-14


# ------------------------------------------------------------------ a5
def _simplex_rule(n):
    """Collapsed (Duffy) Gauss-Legendre rule on the unit 3-simplex; returns
    barycentric coordinates [npts,4] and weights normalised to sum 1."""
    x, wx = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1)
    wx = 0.5 * wx
    u, v, t = np.meshgrid(x, x, x, indexing="ij")
    wu, wv, wt = np.meshgrid(wx, wx, wx, indexing="ij")
    l1 = u
    l2 = (1 - u) * v
    l3 = (1 - u) * (1 - v) * t
    jac = (1 - u) ** 2 * (1 - v)
    w = (wu * wv * wt * jac).ravel()
    lam = np.stack([1 - l1 - l2 - l3, l1, l2, l3], -1).reshape(-1, 4)
    return lam, w / w.sum()


LAM, WQ = _simplex_rule(70)


@pytest.mark.parametrize("e,z", [
    ([0.1, 0.5, 0.9, 1.3], 0.7 + 0.3j),
    ([0.4, 0.4000001, 0.8, 1.1], 0.6 + 0.25j),      # near-degenerate pair
    ([0.5, 0.5, 0.9, 0.9], 0.2 + 0.4j),             # exactly degenerate pairs
    ([0.7, 0.7, 0.7, 0.7 + 1e-9], -0.3 + 0.35j),    # nearly flat
    ([-0.3, 0.6, 0.2, 0.25], 0.1 - 0.3j),           # lower half plane
    ([1.0, 1.2, 2.5, 3.1], 0.05 + 0.5j),
])
def test_vertex_integral_vs_simplex_quadrature(e, z):
    """I_i(z) = <lambda_i/(z-e(lambda))>_T by brute-force quadrature."""
    e = np.array(e)
    ee = LAM @ e
    for i in range(4):
        q = np.sum(WQ * LAM[:, i] / (z - ee))
        got = oracle.vertex_integral(z, e, i)
        assert abs(got - q) < 1e-12 * max(1.0, abs(q)), (i, got, q)


def test_vertex_integral_flat_limit_and_sum_rule():
    z = 0.3 + 0.01j
    for e0 in (-1.0, 0.2, 0.31):
        for i in range(4):
            assert abs(oracle.vertex_integral(z, [e0] * 4, i) - 0.25 / (z - e0)) < 1e-13 / abs(z - e0)
    rng = np.random.default_rng(5)
    for _ in range(20):
        e = np.sort(rng.uniform(-1, 2, 4))
        if np.min(np.diff(e)) < 0.05:
            continue
        z = complex(rng.uniform(-1, 2), rng.uniform(0.003, 0.2))
        s = sum(oracle.vertex_integral(z, e, i) for i in range(4))
        sc = oracle.tetra_scalar(z, e)
        assert abs(s - sc) < 1e-11 * abs(sc)


def test_vertex_integral_large_z_moments():
    """I_i(z) = 1/(4z) + <lambda_i e>/z^2 + <lambda_i e^2>/z^3 + O(z^-4) with
    the Dirichlet(1,1,1,1) moments <l_a l_b> = (1+d_ab)/20 and
    <l_a l_b l_c> = (multiplicity factorials)/120."""
    e = np.array([0.3, -0.2, 0.8, 0.5])
    z = 2.0e3 + 1.0j
    for i in range(4):
        m1 = (e[i] + e.sum()) / 20.0
        m2 = 0.0
        for j in range(4):
            for k in range(4):
                idx = sorted((i, j, k))
                mult = [idx.count(t) for t in set(idx)]
                m2 += e[j] * e[k] * np.prod([math.factorial(c) for c in mult]) / 120.0
        I_ = oracle.vertex_integral(z, e, i)
        assert abs((I_ - 0.25 / z) * z * z - m1) < 1e-4
        assert abs((I_ - 0.25 / z - m1 / z ** 2) * z ** 3 - m2) < 1e-4


def test_vertex_integral_continuous_at_degeneracy():
    z = 0.45 + 0.02j
    base = np.array([0.2, 0.5, 0.5, 0.9])
    for i in range(4):
        a = oracle.vertex_integral(z, base, i)
        for eps in (1e-12, 1e-9, 1e-6):
            b = oracle.vertex_integral(z, base + np.array([0, 0, eps, 0]), i)
            assert abs(a - b) < 50 * eps * abs(a) + 1e-13 * abs(a)


def _flat_problem(iq=(1, 0, 0), kmesh=(3, 3, 3)):
    nk = int(np.prod(kmesh))
    E = np.zeros((nk, 3))
    E[:, 0] = -2.0
    E[:, 1] = 3.0
    E[:, 2] = 7.5
    return kmesh, iq, E


def test_weights_flat_band_equals_textbook_X():
    """Energies constant over k: the tetrahedron weight reduces to Eq. Xakqbk."""
    kmesh, iq, E = _flat_problem()
    freq = np.array([0.0, 4.0, 5.0, 9.5, 2.0j])
    delta = 0.2
    w = oracle.weights(kmesh, iq, E, None, 0, 1, 1, 3, 0, 27, freq, delta, 0)
    ws = oracle.weights(kmesh, iq, E, None, 0, 1, 1, 3, 0, 27, freq, delta, 1)
    nk = 27
    for f, om in enumerate(freq):
        for a, ea in ((0, 3.0), (1, 7.5)):
            de = (ea + 2.0) / HARTREE_EV
            o = om / HARTREE_EV
            dl = delta / HARTREE_EV
            X = 1 / (o - de + 1j * dl) - 1 / (o + de - 1j * dl)
            idx = np.arange(nk) * 2 + a
            assert np.max(np.abs(w[f, idx] - 2 / nk * X)) < 1e-13 * abs(2 / nk * X)
            assert np.max(np.abs(ws[f, idx] - 2 / nk * X)) < 1e-13 * abs(2 / nk * X)


def _hat_quadrature(kmesh, iq, Ea, Eb, k, z, zp, nsub=24):
    """x(k) = N_k * int_BZ hat_k(x) [1/(z-e(x)) + 1/(z'-e(x))] dx by a midpoint
    rule in the eight subcells around k.  The interpolant is located by
    sorting the fractional coordinates inside a subcell (Freudenthal cells
    t_s0 >= t_s1 >= t_s2), independently of how the oracle enumerates its
    tetrahedra."""
    K = np.array(kmesh)
    n = np.array(np.unravel_index(k, kmesh))
    h = (np.arange(nsub) + 0.5) / nsub
    t = np.stack(np.meshgrid(h, h, h, indexing="ij"), -1).reshape(-1, 3)
    order = np.argsort(-t, axis=1, kind="stable")
    ts = np.take_along_axis(t, order, 1)
    lam = np.stack([1 - ts[:, 0], ts[:, 0] - ts[:, 1], ts[:, 1] - ts[:, 2], ts[:, 2]], -1)
    # vertex offsets: 0, e_s0, e_s0+e_s1, (1,1,1)
    off = np.zeros((len(t), 4, 3), int)
    for v in range(1, 4):
        off[:, v] = off[:, v - 1]
        np.put_along_axis(off[:, v], order[:, v - 1:v], 1, axis=1)
    total = 0.0 + 0.0j
    for s in itertools.product((0, 1), repeat=3):
        c = n - np.array(s)
        verts = c[None, None, :] + off
        vi = np.ravel_multi_index(tuple(np.moveaxis(verts % K, -1, 0)), kmesh)
        vq = np.ravel_multi_index(tuple(np.moveaxis((verts + np.array(iq)) % K, -1, 0)), kmesh)
        e = Ea[vq] - Eb[vi]
        ee = np.sum(lam * e, 1)
        hat = np.sum(lam * np.all(off == np.array(s)[None, None, :], axis=2), 1)
        total += np.mean(hat * (1 / (z - ee) + 1 / (zp - ee)))
    return total


def test_weights_geometry_vs_interpolant_quadrature():
    """Tetrahedron weights integrate the piecewise-linear interpolant of
    E_a(k+q) - E_b(k) against the hat function of k (midpoint rule, loose)."""
    kmesh, iq = (3, 3, 3), (1, 2, 0)
    rng = np.random.default_rng(9)
    nk = 27
    E = np.zeros((nk, 2))
    E[:, 0] = rng.uniform(-3, -1, nk)
    E[:, 1] = rng.uniform(1, 6, nk)
    freq = np.array([3.0 + 0j])
    delta = 3.0   # broad, so that the midpoint rule converges
    w = oracle.weights(kmesh, iq, E, None, 0, 1, 1, 2, 0, nk, freq, delta, 0)
    z = (3.0 + 1j * delta) / HARTREE_EV
    zp = (-3.0 + 1j * delta) / HARTREE_EV
    for k in (0, 13, 26):
        want = _hat_quadrature(kmesh, iq, E[:, 1] / HARTREE_EV, E[:, 0] / HARTREE_EV, k, z, zp)
        got = w[0, k] * nk / 2.0
        assert abs(got - want) < 2e-3 * abs(want), (k, got, want)


def test_weights_absorption_symmetry_and_crpa():
    p = make_problem(name="t", a_bohr=7.26, fft=(8, 8, 8), kmesh=(3, 3, 2), iq=(1, 1, 0),
                     nocc=2, nemp=3, gpsi=1.8, ng=5, freq_eV=np.linspace(0, 12, 7),
                     delta_eV=0.1, crpa=True, seed=11)
    nk = p.nk
    w = oracle.weights(p.kmesh, p.iq, p.energy_eV, None, 0, 2, 2, 5, 0, nk, p.freq_eV, 0.1, 0)
    assert np.all(w.imag[1:] < 0)                       # absorption, real omega > 0
    wm = oracle.weights(p.kmesh, p.iq, p.energy_eV, None, 0, 2, 2, 5, 0, nk, -p.freq_eV, 0.1, 0)
    assert np.max(np.abs(w - wm)) < 1e-15 * np.abs(w).max()   # x(-w) = x(w)
    wt = oracle.weights(p.kmesh, p.iq, p.energy_eV, p.T, 0, 2, 2, 5, 0, nk, p.freq_eV, 0.1, 0)
    kp, _ = oracle.kq(p.kmesh, p.iq)
    for k in range(nk):
        for a in range(3):
            for b in range(2):
                pi = (k * 3 + a) * 2 + b
                fac = 1 - p.T[kp[k], 2 + a] * p.T[k, b]
                assert np.max(np.abs(wt[:, pi] - fac * w[:, pi])) < 1e-15 * np.abs(w).max()
    assert np.any(np.abs(wt - w) > 1e-6 * np.abs(w).max())
    # imaginary axis, delta = 0: real, negative weights
    wi = oracle.weights(p.kmesh, p.iq, p.energy_eV, None, 0, 2, 2, 5, 0, nk,
                        1j * np.array([0.0, 0.5, 3.0, 40.0]), 0.0, 0)
    assert np.max(np.abs(wi.imag)) < 1e-13 * np.abs(wi).max()
    assert np.all(wi.real < 0)


# ------------------------------------------------------------------ a6
def test_chi_plane_wave_closed_form():
    """One plane-wave valence and conduction band with flat energies:
    M(G) = [G = Ga - G0(k)], so chi is diagonal with entries
    (2/N_k) X(w) * #{k : Ga - G0(k) = G}   (Eq. chi)."""
    kmesh, iq = (2, 2, 2), (1, 1, 0)
    fft = (8, 8, 8)
    Ga = np.array([1, 0, 0])
    gs = np.array([[0, 0, 0], [1, 0, 0], [0, -1, 0], [1, -1, 0], [0, 0, 1], [-1, 0, 0]], np.int32)
    kp, g0 = oracle.kq(kmesh, iq)
    ub = _numpy_u(fft, np.zeros((1, 3), np.int32), np.array([1.0 + 0j]))
    ua = _numpy_u(fft, Ga[None].astype(np.int32), np.array([1.0 + 0j]))
    M = np.array([oracle.pair_density(fft, ua, ub, g0[k], gs) for k in range(8)])
    E = np.zeros((8, 2))
    E[:, 0], E[:, 1] = -1.0, 2.5
    freq = np.array([0.0, 1.0, 3.5])
    w = oracle.weights(kmesh, iq, E, None, 0, 1, 1, 2, 0, 8, freq, 0.1, 0)
    chi = oracle.chi0(M, w)
    de, dl = 3.5 / HARTREE_EV, 0.1 / HARTREE_EV
    for f, om in enumerate(freq / HARTREE_EV):
        X = 1 / (om - de + 1j * dl) - 1 / (om + de - 1j * dl)
        want = np.zeros((6, 6), complex)
        for k in range(8):
            g = Ga - g0[k]
            idx = np.where(np.all(gs == g, axis=1))[0]
            if len(idx):
                want[idx[0], idx[0]] += 2 / 8 * X
        assert np.max(np.abs(chi[f] - want)) < 1e-14 * np.abs(want).max()
        assert np.abs(want).max() > 0


def _small_path_problem(**kw):
    args = dict(name="t", a_bohr=7.26, fft=(12, 12, 12), kmesh=(2, 2, 2), iq=(1, 0, 0),
                nocc=3, nemp=4, gpsi=2.6, ng=15, freq_eV=[0.0, 2.0, 9.0], delta_eV=0.1,
                seed=21)
    args.update(kw)
    return make_problem(**args)


def test_chi_structure_and_gauge_invariance():
    p = _small_path_problem()
    M = oracle.pair_densities(p, 0, 3, 3, 7, 0, p.nk)
    w = oracle.prob_weights(p, 0, 3, 3, 7, 0, p.nk)
    chi = oracle.chi0(M, w)
    # absorptive part B = (chi - chi^H)/2i is negative semidefinite at real w
    for f in range(chi.shape[0]):
        B = (chi[f] - chi[f].conj().T) / 2j
        assert np.max(np.linalg.eigvalsh(B)) < 1e-12 * np.abs(B).max()
    # random band phases change M but not chi
    rng = np.random.default_rng(1)
    q = p.coef * np.exp(1j * rng.uniform(0, 2 * np.pi, p.coef.shape[:2]))[:, :, None]
    p2 = _small_path_problem()
    p2.coef = q
    M2 = oracle.pair_densities(p2, 0, 3, 3, 7, 0, p.nk)
    assert np.max(np.abs(M2 - M)) > 1e-3
    chi2 = oracle.chi0(M2, w)
    assert np.max(np.abs(chi2 - chi)) < 1e-13 * np.abs(chi).max()
    # imaginary axis (delta = 0): chi Hermitian and negative definite
    wi = oracle.weights(p.kmesh, p.iq, p.energy_eV, None, 0, 3, 3, 7, 0, p.nk,
                        1j * np.array([0.0, 1.0, 10.0]), 0.0, 0)
    ci = oracle.chi0(M, wi)
    for f in range(3):
        assert np.max(np.abs(ci[f] - ci[f].conj().T)) < 1e-12 * np.abs(ci[f]).max()
        assert np.max(np.linalg.eigvalsh((ci[f] + ci[f].conj().T) / 2)) < 1e-12 * np.abs(ci[f]).max()
    # single pair: chi = w M M^H
    c1 = oracle.chi0(M[5:6], w[:, 5:6])
    assert np.max(np.abs(c1[1] - w[1, 5] * np.outer(M[5], M[5].conj()))) < 1e-16


# ------------------------------------------------------------------ a7-a9
def _qg(lat, kmesh, iq, gs):
    b = 2 * np.pi * np.linalg.inv(lat).T
    return np.linalg.norm((np.array(iq) / np.array(kmesh) + gs) @ b, axis=1)


def test_screen_zero_chi_gives_bare_coulomb():
    lat = np.diag([7.0, 7.5, 8.0])
    gs = np.array([[0, 0, 0], [1, 0, 0], [0, -1, 1], [2, 1, 0]], np.int32)
    kmesh, iq = (4, 4, 2), (1, 2, 1)
    chi = np.zeros((2, 4, 4), complex)
    eps, einv, W = oracle.screen(lat, kmesh, iq, gs, chi)
    vol = np.linalg.det(lat)
    bare = 4 * np.pi / vol / _qg(lat, kmesh, iq, gs) ** 2 * HARTREE_EV
    for f in range(2):
        assert np.max(np.abs(einv[f] - np.eye(4))) == 0
        assert np.max(np.abs(W[f] - np.diag(bare))) < 1e-13 * bare.max()


def test_screen_scalar_case_and_library_inverse():
    lat = np.eye(3) * 6.0
    gs = np.array([[0, 1, 0]], np.int32)
    kmesh, iq = (2, 2, 2), (1, 0, 0)
    chi = np.array([[[-0.3 + 0.05j]], [[-0.01 - 0.2j]]])
    _, einv, W = oracle.screen(lat, kmesh, iq, gs, chi)
    v = 4 * np.pi / 216.0 / _qg(lat, kmesh, iq, gs)[0] ** 2
    for f in range(2):
        assert abs(einv[f, 0, 0] - 1 / (1 - v * chi[f, 0, 0])) < 1e-15
    rng = np.random.default_rng(2)
    A = _rand_c((37, 37), rng) + 3 * np.eye(37)
    inv = oracle.invert(A)
    assert np.max(np.abs(inv - np.linalg.inv(A))) < 1e-13
    assert np.max(np.abs(A @ inv - np.eye(37))) < 1e-13
    # a matrix needing row exchanges
    P = np.eye(6)[[3, 0, 5, 1, 4, 2]]
    A = P @ (np.triu(_rand_c((6, 6), rng)) + 2 * np.eye(6))
    assert A[0, 0] == 0      # forces a row exchange at the first pivot
    assert np.max(np.abs(oracle.invert(A) @ A - np.eye(6))) < 1e-12


def test_screen_static_spectrum():
    """chi Hermitian negative semidefinite (omega = 0, delta = 0) =>
    eps >= 1 and eps^-1 in (0, 1]."""
    p = _small_path_problem()
    M = oracle.pair_densities(p, 0, 3, 3, 7, 0, p.nk)
    w0 = oracle.weights(p.kmesh, p.iq, p.energy_eV, None, 0, 3, 3, 7, 0, p.nk,
                        np.array([0.0]), 0.0, 0)
    chi = oracle.chi0(M, w0) * 200.0   # strong screening
    eps, einv, _ = oracle.screen(p.lat, p.kmesh, p.iq, p.gsph, chi)
    ev = np.linalg.eigvalsh((eps[0] + eps[0].conj().T) / 2)
    evi = np.linalg.eigvalsh((einv[0] + einv[0].conj().T) / 2)
    assert ev.min() > 1 - 1e-12 and ev.max() > 1.5
    assert evi.min() > 0 and evi.max() < 1 + 1e-12


# ------------------------------------------------------------------ a10
def test_wannier_rho_analytic_gaussian():
    """A normalised Gaussian density exp(-2 alpha r^2) has transform
    e^{iQ.R} exp(-|Q|^2 / (8 alpha)); grid resolved and contained at 1e-12."""
    a = 7.26
    lat = np.eye(3) * a
    fft = (40, 40, 40)
    kmesh, iq = (4, 4, 4), (1, 2, 3)
    centre = np.array([[0.1, 0.7, 0.45], [0.9, 0.05, 0.5]])
    alpha = np.array([1.15, 1.3])
    phi = gaussian_orbitals(lat, fft, centre, alpha)
    gs = np.array([[0, 0, 0], [1, 0, 0], [-1, 2, 0], [3, -2, 1], [0, 0, -4]], np.int32)
    rho = oracle.wannier_rho(lat, fft, kmesh, iq, phi, centre, gs)
    b = 2 * np.pi / a
    Q = (np.array(iq) / np.array(kmesh) + gs) * b
    Qn = np.linalg.norm(Q, axis=1)
    for i in range(2):
        want = np.exp(1j * Q @ (centre[i] * a)) * np.exp(-Qn ** 2 / (8 * alpha[i])) / Qn
        assert np.max(np.abs(rho[i] - want)) < 1e-11
    phi12 = gaussian_orbitals(lat, (12, 12, 12), centre, alpha)
    rd = oracle.wannier_rho(lat, (12, 12, 12), kmesh, iq, phi12, centre, gs, direct=True)
    rs = oracle.wannier_rho(lat, (12, 12, 12), kmesh, iq, phi12, centre, gs)
    assert np.max(np.abs(rd - rs)) < 1e-13


def test_wannier_W_bare_gaussian_coulomb_sum():
    """eps^-1 = I: W_ij = (4pi/(Omega N_q)) sum_G rho_i(G) conj(rho_j(G)) over
    S_eps and the tail, evaluated here from the analytic Gaussian transforms."""
    p = make_problem(name="t", a_bohr=7.26, fft=(40, 40, 40), kmesh=(2, 2, 2), iq=(1, 0, 0),
                     nocc=1, nemp=1, gpsi=6.0, ng=30, freq_eV=[0.0], delta_eV=0.1,
                     nwan=2, alpha_range=(1.15, 1.3), seed=4)
    re_ = oracle.wannier_rho(p.lat, p.fft, p.kmesh, p.iq, p.phi, p.centre_frac, p.gsph)
    rt = oracle.wannier_rho(p.lat, p.fft, p.kmesh, p.iq, p.phi, p.centre_frac, p.gtail)
    einv = np.eye(p.ng)[None].astype(complex)
    Wij = oracle.wannier_W(p.lat, p.kmesh, re_, rt, einv)[0]
    b = 2 * np.pi / 7.26
    allg = np.concatenate([p.gsph, p.gtail])
    Q = (np.array(p.iq) / 2 + allg) * b
    Qn2 = np.sum(Q * Q, 1)
    R = p.centre_frac * 7.26
    want = np.empty((2, 2), complex)
    for i in range(2):
        for j in range(2):
            want[i, j] = np.sum(np.exp(1j * Q @ (R[i] - R[j])) *
                                np.exp(-Qn2 * (1 / (8 * p.alpha[i]) + 1 / (8 * p.alpha[j]))) / Qn2)
    want *= 4 * np.pi / (7.26 ** 3 * 8) * HARTREE_EV
    assert np.max(np.abs(Wij - want)) < 1e-10 * np.abs(want).max()
    assert np.max(np.abs(Wij - Wij.conj().T)) < 1e-12 * np.abs(want).max()


def test_wannier_static_screening_reduces_W():
    p = _small_path_problem(nwan=2, alpha_range=(1.0, 2.0), freq_eV=[0.0], fft=(16, 16, 16))
    out = oracle.run_path(p)
    bare = oracle.wannier_W(p.lat, p.kmesh, out["rho_eps"], out["rho_tail"],
                            np.eye(p.ng)[None].astype(complex))
    for i in range(2):
        assert out["Wij"][0, i, i].real < bare[0, i, i].real


def test_crpa_removes_only_target_transitions():
    """T = 1 on occupied band b* at every k and on empty band a* only at the
    mesh point k1: Eq. chi's factor (1 - T_{a,k+q} T_{b,k}) must zero exactly
    the pairs (k, a*, b*) with k + q = k1 (mod mesh), and nothing else."""
    kmesh, iq = (3, 2, 2), (2, 1, 0)
    nk = 12
    rng = np.random.default_rng(3)
    E = np.concatenate([np.sort(rng.uniform(-6, -1, (nk, 2)), 1),
                        np.sort(rng.uniform(1, 9, (nk, 3)), 1)], 1)
    k1 = 7
    T = np.zeros((nk, 5))
    T[:, 1] = 1.0
    T[k1, 3] = 1.0
    freq = np.array([0.5, 4.0])
    w = oracle.weights(kmesh, iq, E, None, 0, 2, 2, 5, 0, nk, freq, 0.1, 0)
    wt = oracle.weights(kmesh, iq, E, T, 0, 2, 2, 5, 0, nk, freq, 0.1, 0)
    n1 = np.array(np.unravel_index(k1, kmesh))
    ksrc = np.ravel_multi_index(tuple((n1 - np.array(iq)) % np.array(kmesh)), kmesh)
    for k in range(nk):
        for a in range(3):
            for b in range(2):
                pi = (k * 3 + a) * 2 + b
                if k == ksrc and a == 1 and b == 1:
                    assert np.all(wt[:, pi] == 0)
                else:
                    assert np.all(wt[:, pi] == w[:, pi])


def test_wannier_W_rank_one_screening():
    """eps^-1 = I + u v^H gives W_ij = bare_ij + c (rho_i . u) conj(rho_j . v),
    c = HA * 4pi/(Omega N_q): pins the orientation of eps^-1 in the projection."""
    rng = np.random.default_rng(8)
    lat = np.eye(3) * 7.0
    kmesh = (2, 3, 2)
    ng, nt, nw = 9, 5, 3
    re_, rt = _rand_c((nw, ng), rng), _rand_c((nw, nt), rng)
    u, v = _rand_c(ng, rng), _rand_c(ng, rng)
    einv = (np.eye(ng) + np.outer(u, v.conj()))[None]
    Wij = oracle.wannier_W(lat, kmesh, re_, rt, einv)[0]
    c = HARTREE_EV * 4 * np.pi / (343.0 * 12)
    want = c * (re_ @ re_.conj().T + rt @ rt.conj().T + np.outer(re_ @ u, (re_ @ v).conj()))
    assert np.max(np.abs(Wij - want)) < 1e-13 * np.abs(want).max()
