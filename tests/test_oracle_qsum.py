"""Pins of the q-sum oracle (oracle/qsum.py) against closed forms, library
routines and the pinned density oracle: Eqs. W, Wq, matrix_U, rhoiqG,
matrix_V, matrix_J, matrix_X."""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import qsum
from synth.gen import gaussian_orbitals

HA = qsum.HARTREE_EV


def _gauss_pair(lat, alpha, cen, R, i, j, Q):
    """Closed-form transform of phi_i0 phi_jR for normalized Gaussians
    (2 alpha/pi)^{3/4} exp(-alpha |r - C|^2): the product is a Gaussian of
    exponent s = alpha_i + alpha_j centred at P = (alpha_i A + alpha_j B)/s,
    scaled by exp(-mu |A - B|^2), mu = alpha_i alpha_j / s."""
    A = cen[i] @ lat
    B = (cen[j] + R) @ lat
    ai, aj = alpha[i], alpha[j]
    s = ai + aj
    P = (ai * A + aj * B) / s
    norm = (2 * ai / math.pi) ** 0.75 * (2 * aj / math.pi) ** 0.75 * (math.pi / s) ** 1.5
    return norm * math.exp(-ai * aj / s * np.sum((A - B) ** 2)) * np.exp(1j * Q @ P - np.sum(Q * Q, 1) / (4 * s))


def test_exchange_density_analytic_gaussians():
    """Overlap densities of resolved Gaussians, home cell and neighbouring
    cells (centres near the faces so that phi_jR reaches phi_i0): the grid
    transform equals the closed form to 1e-11."""
    a = 7.26
    lat = np.eye(3) * a
    fft = (40, 40, 40)
    kmesh, iq = (4, 4, 4), (1, 2, 3)
    cen = np.array([[0.06, 0.48, 0.5], [0.9, 0.55, 0.42], [0.5, 0.5, 0.93]])
    alpha = np.array([1.6, 1.75, 1.9])
    phi = gaussian_orbitals(lat, fft, cen, alpha)
    R = np.array([[0, 0, 0], [-1, 0, 0], [0, 0, -1], [1, 0, 0]])
    gs = np.array([[0, 0, 0], [1, 0, 0], [-1, 2, 0], [3, -2, 1], [0, 0, -4]])
    nt = qsum.exchange_ntilde(lat, fft, kmesh, iq, phi, cen, R, gs)
    Q = (np.array(iq) / np.array(kmesh) + gs) @ qsum.reciprocal(lat)
    big = 0.0
    for r in range(len(R)):
        for i in range(3):
            for j in range(3):
                want = _gauss_pair(lat, alpha, cen, R[r], i, j, Q)
                big = max(big, np.abs(want).max())
                assert np.max(np.abs(nt[r, i, j] - want)) < 1e-11, (r, i, j)
    assert big > 1e-3        # the neighbouring-cell pairs overlap


def test_exchange_density_diagonal_is_the_direct_density():
    """rho_ii0q of the exchange densities is the direct density rho_iq of the
    (separately pinned) C oracle, off the analytic case (random orbitals)."""
    rng = np.random.default_rng(11)
    lat = np.array([[7.0, 0.3, 0.0], [0.0, 6.5, 0.2], [0.1, 0.0, 7.4]])
    fft, kmesh, iq = (12, 10, 14), (3, 2, 4), (2, 1, 3)
    phi = rng.standard_normal((2, *fft))
    cen = rng.uniform(0, 1, (2, 3))
    gs = np.array([[0, 0, 0], [1, -1, 0], [2, 0, 3], [-3, 1, -2]])
    nt = qsum.exchange_ntilde(lat, fft, kmesh, iq, phi, cen, [[0, 0, 0]], gs)
    want = oracle.wannier_rho(lat, fft, kmesh, iq, phi, cen, gs) * qsum.qg_norm(lat, kmesh, iq, gs)
    for i in range(2):
        assert np.max(np.abs(nt[0, i, i] - want[i])) < 1e-12 * np.abs(want).max()


def test_cell_average_cube_closed_form():
    """Cubic cell of edge s = 2 pi/(a N): int_cell d^3q/|q|^2 = s C with
    C = 12 int_0^1 atan(1/sqrt(1+u^2)) / sqrt(1+u^2) du (the six face
    pyramids with the inner integral done in closed form), so
    A = N_q Omega/(2 pi)^3 s C = (a N / (2 pi))^2 C."""
    C, _ = integrate.quad(lambda u: math.atan(1 / math.sqrt(1 + u * u)) / math.sqrt(1 + u * u), 0, 1,
                          epsabs=1e-14, epsrel=1e-13)
    C *= 12
    for a, N in ((7.26, 4), (5.0, 2), (10.0, 8)):
        got = qsum.cell_average(np.eye(3) * a, (N, N, N))
        want = (a * N / (2 * math.pi)) ** 2 * C
        assert abs(got - want) < 1e-12 * want, (a, N, got, want)


def test_cell_average_sheared_cell_brute_force():
    """A triclinic cell against the inscribed ball (4 pi r0 exactly) plus a
    midpoint sum over the rest of the cell on a fine grid (1e-3)."""
    lat = np.array([[6.0, 0.8, 0.0], [0.5, 7.0, 0.0], [0.3, -0.4, 6.5]])
    kmesh = (3, 2, 4)
    e = qsum.reciprocal(lat) / np.array(kmesh)[:, None]
    normals = [np.cross(e[(a + 1) % 3], e[(a + 2) % 3]) for a in range(3)]
    r0 = min(abs(0.5 * e[a] @ n) / np.linalg.norm(n) for a, n in enumerate(normals))
    m = 160
    x = (np.arange(m) + 0.5) / m - 0.5
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3) @ e
    q2 = np.sum(X * X, 1)
    dv = abs(np.linalg.det(e)) / m ** 3
    rest = np.sum(np.where(q2 > r0 * r0, 1.0 / q2, 0.0)) * dv
    integral = 4 * math.pi * r0 + rest
    want = np.prod(kmesh) * abs(np.linalg.det(lat)) / (2 * math.pi) ** 3 * integral
    got = qsum.cell_average(lat, kmesh)
    assert abs(got - want) < 1e-3 * want


def _rand_c(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_qterm_bare_limits_and_rank_one_screening():
    """eps^-1 = I: U = V and J = X; eps^-1 = I + u v^H adds
    pre e^{-iq.R} (rho_i . u) conj(rho_j . v) to U and
    pre (rho_v . u) conj(rho_v . v) to J (orientation of eps^-1)."""
    rng = np.random.default_rng(2)
    lat = np.diag([7.0, 6.0, 8.0])
    kmesh, iq = (2, 3, 2), (1, 2, 1)
    ng, nt, nw = 7, 4, 2
    gl = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [1, 1, 0], [0, -1, 1], [2, 0, 0],
                   [0, 2, 0], [0, 0, -2], [1, -1, 1], [-2, 0, 1]])
    n_u = _rand_c((nw, ng + nt), rng)
    R = np.array([[0, 0, 0], [1, -1, 2]])
    n_x = _rand_c((2, nw, nw, ng + nt), rng)
    eye = np.eye(ng)[None].astype(complex)
    t = qsum.qterm(lat, kmesh, iq, n_u, n_x, ng, eye, R, gl)
    assert np.allclose(t["U"][0], t["V"], rtol=0, atol=1e-14 * np.abs(t["V"]).max())
    assert np.allclose(t["J"][0], t["X"], rtol=0, atol=1e-14 * np.abs(t["X"]).max())
    u, v = _rand_c(ng, rng), _rand_c(ng, rng)
    t1 = qsum.qterm(lat, kmesh, iq, n_u, n_x, ng, (np.eye(ng) + np.outer(u, v.conj()))[None], R, gl)
    qn = qsum.qg_norm(lat, kmesh, iq, gl)
    ru, rx = n_u / qn, n_x / qn
    pre = HA * 4 * math.pi / (np.linalg.det(lat) * 12)
    ph = np.exp(-2j * math.pi * (R @ (np.array(iq) / np.array(kmesh))))
    for r in range(2):
        du = pre * ph[r] * np.outer(ru[:, :ng] @ u, (ru[:, :ng] @ v).conj())
        assert np.max(np.abs(t1["U"][0, r] - t["U"][0, r] - du)) < 1e-12 * np.abs(du).max()
        dx = pre * (rx[r, ..., :ng] @ u) * (rx[r, ..., :ng] @ v).conj()
        assert np.max(np.abs(t1["J"][0, r] - t["J"][0, r] - dx)) < 1e-12 * np.abs(dx).max()


def test_qterm_gamma_head_only_through_the_average():
    """At q = 0 the G = 0 entries enter only as A eps^-1_00 ntilde_a(0)
    conj(ntilde_b(0)): changing eps^-1's wings leaves U and J unchanged, and
    the head contributes exactly that term."""
    rng = np.random.default_rng(4)
    lat = np.eye(3) * 6.0
    kmesh = (2, 2, 2)
    gl = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [1, 1, 1]])
    ng = 4
    n_u = _rand_c((2, 6), rng)
    n_x = _rand_c((1, 2, 2, 6), rng)
    E = np.eye(ng, dtype=complex)[None] + 0.1 * _rand_c((1, ng, ng), rng)
    A = 3.7
    t = qsum.qterm(lat, kmesh, (0, 0, 0), n_u, n_x, ng, E, [[0, 0, 0]], gl, head_avg=A)
    E2 = E.copy()
    E2[0, 0, 1:] += 5.0
    E2[0, 1:, 0] -= 2.0j
    t2 = qsum.qterm(lat, kmesh, (0, 0, 0), n_u, n_x, ng, E2, [[0, 0, 0]], gl, head_avg=A)
    assert np.max(np.abs(t2["U"] - t["U"])) < 1e-13 * np.abs(t["U"]).max()
    assert np.max(np.abs(t2["J"] - t["J"])) < 1e-13 * np.abs(t["J"]).max()
    E3 = E.copy()
    E3[0, 0, 0] += 1.0
    t3 = qsum.qterm(lat, kmesh, (0, 0, 0), n_u, n_x, ng, E3, [[0, 0, 0]], gl, head_avg=A)
    pre = HA * 4 * math.pi / (216.0 * 8)
    want = pre * A * np.outer(n_u[:, 0], n_u[:, 0].conj())
    assert np.max(np.abs(t3["U"][0, 0] - t["U"][0, 0] - want)) < 1e-12 * np.abs(want).max()
    wantx = pre * A * np.abs(n_x[0, :, :, 0]) ** 2
    assert np.max(np.abs(t3["J"][0, 0] - t["J"][0, 0] - wantx)) < 1e-12 * np.abs(wantx).max()
    with pytest.raises(ValueError):
        qsum.qterm(lat, kmesh, (0, 0, 0), n_u, n_x, ng, E, [[0, 0, 0]], gl[::-1].copy(), head_avg=A)


def test_bare_qsum_analytic_gaussians():
    """The whole q-mesh sum of the bare terms from grid densities equals the
    same sum from the closed-form Gaussian transforms (phases e^{-iq.R},
    normalization 4 pi/(Omega N_q), exchange densities of neighbouring cells,
    the Gamma head through the cell average) to 1e-10; the diagonal exchange
    X_{i0i0} equals V_{i0i0}."""
    a = 7.26
    lat = np.eye(3) * a
    fft, kmesh = (36, 36, 36), (2, 2, 2)
    cen = np.array([[0.08, 0.5, 0.5], [0.93, 0.45, 0.55]])
    alpha = np.array([1.6, 1.8])
    phi = gaussian_orbitals(lat, fft, cen, alpha)
    R = np.array([[0, 0, 0], [-1, 0, 0], [1, 0, 0], [0, 1, 0]])
    A = qsum.cell_average(lat, kmesh)
    rec = qsum.reciprocal(lat)
    rng_g = np.arange(-5, 6)
    allg = np.stack(np.meshgrid(rng_g, rng_g, rng_g, indexing="ij"), -1).reshape(-1, 3)
    V = np.zeros((len(R), 2, 2), complex)
    X = np.zeros((len(R), 2, 2), complex)
    Vw = np.zeros_like(V)
    Xw = np.zeros_like(X)
    nq = 8
    pre = HA * 4 * math.pi / (a ** 3 * nq)
    for iq in np.ndindex(*kmesh):
        Q = (np.array(iq) / np.array(kmesh) + allg) @ rec
        gcut = allg[np.linalg.norm(Q, axis=1) <= 4.5]
        # S_eps: the 20 shortest |q+G| (G = 0 first at q = 0); the rest is the tail
        qn = qsum.qg_norm(lat, kmesh, iq, gcut)
        order = np.lexsort((gcut[:, 2], gcut[:, 1], gcut[:, 0], qn))
        gl = gcut[order]
        ng = 20
        n_u = np.stack([qsum.exchange_ntilde(lat, fft, kmesh, iq, phi, cen, [[0, 0, 0]], gl)[0, i, i]
                        for i in range(2)])
        n_x = qsum.exchange_ntilde(lat, fft, kmesh, iq, phi, cen, R, gl)
        t = qsum.qterm(lat, kmesh, iq, n_u, n_x, ng, np.eye(ng)[None].astype(complex), R, gl,
                       head_avg=A if iq == (0, 0, 0) else None)
        V += t["V"]
        X += t["X"]
        # closed form
        Qg = (np.array(iq) / np.array(kmesh) + gl) @ rec
        q2 = np.sum(Qg * Qg, 1)
        inv = np.where(q2 > 0, 1 / np.where(q2 > 0, q2, 1), 0.0)
        qf = np.array(iq) / np.array(kmesh)
        for r in range(len(R)):
            ph = np.exp(-2j * math.pi * (R[r] @ qf))
            for i in range(2):
                for j in range(2):
                    ni = _gauss_pair(lat, alpha, cen, np.zeros(3), i, i, Qg)
                    nj = _gauss_pair(lat, alpha, cen, np.zeros(3), j, j, Qg)
                    v = np.sum(ni * nj.conj() * inv)
                    nx = _gauss_pair(lat, alpha, cen, R[r], i, j, Qg)
                    x = np.sum(np.abs(nx) ** 2 * inv)
                    if iq == (0, 0, 0):
                        v += A * ni[0] * np.conj(nj[0])
                        x += A * abs(nx[0]) ** 2
                    Vw[r, i, j] += pre * ph * v
                    Xw[r, i, j] += pre * x
    assert np.max(np.abs(V - Vw)) < 1e-10 * np.abs(Vw).max()
    assert np.max(np.abs(X - Xw)) < 1e-10 * np.abs(Xw).max()
    assert np.abs(Xw[1, 0, 1]) > 1e-4 * np.abs(Xw[0, 0, 0])   # the neighbouring-cell pair counts
    for i in range(2):
        assert abs(X[0, i, i] - V[0, i, i]) < 1e-12 * abs(V[0, i, i])
    # V real up to rounding after the full mesh sum (q and -q pair up)
    assert np.max(np.abs(V.imag)) < 1e-10 * np.abs(V).max()
