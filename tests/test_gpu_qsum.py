"""GPU parity of one q-point's term of the q-mesh sums of U, V, J and X
(rp_wannier_qterm; Eqs. W, Wq, matrix_U, rhoiqG, matrix_V, matrix_J,
matrix_X) against the oracle (oracle/qsum.py), element by element to 1e-10
relative to the largest element, on seeded synthetic orbitals and a seeded
random eps^-1: away from Gamma, at Gamma with the head term, with the
exchange densities in several passes and with accumulation over q."""


import numpy as np
import pytest

import oracle
from oracle import qsum
from synth.gen import gaussian_orbitals

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def rp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_02351_amd as rp
    rp.load()
    return rp


@pytest.fixture(scope="module")
def ctx(rp):
    c = rp.Context(0)
    yield c
    c.close()


def _dev(a):
    a = np.ascontiguousarray(a)
    if np.iscomplexobj(a):
        a = np.stack([a.real, a.imag], -1)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _c(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def _case(iq, nR, nwan=3, fft=(16, 16, 16), kmesh=(2, 3, 2), ng=150, ntail=37, nfreq=2, seed=0):
    """Orbitals (Gaussians, two near a face so that neighbouring cells
    overlap), R vectors (the home cell first), a G list sorted by |q+G| (G = 0
    first at Gamma) and a random eps^-1 near the identity."""
    rng = np.random.default_rng(seed)
    a = 7.26
    lat = np.array([[a, 0.0, 0.0], [0.2, a, 0.0], [0.0, -0.3, a]])
    cen = rng.uniform(0, 1, (nwan, 3))
    cen[0, 0], cen[1, 0] = 0.04, 0.93
    cen[1, 1:] = (cen[0, 1:] + 0.05) % 1.0
    alpha = rng.uniform(0.6, 1.0, nwan)
    phi = gaussian_orbitals(lat, fft, cen, alpha)
    Rs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0)]
    while len(Rs) < nR:
        r = tuple(int(x) for x in rng.integers(-2, 3, 3))
        if r not in Rs:
            Rs.append(r)
    R = np.array(Rs[:nR], np.int32)
    span = np.arange(-6, 7)
    allg = np.stack(np.meshgrid(span, span, span, indexing="ij"), -1).reshape(-1, 3)
    qn = qsum.qg_norm(lat, kmesh, iq, allg)
    order = np.lexsort((allg[:, 2], allg[:, 1], allg[:, 0], qn))
    gl = allg[order][: ng + ntail].astype(np.int32)
    E = np.eye(ng)[None] + 0.05 * (rng.standard_normal((nfreq, ng, ng)) + 1j * rng.standard_normal((nfreq, ng, ng)))
    return dict(lat=lat, fft=fft, kmesh=kmesh, iq=tuple(iq), cen=cen, phi=phi, R=R, gl=gl, ng=ng, ntail=ntail, E=E)


def _want(c):
    gamma = all(x == 0 for x in c["iq"])
    n_u = np.stack([qsum.exchange_ntilde(c["lat"], c["fft"], c["kmesh"], c["iq"], c["phi"], c["cen"],
                                         [[0, 0, 0]], c["gl"])[0, i, i] for i in range(len(c["cen"]))])
    n_x = qsum.exchange_ntilde(c["lat"], c["fft"], c["kmesh"], c["iq"], c["phi"], c["cen"], c["R"], c["gl"])
    A = qsum.cell_average(c["lat"], c["kmesh"]) if gamma else None
    return qsum.qterm(c["lat"], c["kmesh"], c["iq"], n_u, n_x, c["ng"], c["E"], c["R"], c["gl"], head_avg=A)


def _run(rp, ctx, c, accumulate=0, out=None):
    nf, nR, nw = c["E"].shape[0], len(c["R"]), len(c["cen"])
    cell = rp.make_cell(c["lat"], c["fft"], c["kmesh"])
    if out is None:
        out = dict(U=torch.zeros((nf, nR, nw, nw, 2), dtype=torch.float64, device="cuda"),
                   J=torch.zeros((nf, nR, nw, nw, 2), dtype=torch.float64, device="cuda"),
                   V=torch.zeros((nR, nw, nw, 2), dtype=torch.float64, device="cuda"),
                   X=torch.zeros((nR, nw, nw, 2), dtype=torch.float64, device="cuda"))
    ng = c["ng"]
    rp.rp_wannier_qterm(ctx, cell, c["iq"], nw, _dev(c["phi"]), c["cen"], c["R"], ng, c["gl"][:ng],
                        c["ntail"], c["gl"][ng:], nf, _dev(c["E"]), accumulate, **out)
    rp.rp_synchronize(ctx)
    return out


def _check(got, want, label):
    for k in ("U", "J", "V", "X"):
        g, w = _c(got[k]), want[k]
        err = np.max(np.abs(g - w)) / np.abs(w).max()
        print(f"[qsum] {label} {k}: max |diff| / max |want| = {err:.2e}", flush=True)
        assert err < TOL, (label, k, err)


@pytest.mark.parametrize("iq", [(1, 2, 0), (0, 1, 1)])
def test_qterm_matches_oracle(rp, ctx, iq):
    c = _case(iq, nR=5)
    got = _run(rp, ctx, c)
    want = _want(c)
    _check(got, want, f"iq={iq}")
    # the direct and exchange routes agree on i = j, R = 0
    U, J = _c(got["U"]), _c(got["J"])
    for i in range(3):
        assert np.max(np.abs(U[:, 0, i, i] - J[:, 0, i, i])) < 1e-12 * np.abs(U).max()


def test_qterm_gamma_head(rp, ctx):
    """q = 0: G = 0 first, the head term through the cell average, the
    wings dropped."""
    c = _case((0, 0, 0), nR=4, seed=3)
    got = _run(rp, ctx, c)
    _check(got, _want(c), "Gamma")


def test_qterm_several_passes_and_accumulation(rp, ctx):
    """64 R vectors x 3^2 pairs = 576 exchange densities (two passes of at
    most 512), ragged G tiles; two q-points accumulated."""
    c1 = _case((1, 0, 1), nR=64, ng=70, ntail=20, nfreq=1, seed=5)
    c2 = dict(c1)
    c2["iq"] = (0, 2, 1)
    span = np.arange(-6, 7)
    allg = np.stack(np.meshgrid(span, span, span, indexing="ij"), -1).reshape(-1, 3)
    qn = qsum.qg_norm(c1["lat"], c1["kmesh"], c2["iq"], allg)
    order = np.lexsort((allg[:, 2], allg[:, 1], allg[:, 0], qn))
    c2["gl"] = allg[order][:90].astype(np.int32)
    c2["E"] = np.conj(c1["E"]).transpose(0, 2, 1).copy()
    out = _run(rp, ctx, c1)
    out = _run(rp, ctx, c2, accumulate=1, out=out)
    w1, w2 = _want(c1), _want(c2)
    _check(out, {k: w1[k] + w2[k] for k in w1}, "two q-points")


def test_qterm_rejects_bad_arguments(rp, ctx):
    c = _case((0, 0, 0), nR=2)
    nf, nw = c["E"].shape[0], 3
    cell = rp.make_cell(c["lat"], c["fft"], c["kmesh"])
    phi, E = _dev(c["phi"]), _dev(c["E"])
    U = torch.zeros((nf, 2, nw, nw, 2), dtype=torch.float64, device="cuda")
    ng = c["ng"]
    gl = c["gl"]
    with pytest.raises(rp.RpError) as e:   # G = 0 not first at q = 0
        rp.rp_wannier_qterm(ctx, cell, (0, 0, 0), nw, phi, c["cen"], c["R"], ng, gl[1:ng + 1], 0, None, nf, E,
                            0, U=U)
    assert e.value.status == 3
    with pytest.raises(rp.RpError) as e:   # G = 0 again in the tail
        rp.rp_wannier_qterm(ctx, cell, (0, 0, 0), nw, phi, c["cen"], c["R"], ng, gl[:ng], 1, gl[:1], nf, E,
                            0, U=U)
    assert e.value.status == 3
    with pytest.raises(rp.RpError) as e:   # no output
        rp.rp_wannier_qterm(ctx, cell, (0, 0, 0), nw, phi, c["cen"], c["R"], ng, gl[:ng], 0, None, nf, E, 0)
    assert e.value.status == 1
    with pytest.raises(rp.RpError) as e:
        rp.rp_wannier_qterm(ctx, cell, (0, 0, 0), nw, phi, c["cen"], c["R"], ng, gl[:ng], 0, None, nf, E, 2, U=U)
    assert e.value.status == 3
    rp.rp_synchronize(ctx)


def test_full_qmesh_sum_matches_oracle(rp, ctx):
    """U, J, V, X summed over a 2x2x2 q mesh through the whole FP64 path
    (pair densities, weights, chi0, eps^-1 with the head at Gamma, the
    q-terms) against the oracle's chain, to 1e-10."""
    import copy

    from oracle import head as ohead
    from paper_2001_02351_amd import path
    from synth import at_qpoint, make_problem
    p = make_problem(name="qmesh", a_bohr=7.26, fft=(16, 16, 16), kmesh=(2, 2, 2), iq=(0, 0, 0), nocc=4,
                     nemp=10, gpsi=2.4, ng=30, freq_eV=np.array([0.0, 6.0]), delta_eV=0.1, nwan=2,
                     alpha_range=(0.8, 1.2), seed=41)
    R = np.array([[0, 0, 0], [1, 0, 0], [0, -1, 0]], np.int32)
    qhat = (1.0, 0.0, 0.0)
    d = path.DeviceInputs(p)
    got = path.interaction(ctx, d, R, lambda iq: at_qpoint(p, iq), prec=rp.RP_FP64, kbatch=4, qhat=qhat)
    rp.rp_synchronize(ctx)
    A = qsum.cell_average(p.lat, p.kmesh)
    want = None
    for iq in np.ndindex(*p.kmesh):
        pq = at_qpoint(p, iq)
        if iq == (0, 0, 0):
            gl = np.concatenate([np.zeros((1, 3), np.int32), pq.gsph]).astype(np.int32)
            q = copy.copy(pq)
            q.gsph = gl
            M = oracle.pair_densities(q, 0, p.nocc, p.nocc, p.nband, 0, p.nk)
            M[:, 0] = ohead.head_density(pq, 0, p.nocc, p.nocc, p.nband, 0, p.nk, qhat)
            w = oracle.prob_weights(pq, 0, p.nocc, p.nocc, p.nband, 0, p.nk)
            _, einv = ohead.screen_head(p.lat, gl, oracle.chi0(M, w), oracle.invert)
        else:
            gl = pq.gsph
            einv = oracle.run_path(pq)["eps_inv"]
        allg = np.concatenate([gl, pq.gtail])
        n_u = np.stack([qsum.exchange_ntilde(p.lat, p.fft, p.kmesh, iq, p.phi, p.centre_frac, [[0, 0, 0]],
                                             allg)[0, i, i] for i in range(2)])
        n_x = qsum.exchange_ntilde(p.lat, p.fft, p.kmesh, iq, p.phi, p.centre_frac, R, allg)
        t = qsum.qterm(p.lat, p.kmesh, iq, n_u, n_x, len(gl), einv, R, allg,
                       head_avg=A if iq == (0, 0, 0) else None)
        want = t if want is None else {k: want[k] + t[k] for k in t}
    _check(got, want, "2x2x2 q mesh")
    # static screening lowers the on-site direct term below the bare one
    U = _c(got["U"])
    V = _c(got["V"])
    for i in range(2):
        assert U[0, 0, i, i].real < V[0, i, i].real
