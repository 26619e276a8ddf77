"""GPU parity of the symmetry unfolding (rp_unfold_coef, rp_unfold_eps_inv;
Eqs. coef-G, symeps) against the oracle (oracle/symmetry.py) on the
synthetic 4_1-screw crystal: unfolded coefficients and rotated matrices
element by element, and chi on the GPU from GPU-unfolded bands against the
oracle's chi from the bands diagonalized at every k."""

import dataclasses

import numpy as np
import pytest

import oracle
from oracle import symmetry as osym
from synth.gen import mesh_fractions
from synth.symmetric import star_table, symmetric_problem, with_gvectors

torch = pytest.importorskip("torch")


def _rel(a, b):
    """The larger of the relative Frobenius norm of a - b and the largest
    element-wise deviation over the largest |b|."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    return max(np.linalg.norm(d) / np.linalg.norm(b), d.max() / np.abs(b).max())
pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def model():
    p, ops = symmetric_problem()
    return p, ops, star_table(p.kmesh, ops), mesh_fractions(p.kmesh)


def _idx(kf, kmesh):
    return [int(round(x * K)) % K for x, K in zip(kf, kmesh)]


def _c(t):
    a = t.cpu().numpy()
    return a[..., 0::2] + 1j * a[..., 1::2] if t.dim() == 2 else a[..., 0] + 1j * a[..., 1]


def _unfold_all(rp, ctx, p, ops, tab, kf, d):
    """Every k of the mesh unfolded on the GPU from its representative."""
    cell = rp.make_cell(p.lat, p.fft, p.kmesh)
    out = torch.zeros_like(d.coef)
    for k, (i, g, _) in enumerate(tab):
        W, t = ops[g]
        n, ni = int(p.npw[k]), int(p.npw[i])
        rp.rp_unfold_coef(ctx, cell, W, t, _idx(kf[i], p.kmesh), p.miller[i, :ni], d.coef[i], _idx(kf[k], p.kmesh),
                          p.miller[k, :n], out[k])
    rp.rp_synchronize(ctx)
    return out


def test_unfold_coef_matches_oracle(rp, ctx, model):
    from paper_2001_02351_amd import path
    p, ops, tab, kf = model
    d = path.DeviceInputs(p)
    got = _unfold_all(rp, ctx, p, ops, tab, kf, d).cpu().numpy().view(np.complex128)
    worst = 0.0
    for k, (i, g, _) in enumerate(tab):
        W, t = ops[g]
        n, ni = int(p.npw[k]), int(p.npw[i])
        want = osym.unfold_coef(W, t, kf[i], p.miller[i, :ni], p.coef[i, :, :ni], kf[k], p.miller[k, :n])
        worst = max(worst, np.max(np.abs(got[k, :, :n] - want)))
        assert np.all(got[k, :, n:] == 0)
    print(f"[symmetry] coefficients max |diff| = {worst:.1e}", flush=True)
    assert worst < 1e-14


def test_chi_from_unfolded_bands(rp, ctx, model):
    """chi (FP64) on the GPU from bands unfolded on the GPU equals the
    oracle's chi from the bands diagonalized at every k.  The weights are
    taken at each k (sampling): the unfolded and the diagonalized bands differ
    by rotations inside degenerate multiplets, which such weights do not see,
    while tetrahedron weights, interpolating each band index across the
    neighbouring k, do."""
    from paper_2001_02351_amd import path
    p, ops, tab, kf = model
    d = path.DeviceInputs(p)
    d.coef = _unfold_all(rp, ctx, p, ops, tab, kf, d)
    nb = p.nocc + p.nemp
    for iq in ((1, 0, 0), (1, 2, 1)):
        pq = with_gvectors(p, iq)
        dq = d.at_q(pq)
        M = path.pair_density(ctx, dq, 0, p.nk, prec=rp.RP_FP64)
        chi = torch.empty((dq.nfreq, dq.ng, dq.ng, 2), dtype=torch.float64, device="cuda")
        rp.rp_chi0_accumulate(ctx, dq.cell, pq.iq, nb, dq.energy, dq.T, 0, p.nocc, p.nocc, nb, 0, p.nk, dq.ng, M,
                              dq.nfreq, pq.freq_eV, pq.delta_eV, rp.RP_W_SAMPLING, rp.RP_FP64, 0, chi)
        rp.rp_synchronize(ctx)
        got = path.to_complex(chi)
        Mo = oracle.pair_densities(pq, 0, p.nocc, p.nocc, nb, 0, p.nk)
        want = oracle.chi0(Mo, oracle.prob_weights(pq, 0, p.nocc, p.nocc, nb, 0, p.nk, mode=1))
        err = max(_rel(got[f], want[f]) for f in range(len(want)))
        print(f"[symmetry] chi at iq={iq} from unfolded bands: rel {err:.1e}", flush=True)
        assert err < 1e-10


def test_unfold_eps_inv_matches_oracle(rp, ctx, model):
    """Rotation of a G-indexed matrix for every operation: the oracle's chi
    at q* and a random matrix on a 300-vector list (several row blocks)."""
    p, ops, _, _ = model
    cell = rp.make_cell(p.lat, p.fft, p.kmesh)
    qs = np.array([1, 0, 1])
    qf = qs / np.array(p.kmesh)
    ps = with_gvectors(p, tuple(qs))
    nb = p.nocc + p.nemp
    chis = oracle.chi0(oracle.pair_densities(ps, 0, p.nocc, p.nocc, nb, 0, p.nk),
                       oracle.prob_weights(ps, 0, p.nocc, p.nocc, nb, 0, p.nk))
    rng = np.random.default_rng(3)
    big = with_gvectors(dataclasses.replace(p, gsph=np.zeros((300, 3), np.int32)), tuple(qs)).gsph
    rnd = rng.standard_normal((2, 300, 300)) + 1j * rng.standard_normal((2, 300, 300))
    for gl, X in ((ps.gsph, chis), (big, rnd)):
        src = torch.from_numpy(np.ascontiguousarray(np.stack([X.real, X.imag], -1))).cuda()
        for W, t in ops:
            S = osym.op_S(W)
            iq = _idx(S @ qf, p.kmesh)
            qg = np.array(iq) / np.array(p.kmesh)
            tgt = np.ascontiguousarray((gl @ S.T - osym.rewind(W, qf, qg)).astype(np.int32))
            dst = torch.empty_like(src)
            rp.rp_unfold_eps_inv(ctx, cell, W, t, qs, gl, iq, tgt, src, dst)
            rp.rp_synchronize(ctx)
            want = osym.unfold_matrix(W, t, qf, gl, X, qg, tgt)
            assert np.max(np.abs(_c(dst) - want)) < 1e-14 * np.abs(want).max()


def test_unfold_rejects_bad_arguments(rp, ctx, model):
    p, ops, tab, kf = model
    from paper_2001_02351_amd import path
    d = path.DeviceInputs(p)
    cell = rp.make_cell(p.lat, p.fft, p.kmesh)
    out = torch.zeros_like(d.coef[0])
    n0 = int(p.npw[0])
    W, t = ops[1]
    cases = [
        (np.diag([2, 1, 1]), t, [0, 0, 0], [0, 0, 0], p.miller[0, :n0]),      # det 2
        (W, t, [1, 0, 0], [1, 0, 0], p.miller[0, :n0]),                       # (1,0,0) -> (0,1,0), not (1,0,0)
        (W, t, [0, 0, 0], [0, 0, 0], np.array([[9, 9, 9]], np.int32)),        # no source vector
    ]
    for Wb, tb, ki, kt, mt in cases:
        with pytest.raises(rp.RpError) as e:
            rp.rp_unfold_coef(ctx, cell, Wb, tb, ki, p.miller[0, :n0], d.coef[0], kt, mt, out)
        assert e.value.status == 3
    X = torch.zeros((1, 4, 4, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(rp.RpError) as e:
        rp.rp_unfold_eps_inv(ctx, cell, W, t, [0, 0, 0], p.gsph[:4], [0, 0, 0], p.gsph[:4], X, X)
    assert e.value.status == 4
    rp.rp_synchronize(ctx)
