"""Parity at the full SrVO3-shaped sizes (48^3 grid, 8^3 k, 40+200 bands,
N_G = 1500, 20 real frequencies, 10 Wannier orbitals) in the launch
configurations bench.py times (k batches of two and of sixteen k-points, all
frequencies per launch), on outputs the oracle can compute one by one, and on
properties that hold at any size:

* pair densities and weights of sampled pairs of a full k batch,
* chi over a k batch for a band subset, restricted to sampled rows/columns
  (the oracle's chi0 of the sampled columns of M is exactly that restriction),
* eps^-1 / W and W_ij at N_G = 1500 for two frequencies of a synthetic chi,
* batch linearity of chi at full size; the 16-k-point sliced launch against
  two-k-point launches and the FP64 contraction,
* that launch (split-BF16 and FP64) against the oracle's Eq. chi of all its
  128 000 pairs on 48 sampled rows and columns.
"""

import numpy as np
import pytest

import oracle
from synth import srvo3_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KB = (36, 38)          # one k batch of the bench's size (kbatch = 2)


def _rel(a, b):
    """The larger of the relative Frobenius norm of a - b and the largest
    element-wise deviation over the largest |b|."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    return max(np.linalg.norm(d) / np.linalg.norm(b), d.max() / np.abs(b).max())


@pytest.fixture(scope="module")
def rp():
    import paper_2001_02351_amd as rp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rp.load()
    return rp


@pytest.fixture(scope="module")
def ctx(rp):
    c = rp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c2():
    print("[fullsize] generating the 48^3 / 8^3 k / 240-band workload", flush=True)
    return srvo3_workload()


@pytest.fixture(scope="module")
def d2(c2, rp):
    from paper_2001_02351_amd.path import DeviceInputs
    return DeviceInputs(c2)


def _sample_pairs(p, rng, n):
    out = []
    for _ in range(n):
        k = int(rng.integers(*KB))
        a = int(rng.integers(p.nocc, p.nband))
        b = int(rng.integers(0, p.nocc))
        out.append((k, a, b))
    out += [(KB[0], p.nocc, 0), (KB[1] - 1, p.nband - 1, p.nocc - 1)]   # corners
    return out


def _oracle_pair(p, k, a, b):
    kp, g0 = oracle.kq(p.kmesh, p.iq)
    kk = int(kp[k])
    ub = oracle.u_grids(p.fft, p.miller[k, :p.npw[k]], p.coef[k, b:b + 1, :p.npw[k]])
    ua = oracle.u_grids(p.fft, p.miller[kk, :p.npw[kk]], p.coef[kk, a:a + 1, :p.npw[kk]])
    return oracle.pair_batch(p.fft, ua, ub, g0[k], p.gsph)[0, 0]


def test_pair_density_and_weights_sampled(ctx, rp, c2, d2):
    from paper_2001_02351_amd import path
    p = c2
    rng = np.random.default_rng(5)
    samples = _sample_pairs(p, rng, 10)
    nO, nE = p.nocc, p.nemp
    M64 = path.to_complex(path.pair_density(ctx, d2, *KB, prec=rp.RP_FP64))
    M32 = path.to_complex(path.pair_density(ctx, d2, *KB, prec=rp.RP_SPLIT_BF16))
    w = path.to_complex(path.weights(ctx, d2, *KB))
    for (k, a, b) in samples:
        pi = ((k - KB[0]) * nE + (a - p.nocc)) * nO + b
        want = _oracle_pair(p, k, a, b)
        assert _rel(M64[pi], want) < 1e-12, (k, a, b)
        assert _rel(M32[pi], want) < 2e-6, (k, a, b)
        ww = oracle.prob_weights(p, b, b + 1, a, a + 1, k, k + 1)[:, 0]
        assert np.max(np.abs(w[:, pi] - ww)) < 1e-12 * np.abs(ww).max(), (k, a, b)
    print(f"[fullsize] {len(samples)} sampled pairs checked", flush=True)


@pytest.fixture(scope="module")
def chi_subset(c2):
    """Oracle M and w for the k batch, all occupied x 40 empty bands."""
    p = c2
    o, e = (0, p.nocc), (p.nocc, p.nocc + 40)
    print("[fullsize] oracle pair densities for 3200 pairs", flush=True)
    M = oracle.pair_densities(p, *o, *e, *KB)
    w = oracle.prob_weights(p, *o, *e, *KB)
    rng = np.random.default_rng(11)
    cols = np.unique(np.concatenate([rng.choice(p.ng, 40, replace=False), [0, 1, p.ng - 2, p.ng - 1]]))
    return o, e, M, w, cols


# The six-product form's bound: its products are FP32-accurate, so chi's error
# comes from the FP32 pair densities (about 1e-7) and from FP32 accumulation
# within one slice of at most 512 matrix-core steps, whose rounding grows like
# 2^-24 sqrt(512) = 1.3e-6 of the partial sums; 5e-6 leaves a factor of about
# four over that estimate (measured 9.4e-7 at this size).
@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5), (2, 5e-6)])
def test_chi_sampled_block(ctx, rp, c2, d2, chi_subset, prec, tol):
    from paper_2001_02351_amd import path
    p = c2
    o, e, M, w, cols = chi_subset
    npair = (KB[1] - KB[0]) * (e[1] - e[0]) * (o[1] - o[0])
    Md = torch.empty((npair, d2.ng, 2), dtype=torch.float64, device="cuda")
    path.pair_density(ctx, d2, *KB, o=o, e=e, out=Md, prec=prec)
    chi = torch.empty((d2.nfreq, d2.ng, d2.ng, 2), dtype=torch.float64, device="cuda")
    rp.rp_chi0_accumulate(ctx, d2.cell, p.iq, d2.nband, d2.energy, d2.T, *o, *e, *KB, d2.ng, Md, d2.nfreq,
                          p.freq_eV, p.delta_eV, path.weight_mode(p), prec, 0, chi)
    got = path.to_complex(chi)[:, cols][:, :, cols]
    want = oracle.chi0(M[:, cols], w)
    err = max(_rel(got[f], want[f]) for f in range(want.shape[0]))
    print(f"[fullsize] chi block prec={prec}: rel err {err:.2e}", flush=True)
    assert err < tol


def test_chi_batch_linearity_fullsize(ctx, rp, c2, d2):
    from paper_2001_02351_amd import path
    whole = path.to_complex(path.chi0(ctx, d2, kbatch=2, k0=KB[0], k1=KB[1]))
    a = path.to_complex(path.chi0(ctx, d2, kbatch=1, k0=KB[0], k1=KB[0] + 1))
    b = path.to_complex(path.chi0(ctx, d2, kbatch=1, k0=KB[0] + 1, k1=KB[1]))
    assert max(_rel(a[f] + b[f], whole[f]) for f in range(whole.shape[0])) < 1e-13
    # absorptive part of chi is negative semidefinite (real frequencies)
    for f in (3, 17):
        B = (whole[f] - whole[f].conj().T) / 2j
        assert np.linalg.eigvalsh(B).max() < 1e-10 * np.abs(B).max()


BENCH_K = (32, 48)     # one contraction launch of the bench: 16 k-points, all 40 x 200 bands


@pytest.fixture(scope="module")
def bench_launch(ctx, rp, d2):
    """chi over the bench's 16-k-point launch (128 000 pairs, 20 real
    frequencies): split-BF16 as one launch (4 000 pair steps cut into 8 FP32
    slices summed in FP64) and as eight two-k-point launches, and FP64 as one
    launch."""
    from paper_2001_02351_amd import path
    k0, k1 = BENCH_K
    print("[fullsize] bench launch: split 16-k, split 8 x 2-k, FP64 16-k", flush=True)
    one = path.to_complex(path.chi0(ctx, d2, prec=rp.RP_SPLIT_BF16, kbatch=16, k0=k0, k1=k1))
    eight = path.to_complex(path.chi0(ctx, d2, prec=rp.RP_SPLIT_BF16, kbatch=2, k0=k0, k1=k1))
    ref = path.to_complex(path.chi0(ctx, d2, prec=rp.RP_FP64, kbatch=16, k0=k0, k1=k1))
    return one, eight, ref


@pytest.fixture(scope="module")
def bench_launch_oracle(c2):
    """The oracle's chi of the same 128 000 pairs on sampled G columns: 48
    columns from the slab |m3| <= 1 of the sphere (which keeps the oracle's
    separable transform to a three-plane window), spread so that every
    128-row tile of the padded N_G holds some, and the oracle's weights."""
    p = c2
    rng = np.random.default_rng(21)
    slab = np.where(np.abs(p.gsph[:, 2]) <= 1)[0]
    cols = []
    for t in range(0, p.ng, 128):
        cand = slab[(slab >= t) & (slab < t + 128)]
        if len(cand):
            cols.append(int(rng.choice(cand)))
    rest = np.setdiff1d(slab, cols)
    cols = np.unique(np.concatenate([cols, rng.choice(rest, 48 - len(cols), replace=False)]))
    print(f"[fullsize] oracle pair densities of the bench launch on {len(cols)} columns (128 000 pairs)",
          flush=True)
    sub = _with_gsph(p, p.gsph[cols])
    M = oracle.pair_densities(sub, 0, p.nocc, p.nocc, p.nband, *BENCH_K)
    w = oracle.prob_weights(p, 0, p.nocc, p.nocc, p.nband, *BENCH_K)
    print("[fullsize] oracle chi of the bench launch on the sampled columns", flush=True)
    return cols, oracle.chi0(M, w)


def _with_gsph(p, gsph):
    from dataclasses import replace
    return replace(p, gsph=np.ascontiguousarray(gsph, dtype=np.int32))


def test_chi_bench_launch_fullsize(bench_launch, d2):
    """The split launch against eight two-k-point launches (other slicing and
    FP32 groupings) and both against the FP64 contraction of the same pair
    densities, to the split form's 1e-5; the absorptive part stays negative
    semidefinite."""
    one, eight, ref = bench_launch
    d_one = max(_rel(one[f], ref[f]) for f in range(d2.nfreq))
    d_eight = max(_rel(eight[f], ref[f]) for f in range(d2.nfreq))
    d_batch = max(_rel(one[f], eight[f]) for f in range(d2.nfreq))
    print(f"[fullsize] vs FP64: 16-k launch {d_one:.1e}, 2-k launches {d_eight:.1e}; between them {d_batch:.1e}",
          flush=True)
    assert d_one < 1e-5 and d_eight < 1e-5 and d_batch < 1e-5
    for f in (9, 19):
        ev = np.linalg.eigvalsh((one[f] - one[f].conj().T) / 2j)
        assert ev.max() < 1e-5 * abs(ev.min())


def test_chi_bench_launch_fused_equals_two_calls(ctx, rp, bench_launch, d2):
    """The bench's launch through rp_chi0_run (the pair kernels write the
    contraction's split operands) equals rp_pair_density + rp_chi0_accumulate
    (the operands prepared from FP64 M) bit for bit."""
    from paper_2001_02351_amd import path
    one, _, _ = bench_launch
    p = d2.prob
    k0, k1 = BENCH_K
    M = path.pair_density(ctx, d2, k0, k1, prec=rp.RP_SPLIT_BF16)
    chi = torch.empty((d2.nfreq, d2.ng, d2.ng, 2), dtype=torch.float64, device="cuda")
    rp.rp_chi0_accumulate(ctx, d2.cell, p.iq, d2.nband, d2.energy, d2.T, 0, p.nocc, p.nocc, p.nband, k0, k1, d2.ng,
                          M, d2.nfreq, p.freq_eV, p.delta_eV, path.weight_mode(p), rp.RP_SPLIT_BF16, 0, chi)
    rp.rp_synchronize(ctx)
    del M
    two = path.to_complex(chi)
    print(f"[fullsize] fused vs two calls: max |diff| {np.abs(one - two).max():.1e}", flush=True)
    assert np.array_equal(one, two)


def test_chi_bench_launch_against_the_oracle(bench_launch, bench_launch_oracle, d2):
    """The bench's launch (split-BF16 as one sliced launch, and FP64) against
    the oracle's Eq. chi of all 128 000 pairs on the sampled rows and columns,
    per frequency: relative Frobenius norm and largest element-wise deviation
    over the largest |chi|, FP64 1e-10 and split-BF16 1e-5."""
    one, _, ref = bench_launch
    cols, want = bench_launch_oracle
    for name, got, tol in (("FP64", ref, 1e-10), ("split-BF16", one, 1e-5)):
        blk = got[:, cols][:, :, cols]
        err = max(_rel(blk[f], want[f]) for f in range(d2.nfreq))
        print(f"[fullsize] bench launch {name} vs oracle on {len(cols)} columns: {err:.2e}", flush=True)
        assert err < tol


@pytest.fixture(scope="module")
def screened(c2):
    """A synthetic full-size chi (negative semidefinite Hermitian part plus an
    absorptive part) for two frequencies, and the oracle's eps^-1 / W."""
    p = c2
    rng = np.random.default_rng(3)
    ng = p.ng
    A = (rng.standard_normal((ng, 120)) + 1j * rng.standard_normal((ng, 120))) * 0.02
    Bm = (rng.standard_normal((ng, 60)) + 1j * rng.standard_normal((ng, 60))) * 0.01
    chi = np.stack([-(A @ A.conj().T), -(A @ A.conj().T) * 0.7 - 1j * (Bm @ Bm.conj().T)])
    print("[fullsize] oracle inversion of two 1500x1500 dielectric matrices", flush=True)
    _, einv, W = oracle.screen(p.lat, p.kmesh, p.iq, p.gsph, chi)
    return chi, einv, W


def test_screen_fullsize(ctx, rp, c2, d2, screened):
    from paper_2001_02351_amd import path
    p = c2
    chi, einv, W = screened
    chi_t = torch.from_numpy(np.ascontiguousarray(chi).view(np.float64).reshape(chi.shape + (2,))).cuda()
    e_t = torch.empty_like(chi_t)
    W_t = torch.empty_like(chi_t)
    rp.rp_screen_W(ctx, d2.cell, p.iq, d2.ng, p.gsph, 2, chi_t, e_t, W_t)
    rp.rp_synchronize(ctx)
    ge, gW = path.to_complex(e_t), path.to_complex(W_t)
    for f in range(2):
        assert _rel(ge[f], einv[f]) < 1e-10
        assert _rel(gW[f], W[f]) < 1e-10


def test_wannier_fullsize(ctx, rp, c2, d2, screened):
    from paper_2001_02351_amd import path
    p = c2
    _, einv, _ = screened
    print("[fullsize] oracle Wannier densities (10 orbitals, 48^3)", flush=True)
    rho_e = oracle.wannier_rho(p.lat, p.fft, p.kmesh, p.iq, p.phi, p.centre_frac, p.gsph)
    rho_t = oracle.wannier_rho(p.lat, p.fft, p.kmesh, p.iq, p.phi, p.centre_frac, p.gtail)
    want = oracle.wannier_W(p.lat, p.kmesh, rho_e, rho_t, einv)
    e_t = torch.from_numpy(np.ascontiguousarray(einv).view(np.float64).reshape(einv.shape + (2,))).cuda()
    Wij = torch.empty((2, p.nwan, p.nwan, 2), dtype=torch.float64, device="cuda")
    rp.rp_wannier_W(ctx, d2.cell, p.iq, p.nwan, d2.phi, p.centre_frac, d2.ng, p.gsph, p.gtail.shape[0],
                    p.gtail, 2, e_t, Wij)
    got = path.to_complex(Wij)
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-10
