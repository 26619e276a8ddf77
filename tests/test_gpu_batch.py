"""Parity on systems of the batched uneven workload (uneven FFT grids, k meshes,
band counts and N_G; 16 imaginary frequencies with delta = 0): each system runs
through the same C ABI, one after the other.

Per system, on a band subset (8 occupied x 16 empty bands, k < 27):
* pair densities (FP64 and FP32 grids) against the oracle's direct DFT,
* tetrahedron weights on the imaginary axis against the oracle,
* chi (FP64 and split-BF16) on sampled columns against the oracle's chi0,
* chi Hermitian and negative semidefinite (real weights on the imaginary axis).
Systems 7 and 8 have odd grid edges (25, 27): one lane per FFT line in FP32,
the generic pair kernel in FP64; system 18 (30^3) has two lanes per line.
The batch entry point is checked against per-problem calls on uneven batches,
across its bounded graph pieces, and on a batch whose problems take four
different contraction forms.
"""

import numpy as np
import pytest

import oracle
from synth import batch_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# 24^3 / 2^3 k, 25^3 / 2^3 k, 36^3 / 2^3 k, 40^3 / 3^3 k, 30^3 / 3^3 k, 27^3 / 4^3 k:
# every grid edge of the workload (one, two or four lanes per FFT line)
SYSTEMS = [21, 7, 6, 4, 18, 8]


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


@pytest.mark.parametrize("s", SYSTEMS)
def test_batch_system_parity(ctx, rp, s):
    from paper_2001_02351_amd import path
    p = batch_system(s, 0)
    print(f"[batch] system {s}: grid {p.fft}, k {p.kmesh}, q {p.iq}, bands {p.nocc}+{p.nemp}, "
          f"N_G {p.ng}", flush=True)
    d = path.DeviceInputs(p)
    nk = min(d.nk, 27)          # k < 27: a bounded oracle cost on the 4^3 mesh
    o, e = (0, 8), (p.nocc, p.nocc + 16)
    M = oracle.pair_densities(p, *o, *e, 0, nk)
    w = oracle.prob_weights(p, *o, *e, 0, nk)
    # real weights on the imaginary axis (the log branch jump cancels in the
    # fourth divided difference up to rounding)
    assert np.abs(w.imag).max() < 1e-11 * np.abs(w).max()
    npair = M.shape[0]
    for prec, tol in ((rp.RP_FP64, 1e-12), (rp.RP_SPLIT_BF16, 2e-6)):
        Md = torch.empty((npair, d.ng, 2), dtype=torch.float64, device="cuda")
        path.pair_density(ctx, d, 0, nk, o=o, e=e, out=Md, prec=prec)
        assert _rel(path.to_complex(Md), M) < tol, prec
    wd = torch.empty((d.nfreq, npair, 2), dtype=torch.float64, device="cuda")
    rp.rp_weights(ctx, d.cell, p.iq, d.nband, d.energy, d.T, *o, *e, 0, nk, d.nfreq, p.freq_eV,
                  p.delta_eV, path.weight_mode(p), wd)
    assert np.max(np.abs(path.to_complex(wd) - w)) < 1e-12 * np.abs(w).max()

    rng = np.random.default_rng(s)
    cols = np.unique(np.concatenate([rng.choice(p.ng, 40, replace=False), [0, p.ng - 1]]))
    want = oracle.chi0(M[:, cols], w)
    Md = torch.empty((npair, d.ng, 2), dtype=torch.float64, device="cuda")
    for prec, tol in ((rp.RP_FP64, 1e-10), (rp.RP_SPLIT_BF16, 1e-5)):
        path.pair_density(ctx, d, 0, nk, o=o, e=e, out=Md, prec=prec)
        chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device="cuda")
        rp.rp_chi0_accumulate(ctx, d.cell, p.iq, d.nband, d.energy, d.T, *o, *e, 0, nk, d.ng, Md,
                              d.nfreq, p.freq_eV, p.delta_eV, path.weight_mode(p), prec, 0, chi)
        got = path.to_complex(chi)
        err = max(_rel(got[f][cols][:, cols], want[f]) for f in range(d.nfreq))
        print(f"[batch] system {s} prec={prec}: chi rel err {err:.2e}", flush=True)
        assert err < tol
        if prec == rp.RP_FP64:
            for f in (0, d.nfreq - 1):
                c = got[f]
                assert _rel(c, c.conj().T) < 1e-13
                ev = np.linalg.eigvalsh((c + c.conj().T) / 2)
                assert ev.max() < 1e-10 * np.abs(ev).max()


def _per_problem(ctx, rp, d, o, e, prec, kbatch, k=None):
    """chi0 of one problem through rp_pair_density + rp_chi0_accumulate, k
    batches of kbatch k-points (the reference for the batch entry point)."""
    from paper_2001_02351_amd import path
    p = d.prob
    k0, k1 = k if k else (0, d.nk)
    npk = (o[1] - o[0]) * (e[1] - e[0])
    chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device="cuda")
    M = torch.empty((kbatch * npk, d.ng, 2), dtype=torch.float64, device="cuda")
    for ka in range(k0, k1, kbatch):
        kb = min(k1, ka + kbatch)
        Mk = M[: (kb - ka) * npk]
        path.pair_density(ctx, d, ka, kb, o=o, e=e, out=Mk, prec=prec)
        rp.rp_chi0_accumulate(ctx, d.cell, p.iq, d.nband, d.energy, d.T, *o, *e, ka, kb, d.ng, Mk, d.nfreq,
                              p.freq_eV, p.delta_eV, path.weight_mode(p), prec, 0 if ka == k0 else 1, chi)
    return chi


@pytest.mark.parametrize("prec", [0, 1])
def test_chi0_batch_graph_matches_per_problem_calls(ctx, rp, prec):
    """rp_chi0_batch over uneven problems (three systems, two q-points of one,
    a k sub-range, and an empty problem) equals the per-problem calls; the
    graph is relaunched on an unchanged batch and re-captured on a changed one."""
    from paper_2001_02351_amd import path
    systems = [(21, 0), (21, 1), (7, 0), (4, 0)]
    ds = [path.DeviceInputs(batch_system(s, iq)) for s, iq in systems]
    bands = [((0, 8), (d.prob.nocc, d.prob.nocc + 16)) for d in ds]
    kr = [None, (2, 7), None, None]
    kbatch = 3
    chis = [torch.full((d.nfreq, d.ng, d.ng, 2), float("nan"), dtype=torch.float64, device="cuda")
            for d in ds]
    probs = [path.batch_problem(d, c, kbatch, o=o, e=e, k=k) for d, c, (o, e), k in zip(ds, chis, bands, kr)]
    # an empty problem (no k) clears its chi
    zero = torch.full((ds[2].nfreq, ds[2].ng, ds[2].ng, 2), 5.0, dtype=torch.float64, device="cuda")
    probs.append(path.batch_problem(ds[2], zero, kbatch, o=bands[2][0], e=bands[2][1], k=(3, 3)))
    print(f"[batch graph] prec={prec}: {len(probs)} problems", flush=True)
    rp.rp_chi0_batch(ctx, probs, prec)
    rp.rp_synchronize(ctx)
    assert float(zero.abs().max()) == 0.0
    ref = [_per_problem(ctx, rp, d, o, e, prec, kbatch, k) for d, (o, e), k in zip(ds, bands, kr)]
    for i, (c, r) in enumerate(zip(chis, ref)):
        err = _rel(c.cpu().numpy(), r.cpu().numpy())
        print(f"[batch graph] problem {i}: rel diff {err:.1e} (exact: {bool(torch.equal(c, r))})", flush=True)
        assert err <= 1e-14
    # unchanged batch: the same graph again, same result
    before = [c.clone() for c in chis]
    for c in chis:
        c.fill_(float("nan"))
    rp.rp_chi0_batch(ctx, probs, prec)
    rp.rp_synchronize(ctx)
    for c, b in zip(chis, before):
        assert torch.equal(c, b)
    # changed batch (accumulate into chi of problem 0 only): a new capture
    rp.rp_chi0_batch(ctx, [dict(probs[0], accumulate=1)], prec)
    rp.rp_synchronize(ctx)
    assert float(torch.linalg.norm(chis[0] - 2 * before[0]) / torch.linalg.norm(before[0])) <= 1e-14
    # and the oracle on sampled columns of problem 2
    d, (o, e) = ds[2], bands[2]
    M = oracle.pair_densities(d.prob, *o, *e, 0, d.nk)
    w = oracle.prob_weights(d.prob, *o, *e, 0, d.nk)
    cols = np.unique(np.concatenate([np.random.default_rng(9).choice(d.ng, 30, replace=False), [d.ng - 1]]))
    want = oracle.chi0(M[:, cols], w)
    got = path.to_complex(chis[2])
    err = max(_rel(got[f][cols][:, cols], want[f]) for f in range(d.nfreq))
    assert err < (1e-10 if prec == 0 else 1e-5)


def test_chi0_batch_rejects_bad_problems(ctx, rp):
    from paper_2001_02351_amd import path
    d = path.DeviceInputs(batch_system(21, 0))
    chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device="cuda")
    good = path.batch_problem(d, chi, 2)
    with pytest.raises(rp.RpError) as e:
        rp.rp_chi0_batch(ctx, [good, dict(good, kbatch=0)], 0)
    assert e.value.status == 2 and "problem 1" in str(e.value)
    with pytest.raises(rp.RpError) as e:
        rp.rp_chi0_batch(ctx, [dict(good, k1=d.nk + 1)], 0)
    assert e.value.status == 2 and "problem 0" in str(e.value)
    with pytest.raises(rp.RpError) as e:
        rp.rp_chi0_batch(ctx, [good], 7)
    assert e.value.status == 3
    rp.rp_chi0_batch(ctx, [], 0)   # an empty batch is a no-op


@pytest.mark.parametrize("prec", [0, 1])
def test_chi0_batch_across_graph_pieces(ctx, rp, prec):
    """A batch whose launches exceed one graph's node bound (six q-points of
    the 16^3 / 4^3 k parity system, one k-point per batch: 2 304 kernel nodes
    in FP64, 3 072 in the split form) is captured as several graphs launched
    in order; it equals the
    per-problem calls, and problem 0 meets the oracle on sampled columns
    (per frequency, relative Frobenius and element-wise)."""
    from paper_2001_02351_amd import path
    from synth import at_qpoint, parity_workload
    base = parity_workload()
    qs = ((1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1))
    ds = [path.DeviceInputs(at_qpoint(base, iq)) for iq in qs]
    kbatch = 1
    chis = [torch.full((d.nfreq, d.ng, d.ng, 2), float("nan"), dtype=torch.float64, device="cuda") for d in ds]
    probs = [path.batch_problem(d, c, kbatch) for d, c in zip(ds, chis)]
    rp.rp_chi0_batch(ctx, probs, prec)
    rp.rp_synchronize(ctx)
    graphs, nodes = rp.rp_chi0_batch_graphs(ctx)
    print(f"[batch pieces] prec={prec}: {graphs} graphs, {nodes} kernel nodes", flush=True)
    assert graphs >= 2 and nodes > 2048
    assert nodes <= graphs * (2048 + 14)
    for i, d in enumerate(ds):
        ref = _per_problem(ctx, rp, d, (0, d.prob.nocc), (d.prob.nocc, d.prob.nband), prec, kbatch)
        err = _rel(chis[i].cpu().numpy(), ref.cpu().numpy())
        print(f"[batch pieces] problem {i}: rel diff {err:.1e}", flush=True)
        assert err <= 1e-14
    # relaunch of the unchanged batch: the same graphs, the same result
    before = [c.clone() for c in chis]
    rp.rp_chi0_batch(ctx, probs, prec)
    rp.rp_synchronize(ctx)
    assert rp.rp_chi0_batch_graphs(ctx) == (graphs, nodes)
    for c, b in zip(chis, before):
        assert torch.equal(c, b)
    d = ds[0]
    p = d.prob
    M = oracle.pair_densities(p, 0, p.nocc, p.nocc, p.nband, 0, d.nk)
    w = oracle.prob_weights(p, 0, p.nocc, p.nocc, p.nband, 0, d.nk)
    cols = np.unique(np.concatenate([np.random.default_rng(3).choice(d.ng, 30, replace=False), [0, d.ng - 1]]))
    want = oracle.chi0(M[:, cols], w)
    got = path.to_complex(chis[0])[:, cols][:, :, cols]
    tol = 1e-10 if prec == 0 else 1e-5
    fro = max(_rel(got[f], want[f]) for f in range(d.nfreq))
    ew = max(np.abs(got[f] - want[f]).max() / np.abs(want[f]).max() for f in range(d.nfreq))
    print(f"[batch pieces] problem 0 vs oracle: {fro:.1e} (Frobenius), {ew:.1e} (element-wise)", flush=True)
    assert fro < tol and ew < tol


@pytest.mark.parametrize("prec", [1, 2])
def test_chi0_batch_mixed_contraction_forms(ctx, rp, prec):
    """One rp_chi0_batch call whose problems take different contraction forms:
    16 imaginary frequencies (Hermitian, 32-row strips for eight), 12
    (Hermitian, 64-row strips for four), 6 (Hermitian, 128 x 128 tiles of the
    upper triangle) and 8 real frequencies with delta > 0 (complex weights,
    64-row strips over the whole matrix), split-BF16 and x6: each problem
    equals its per-problem calls, and two of them the oracle on sampled
    columns."""
    import dataclasses

    from paper_2001_02351_amd import path
    from synth import make_problem
    p16 = batch_system(21, 0)
    p12 = dataclasses.replace(batch_system(7, 0), freq_eV=batch_system(7, 0).freq_eV[:12])
    p6 = dataclasses.replace(batch_system(4, 0), freq_eV=batch_system(4, 0).freq_eV[:6])
    preal = make_problem(name="mixed", a_bohr=7.26, fft=(16, 16, 16), kmesh=(2, 2, 2), iq=(1, 0, 0), nocc=8,
                         nemp=24, gpsi=2.4, ng=200, freq_eV=np.linspace(0.0, 20.0, 8), delta_eV=0.1, seed=43)
    ds = [path.DeviceInputs(p) for p in (p16, p12, p6, preal)]
    assert [d.nfreq for d in ds] == [16, 12, 6, 8]
    bands = [((0, 8), (d.prob.nocc, d.prob.nocc + 16)) for d in ds]
    kbatch = 3
    chis = [torch.full((d.nfreq, d.ng, d.ng, 2), float("nan"), dtype=torch.float64, device="cuda") for d in ds]
    probs = [path.batch_problem(d, c, kbatch, o=o, e=e) for d, c, (o, e) in zip(ds, chis, bands)]
    print(f"[batch mixed] {len(probs)} problems, N_G {[d.ng for d in ds]}", flush=True)
    rp.rp_chi0_batch(ctx, probs, prec)
    rp.rp_synchronize(ctx)
    for i, (d, (o, e), c) in enumerate(zip(ds, bands, chis)):
        ref = _per_problem(ctx, rp, d, o, e, prec, kbatch)
        rp.rp_synchronize(ctx)
        print(f"[batch mixed] problem {i}: exact {bool(torch.equal(c, ref))}", flush=True)
        assert _rel(c.cpu().numpy(), ref.cpu().numpy()) <= 1e-14
    for i in (1, 3):
        d, (o, e) = ds[i], bands[i]
        M = oracle.pair_densities(d.prob, *o, *e, 0, d.nk)
        w = oracle.prob_weights(d.prob, *o, *e, 0, d.nk)
        cols = np.unique(np.concatenate([np.random.default_rng(11).choice(d.ng, 24, replace=False), [d.ng - 1]]))
        want = oracle.chi0(M[:, cols], w)
        got = path.to_complex(chis[i])
        err = max(_rel(got[f][cols][:, cols], want[f]) for f in range(d.nfreq))
        print(f"[batch mixed] problem {i}: vs oracle {err:.1e}", flush=True)
        assert err < 1e-5
