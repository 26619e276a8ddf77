"""rp_chi0_accumulate_noalloc (the contraction on the library's fixed device
workspace) against rp_chi0_accumulate on the same pair densities: two calls
in a row, the second on a smaller input (fewer k-points and bands), FP64 and
split-BF16, each to the parity bar of its form (1e-10 and 1e-5, relative per
frequency, Frobenius and element-wise); a call whose workspace would exceed
the fixed array is refused before anything is enqueued."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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
def d1(rp):
    from paper_2001_02351_amd.path import DeviceInputs
    from synth import parity_workload
    return DeviceInputs(parity_workload())


def _rel(a, b):
    a, b = torch.view_as_complex(a), torch.view_as_complex(b)
    fro = max(float(torch.linalg.norm(a[f] - b[f]) / torch.linalg.norm(b[f])) for f in range(b.shape[0]))
    ew = max(float((a[f] - b[f]).abs().max() / b[f].abs().max()) for f in range(b.shape[0]))
    return fro, ew


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_the_allocating_entry_point(ctx, rp, d1, prec):
    from paper_2001_02351_amd import path
    p = d1.prob
    tol = 1e-10 if prec == 0 else 1e-5
    calls = [((0, p.nocc), (p.nocc, p.nband), (0, d1.nk)),     # the whole q-point: 12 288 pairs
             ((1, 7), (p.nocc + 2, p.nocc + 14), (5, 25))]    # smaller: 20 k x 6 x 12 bands
    for i, (o, e, k) in enumerate(calls):
        npair = (k[1] - k[0]) * (e[1] - e[0]) * (o[1] - o[0])
        M = torch.empty((npair, d1.ng, 2), dtype=torch.float64, device="cuda")
        path.pair_density(ctx, d1, *k, o=o, e=e, out=M, prec=prec)
        args = (d1.cell, p.iq, d1.nband, d1.energy, d1.T, *o, *e, *k, d1.ng, M, d1.nfreq, p.freq_eV, p.delta_eV,
                path.weight_mode(p), prec, 0)
        ref = torch.empty((d1.nfreq, d1.ng, d1.ng, 2), dtype=torch.float64, device="cuda")
        got = torch.full_like(ref, float("nan"))
        rp.rp_chi0_accumulate(ctx, *args, ref)
        print(f"[noalloc] prec={prec} call {i}: {npair} pairs", flush=True)
        rp.rp_chi0_accumulate_noalloc(ctx, *args, got)
        rp.rp_synchronize(ctx)
        fro, ew = _rel(got, ref)
        print(f"[noalloc] prec={prec} call {i}: {fro:.1e} (Frobenius), {ew:.1e} (element-wise), "
              f"identical: {bool(torch.equal(got, ref))}", flush=True)
        assert fro < tol and ew < tol
        # accumulate = 1 adds into chi
        rp.rp_chi0_accumulate_noalloc(ctx, *args[:-1], 1, got)
        rp.rp_synchronize(ctx)
        fro, ew = _rel(got, 2 * ref)
        assert fro < tol and ew < tol


def test_noalloc_refuses_beyond_the_fixed_workspace(ctx, rp, d1):
    from paper_2001_02351_amd import path
    p = d1.prob
    ng = 1000                      # 12 288 pairs x 1024 padded rows: over 128 MiB of split operands
    npair = d1.nk * p.nocc * p.nemp
    M = torch.zeros((npair, ng, 2), dtype=torch.float64, device="cuda")
    chi = torch.zeros((d1.nfreq, ng, ng, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(rp.RpError) as e:
        rp.rp_chi0_accumulate_noalloc(ctx, d1.cell, p.iq, d1.nband, d1.energy, d1.T, 0, p.nocc, p.nocc, p.nband, 0,
                                      d1.nk, ng, M, d1.nfreq, p.freq_eV, p.delta_eV, path.weight_mode(p), 1, 0, chi)
    assert e.value.status == 2 and "workspace" in str(e.value)
    rp.rp_synchronize(ctx)
    assert float(chi.abs().max()) == 0.0
