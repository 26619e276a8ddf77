"""bench.py's contract on the CPU: it refuses more than one GPU before touching
any device, the committed counter summaries it reads carry the hashes of the
current kernel sources (so the roofline's traffic and the pair-stage bytes are
reported, not null), and its oracle-sample comparison computes the element-wise
and norm errors it reports (with stand-ins for the GPU calls)."""

import os
import subprocess
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

torch = pytest.importorskip("torch")


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_recorded_counters_match_the_sources():
    rec = bench.recorded_traffic()
    assert rec is not None, "profiles/k_chi_rows_traffic.md was taken on another chi_bf16.hip"
    assert rec["traffic_bytes_per_launch"] > 3.17e9 and rec["mfma_mops_per_launch"] > 0
    pc = bench.recorded_pair_counters()
    assert pc is not None, "profiles/pair_stage_hbm_counters.md was taken on another pair.hip or fft.hip"
    assert pc["pair_bytes_per_launch"] > 0.255e9


def test_oracle_sample_errors():
    nf, ng, ngs = 3, 12, 5
    rng = np.random.default_rng(0)
    full = rng.standard_normal((nf, ng, ng)) + 1j * rng.standard_normal((nf, ng, ng))
    rel = {1: 1e-6, 2: 2e-6, 0: 0.0}

    def chi0(ctx, d, prec, kbatch, k0, k1, chi):
        assert (k0, k1) == (0, 1)
        chi.copy_(torch.from_numpy(np.stack([full.real, full.imag], -1) * (1 + rel[prec])))
        return chi

    from paper_2001_02351_amd import path
    rp = types.SimpleNamespace(RP_SPLIT_BF16=1, RP_SPLIT_BF16_X6=2, RP_FP64=0, rp_synchronize=lambda c: None)
    pth = types.SimpleNamespace(chi0=chi0, to_complex=path.to_complex)
    d = types.SimpleNamespace(nfreq=nf, ng=ng, device="cpu")
    out = bench.oracle_sample_errors(rp, pth, None, d, {"chi_sample": full[:, :ngs, :ngs]})
    for name, prec in (("split_bf16", 1), ("split_bf16_x6", 2), ("fp64", 0)):
        assert out[name]["chi"] == pytest.approx(rel[prec], rel=1e-9, abs=1e-15)
        assert out[name]["chi_max_elementwise"] == pytest.approx(rel[prec], rel=1e-9, abs=1e-15)
    assert "500" not in out["sample"] and f"{ngs} x {ngs}" in out["sample"]
