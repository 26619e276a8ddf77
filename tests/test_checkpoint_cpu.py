"""Host logic of the per-q checkpoint and resume (path.run_q_checkpointed) on
the CPU: the two library calls it makes (rp_chi0_run, rp_screen_W) are
replaced by stand-ins on CPU tensors that add a k-dependent term per k-point
into chi (honouring accumulate) and derive eps^-1 and W from chi.  Checked:
an interrupted run leaves progress.json and chi_partial.npy, the resumed run
equals an uninterrupted one, a finished q-point is read back, a left-over
temporary file is ignored, and other parameters or inputs (k batch size,
broadening) raise ValueError.  The GPU path itself is tested in
tests/test_gpu_checkpoint.py."""

import json
import os
import types

import numpy as np
import pytest

from paper_2001_02351_amd import path
from synth import make_problem

torch = pytest.importorskip("torch")


def _fake_chi0_run(ctx, prob, prec):
    chi = prob["chi"]
    nf, ng = chi.shape[0], chi.shape[1]
    # integer values: the sums are exact in any order, like the library's
    # per-k-batch sums are identical whatever the calls' k ranges
    base = torch.arange(nf * ng * ng * 2, dtype=torch.float64).reshape(chi.shape)
    add = sum((k + 1) * base + k * k for k in range(prob["k0"], prob["k1"]))
    if prob["k1"] == prob["k0"]:
        add = torch.zeros_like(chi)
    if prob["accumulate"]:
        chi += add
    else:
        chi.copy_(add)


def _fake_screen(ctx, cell, iq, ng, gsph, nfreq, chi, einv, W):
    if einv is not None:
        einv.copy_(2.0 * chi)
    if W is not None:
        W.copy_(3.0 * chi + 1.0)


def _inputs(p):
    return types.SimpleNamespace(prob=p, cell=None, miller=None, coef=None, energy=None, T=None, mmax=None,
                                 phi=None, nk=int(np.prod(p.kmesh)), nband=p.nocc + p.nemp,
                                 ng=int(p.gsph.shape[0]), nfreq=int(len(p.freq_eV)), device="cpu")


@pytest.fixture
def fake_lib(monkeypatch):
    monkeypatch.setattr(path._rp, "rp_chi0_run", _fake_chi0_run)
    monkeypatch.setattr(path._rp, "rp_screen_W", _fake_screen)


def _problem(delta=0.1):
    return make_problem(name="ckc", a_bohr=7.26, fft=(12, 12, 12), kmesh=(2, 2, 2), iq=(1, 0, 0), nocc=3, nemp=4,
                        gpsi=2.0, ng=19, freq_eV=np.array([0.0, 3.0, 8.0]), delta_eV=delta, seed=2)


def test_checkpoint_host_logic(fake_lib, tmp_path):
    d = _inputs(_problem())
    whole = path.run_q_checkpointed(None, d, str(tmp_path / "whole"), prec=1, kbatch=2, every=4)
    assert whole["source"] == "computed"
    out = str(tmp_path / "q001")
    assert path.run_q_checkpointed(None, d, out, prec=1, kbatch=2, stop_after=1) is None
    with open(os.path.join(out, "progress.json")) as f:
        assert json.load(f)["k_next"] == 2
    assert path.run_q_checkpointed(None, d, out, prec=1, kbatch=2, stop_after=1) is None
    with open(os.path.join(out, "progress.json")) as f:
        assert json.load(f)["k_next"] == 4
    # a save interrupted after its temporary file was written
    open(os.path.join(out, "chi_partial.npy.tmp"), "wb").write(b"partial")
    res = path.run_q_checkpointed(None, d, out, prec=1, kbatch=2)
    assert res["source"] == "resumed"
    for key in ("chi", "eps_inv", "W"):
        assert np.array_equal(res[key], whole[key]), key
    assert np.array_equal(res["eps_inv"], 2.0 * res["chi"])
    back = path.run_q_checkpointed(None, d, out, prec=1, kbatch=2)
    assert back["source"] == "files"
    for key in ("chi", "eps_inv", "W"):
        assert np.array_equal(back[key], whole[key]), key
    with pytest.raises(ValueError):
        path.run_q_checkpointed(None, d, out, prec=1, kbatch=4)
    with pytest.raises(ValueError):
        path.run_q_checkpointed(None, _inputs(_problem(delta=0.2)), out, prec=1, kbatch=2)
    part = str(tmp_path / "partial")
    assert path.run_q_checkpointed(None, d, part, prec=1, kbatch=2, stop_after=1) is None
    with pytest.raises(ValueError):
        path.run_q_checkpointed(None, _inputs(_problem(delta=0.2)), part, prec=1, kbatch=2)
    with pytest.raises(ValueError):
        path.run_q_checkpointed(None, d, part, prec=0, kbatch=2)


def test_run_qpoints_layout(fake_lib, tmp_path):
    ds = [_inputs(_problem()), _inputs(_problem(delta=0.2))]
    res = path.run_qpoints(None, ds, str(tmp_path / "eps"), prec=1, kbatch=3)
    assert [r["source"] for r in res] == ["computed", "computed"]
    assert sorted(os.listdir(tmp_path / "eps")) == ["q001", "q002"]
    again = path.run_qpoints(None, ds, str(tmp_path / "eps"), prec=1, kbatch=3)
    assert [r["source"] for r in again] == ["files", "files"]
