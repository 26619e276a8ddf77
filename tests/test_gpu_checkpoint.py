"""Per-q checkpoint and resume (path.run_q_checkpointed, path.run_qpoints).

On a 16^3 problem with two Wannier orbitals (8 k-points, k batches of 2,
N_G = 200, 6 real frequencies), split-BF16 and FP64:
* a run stopped from the host after two k batches leaves chi_partial.npy and
  progress.json (next k-point 4) and no results;
* the next call resumes there and its chi, eps^-1, W and W_ij equal those
  of an uninterrupted run_q bit for bit;
* a third call reads the finished q-point back without computing;
* a call with other parameters (k batch size) on a finished or a partial
  q-point raises ValueError;
* run_qpoints over two q-points writes q001 and q002 and resumes an
  interrupted second q-point.
"""

import json
import os

import numpy as np
import pytest

from synth import make_problem

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


def _problem(iq=(1, 0, 0)):
    return make_problem(name="ckpt", a_bohr=7.26, fft=(16, 16, 16), kmesh=(2, 2, 2), iq=iq, nocc=8, nemp=24,
                        gpsi=2.4, ng=200, freq_eV=np.linspace(0.0, 20.0, 6), delta_eV=0.1, nwan=2, seed=37)


@pytest.mark.parametrize("prec", [0, 1])
def test_resume_equals_uninterrupted(ctx, rp, prec, tmp_path):
    from paper_2001_02351_amd import path
    d = path.DeviceInputs(_problem())
    ref = {k: path.to_complex(v) for k, v in path.run_q(ctx, d, prec=prec, kbatch=2).items()}
    out = str(tmp_path / "q001")
    print(f"[ckpt] prec={prec}: interrupted run", flush=True)
    assert path.run_q_checkpointed(ctx, d, out, prec=prec, kbatch=2, stop_after=2) is None
    with open(os.path.join(out, "progress.json")) as f:
        assert json.load(f)["k_next"] == 4
    assert os.path.exists(os.path.join(out, "chi_partial.npy"))
    assert not os.path.exists(os.path.join(out, "done.json"))
    print(f"[ckpt] prec={prec}: resume", flush=True)
    res = path.run_q_checkpointed(ctx, d, out, prec=prec, kbatch=2)
    assert res["source"] == "resumed"
    for key in ("chi", "eps_inv", "W", "Wij"):
        assert np.array_equal(res[key], ref[key]), key
    assert sorted(os.listdir(out)) == ["W.npy", "Wij.npy", "chi.npy", "done.json", "eps_inv.npy"]
    again = path.run_q_checkpointed(ctx, d, out, prec=prec, kbatch=2)
    assert again["source"] == "files"
    for key in ("chi", "eps_inv", "W", "Wij"):
        assert np.array_equal(again[key], ref[key]), key
    with pytest.raises(ValueError):
        path.run_q_checkpointed(ctx, d, out, prec=prec, kbatch=4)
    part = str(tmp_path / "partial")
    assert path.run_q_checkpointed(ctx, d, part, prec=prec, kbatch=2, stop_after=1) is None
    with pytest.raises(ValueError):
        path.run_q_checkpointed(ctx, d, part, prec=prec, kbatch=4)


def test_run_qpoints_resumes(ctx, rp, tmp_path):
    from paper_2001_02351_amd import path
    ds = [path.DeviceInputs(_problem((1, 0, 0))), path.DeviceInputs(_problem((0, 1, 1)))]
    root = str(tmp_path / "eps")
    print("[ckpt] first q-point whole, second interrupted", flush=True)
    assert path.run_q_checkpointed(ctx, ds[0], os.path.join(root, "q001"), prec=1, kbatch=2)["source"] == "computed"
    assert path.run_q_checkpointed(ctx, ds[1], os.path.join(root, "q002"), prec=1, kbatch=2, stop_after=3) is None
    res = path.run_qpoints(ctx, ds, root, prec=1, kbatch=2)
    assert [r["source"] for r in res] == ["files", "resumed"]
    for d, r in zip(ds, res):
        ref = path.to_complex(path.run_q(ctx, d, prec=1, kbatch=2)["Wij"])
        assert np.array_equal(r["Wij"], ref)
