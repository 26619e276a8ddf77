"""One q-point through the library: pair densities and chi0 per k batch, then
eps^-1 / W, then W_ij.  Orchestration and device-memory plumbing only; every
step runs in librp.so.

`prob` is any object with the attributes of a plane-wave problem: lat, fft,
kmesh, iq, nocc, nemp, npw, miller, coef, energy_eV, T, gsph, gtail,
freq_eV, delta_eV and optionally phi, centre_frac.
"""

from __future__ import annotations

from typing import Optional

import numpy as np

from . import _rp


class DeviceInputs:
    """Device copies of a problem's large arrays (torch tensors)."""

    def __init__(self, prob, device: int = 0):
        import torch
        dev = torch.device("cuda", device)
        self.prob = prob
        self.cell = _rp.make_cell(prob.lat, prob.fft, prob.kmesh)
        self.miller = torch.from_numpy(np.ascontiguousarray(prob.miller, dtype=np.int32)).to(dev)
        coef = np.ascontiguousarray(prob.coef, dtype=np.complex128)
        self.coef = torch.from_numpy(coef.view(np.float64)).to(dev)
        self.energy = torch.from_numpy(np.ascontiguousarray(prob.energy_eV, dtype=np.float64)).to(dev)
        self.T = None if prob.T is None else torch.from_numpy(np.ascontiguousarray(prob.T, np.float64)).to(dev)
        self.phi = None
        if getattr(prob, "phi", None) is not None:
            self.phi = torch.from_numpy(np.ascontiguousarray(prob.phi, dtype=np.float64)).to(dev)
        self.mmax = np.abs(np.asarray(prob.miller)).max(axis=(0, 1)).astype(np.int32)
        self.nk = int(np.prod(prob.kmesh))
        self.nband = prob.nocc + prob.nemp
        self.ng = int(prob.gsph.shape[0])
        self.nfreq = int(len(prob.freq_eV))
        self.device = dev

    def at_q(self, prob_q) -> "DeviceInputs":
        """A view for another q-point of the same system (prob_q: the same
        band data with that q's iq and G lists); the device arrays are
        shared, nothing is copied."""
        import copy
        v = copy.copy(self)
        v.prob = prob_q
        v.ng = int(prob_q.gsph.shape[0])
        return v


def weight_mode(prob) -> int:
    return _rp.RP_W_SAMPLING if int(np.prod(prob.kmesh)) == 1 else _rp.RP_W_TETRA


def pair_density(ctx, d: DeviceInputs, k0: int, k1: int, o=None, e=None, out=None,
                 prec: int = _rp.RP_FP64):
    import torch
    p = d.prob
    o0, o1 = o if o else (0, p.nocc)
    e0, e1 = e if e else (p.nocc, p.nocc + p.nemp)
    npair = (k1 - k0) * (e1 - e0) * (o1 - o0)
    if out is None:
        out = torch.empty((npair, d.ng, 2), dtype=torch.float64, device=d.device)
    _rp.rp_pair_density(ctx, d.cell, p.iq, d.nband, p.miller.shape[1], p.npw, d.mmax, d.miller, d.coef,
                        o0, o1, e0, e1, k0, k1, d.ng, p.gsph, prec, out)
    return out


def weights(ctx, d: DeviceInputs, k0, k1, o=None, e=None, mode: Optional[int] = None):
    import torch
    p = d.prob
    o0, o1 = o if o else (0, p.nocc)
    e0, e1 = e if e else (p.nocc, p.nocc + p.nemp)
    npair = (k1 - k0) * (e1 - e0) * (o1 - o0)
    w = torch.empty((d.nfreq, npair, 2), dtype=torch.float64, device=d.device)
    _rp.rp_weights(ctx, d.cell, p.iq, d.nband, d.energy, d.T, o0, o1, e0, e1, k0, k1, d.nfreq,
                   p.freq_eV, p.delta_eV, weight_mode(p) if mode is None else mode, w)
    return w


def chi0(ctx, d: DeviceInputs, prec: int = _rp.RP_FP64, kbatch: int = 1, k0: int = 0,
         k1: Optional[int] = None, chi=None):
    """chi0 over k in [k0, k1) (all bands): one rp_chi0_run call, the pair
    densities of kbatch k-points at a time feeding the contraction (in the
    split forms as the contraction's operands, with no FP64 M)."""
    import torch
    k1 = d.nk if k1 is None else k1
    if chi is None:
        chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device=d.device)
    _rp.rp_chi0_run(ctx, batch_problem(d, chi, kbatch, k=(k0, k1)), prec)
    return chi


def batch_problem(d: DeviceInputs, chi, kbatch: int = 1, o=None, e=None, k=None, accumulate: int = 0):
    """The rp_chi0_batch description of chi0 of one problem (all bands and k
    unless band or k ranges are given)."""
    p = d.prob
    o0, o1 = o if o else (0, p.nocc)
    e0, e1 = e if e else (p.nocc, p.nocc + p.nemp)
    k0, k1 = k if k else (0, d.nk)
    return dict(cell=d.cell, iq=p.iq, nband=d.nband, npw_max=p.miller.shape[1], npw=p.npw, mmax=d.mmax,
                miller=d.miller, coef=d.coef, energy_eV=d.energy, T=d.T, o0=o0, o1=o1, e0=e0, e1=e1, k0=k0,
                k1=k1, ng=d.ng, gsph=p.gsph, nfreq=d.nfreq, freq_eV=p.freq_eV, delta_eV=p.delta_eV,
                wm=weight_mode(p), kbatch=kbatch, accumulate=accumulate, chi=chi)


def chi0_batch(ctx, ds, prec: int = _rp.RP_FP64, kbatch: int = 1, chis=None):
    """chi0 of several problems (DeviceInputs) in one rp_chi0_batch call."""
    import torch
    if chis is None:
        chis = [torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device=d.device) for d in ds]
    _rp.rp_chi0_batch(ctx, [batch_problem(d, c, kbatch) for d, c in zip(ds, chis)], prec)
    return chis


def chi0_head(ctx, d: DeviceInputs, qhat, prec: int = _rp.RP_FP64, kbatch: int = 1):
    """chi at q -> 0 (iq = 0) over all k and bands with G = 0 first in the
    sphere and the head density of direction qhat in its row and column.
    Returns (chi, G list)."""
    import torch
    p = d.prob
    if tuple(int(x) for x in p.iq) != (0, 0, 0):
        raise ValueError("the q -> 0 head needs iq = 0")
    gaug = np.ascontiguousarray(np.concatenate([np.zeros((1, 3), np.int32), np.asarray(p.gsph, np.int32)]))
    ng = int(gaug.shape[0])
    npk = p.nocc * p.nemp
    chi = torch.empty((d.nfreq, ng, ng, 2), dtype=torch.float64, device=d.device)
    M = torch.empty((kbatch * npk, ng, 2), dtype=torch.float64, device=d.device)
    o0, o1, e0, e1 = 0, p.nocc, p.nocc, p.nocc + p.nemp
    for ka in range(0, d.nk, kbatch):
        kb = min(d.nk, ka + kbatch)
        Mk = M[: (kb - ka) * npk]
        _rp.rp_pair_density(ctx, d.cell, p.iq, d.nband, p.miller.shape[1], p.npw, d.mmax, d.miller, d.coef,
                            o0, o1, e0, e1, ka, kb, ng, gaug, prec, Mk)
        _rp.rp_head_density(ctx, d.cell, d.nband, p.miller.shape[1], p.npw, d.miller, d.coef, d.energy,
                            o0, o1, e0, e1, ka, kb, qhat, ng, 0, Mk)
        _rp.rp_chi0_accumulate(ctx, d.cell, p.iq, d.nband, d.energy, d.T, o0, o1, e0, e1, ka, kb, ng, Mk,
                               d.nfreq, p.freq_eV, p.delta_eV, weight_mode(p), prec, 0 if ka == 0 else 1, chi)
    return chi, gaug


def screen_head(ctx, d: DeviceInputs, chi, gaug, drude=None):
    """eps^-1 at q -> 0 with head and wings, and the optical quantities
    {Re eps_M, Im eps_M, L, Re sigma, R} per frequency.  drude = (wq_eV2,
    delta_eV) adds the intraband term -wq / (w (w + i delta)) to the head for
    this call (wq = qhat . Omega . qhat from rp_plasma_frequency)."""
    import torch
    p = d.prob
    einv = torch.empty_like(chi)
    optics = torch.empty((d.nfreq, 5), dtype=torch.float64, device=d.device)
    if drude is not None:
        _rp.rp_set_drude(ctx, *drude)
    try:
        _rp.rp_screen_head(ctx, d.cell, int(gaug.shape[0]), gaug, d.nfreq, p.freq_eV, chi, einv, optics)
    finally:
        if drude is not None:
            _rp.rp_set_drude(ctx, 0.0, 0.0)
    return einv, optics


def plasma_tensor(ctx, d: DeviceInputs, b0: int, b1: int, ef_eV: float, crpa: bool = False):
    """The intraband plasma tensor (eV^2, 3 x 3) of bands [b0, b1) at E_F."""
    p = d.prob
    return _rp.rp_plasma_frequency(ctx, d.cell, d.nband, p.miller.shape[1], p.npw, d.miller, d.coef, d.energy,
                                   d.T if crpa else None, b0, b1, ef_eV)


def screen(ctx, d: DeviceInputs, chi, want_eps_inv: bool = True, want_W: bool = True):
    import torch
    p = d.prob
    einv = torch.empty_like(chi) if want_eps_inv else None
    W = torch.empty_like(chi) if want_W else None
    _rp.rp_screen_W(ctx, d.cell, p.iq, d.ng, p.gsph, d.nfreq, chi, einv, W)
    return einv, W


def wannier(ctx, d: DeviceInputs, eps_inv):
    import torch
    p = d.prob
    nwan = int(p.phi.shape[0])
    Wij = torch.empty((d.nfreq, nwan, nwan, 2), dtype=torch.float64, device=d.device)
    gt = p.gtail if p.gtail is not None else np.zeros((0, 3), np.int32)
    _rp.rp_wannier_W(ctx, d.cell, p.iq, nwan, d.phi, p.centre_frac, d.ng, p.gsph, int(gt.shape[0]), gt,
                     d.nfreq, eps_inv, Wij)
    return Wij


def qterm(ctx, d: DeviceInputs, eps_inv, glist, R, out: dict, accumulate: int):
    """Adds this q-point's term of the q-sums of U, J, V, X into out
    (device tensors, any subset of the keys); glist indexes eps_inv (G = 0
    first at q = 0)."""
    p = d.prob
    gt = p.gtail if p.gtail is not None else np.zeros((0, 3), np.int32)
    _rp.rp_wannier_qterm(ctx, d.cell, p.iq, int(p.phi.shape[0]), d.phi, p.centre_frac, R, int(len(glist)), glist,
                         int(gt.shape[0]), gt, d.nfreq, eps_inv, accumulate, **out)


def interaction(ctx, d: DeviceInputs, R, problem_at, prec: int = _rp.RP_FP64, kbatch: int = 1,
                qhat=(1.0, 0.0, 0.0), want=("U", "J", "V", "X")):
    """U, J (complex [nfreq][nR][nwan][nwan]) and V, X ([nR][nwan][nwan]) of
    Eqs. matrix_U, matrix_J, matrix_V, matrix_X summed over the whole q mesh:
    at every q chi0, eps^-1 and that q's term; at q = 0 through the head
    path (G = 0 first, head density along qhat, eps^-1 with head and wings).
    problem_at(iq) gives the system at q = iq/K (same band data, that q's G
    lists; at q = 0 without G = 0).  Returns device tensors."""
    import torch
    p = d.prob
    R = np.ascontiguousarray(np.asarray(R, np.int32).reshape(-1, 3))
    nw = int(p.phi.shape[0])
    shapes = dict(U=(d.nfreq, len(R), nw, nw, 2), J=(d.nfreq, len(R), nw, nw, 2), V=(len(R), nw, nw, 2),
                  X=(len(R), nw, nw, 2))
    out = {k: torch.empty(shapes[k], dtype=torch.float64, device=d.device) for k in want}
    first = True
    for iq in np.ndindex(*p.kmesh):
        dq = d.at_q(problem_at(iq))
        if iq == (0, 0, 0):
            chi, glist = chi0_head(ctx, dq, qhat, prec=prec, kbatch=kbatch)
            einv, _ = screen_head(ctx, dq, chi, glist)
        else:
            chi = chi0(ctx, dq, prec=prec, kbatch=kbatch)
            einv, _ = screen(ctx, dq, chi, want_W=False)
            glist = dq.prob.gsph
        qterm(ctx, dq, einv, glist, R, out, 0 if first else 1)
        first = False
    return out


def run_q(ctx, d: DeviceInputs, prec: int = _rp.RP_FP64, kbatch: int = 1):
    """a1..a10 for one q-point; returns device tensors (complex as [..., 2])."""
    chi = chi0(ctx, d, prec=prec, kbatch=kbatch)
    einv, W = screen(ctx, d, chi)
    out = dict(chi=chi, eps_inv=einv, W=W)
    if d.phi is not None:
        out["Wij"] = wannier(ctx, d, einv)
    return out


def _save_atomic(path: str, obj) -> None:
    """Writes a numpy array (.npy format) or a JSON-ready dict to path + ".tmp"
    and renames it over path, so that an interrupted save never leaves a
    partial file under the final name."""
    import json
    import os
    tmp = path + ".tmp"
    if isinstance(obj, np.ndarray):
        with open(tmp, "wb") as f:
            np.save(f, obj)
    else:
        with open(tmp, "w") as f:
            json.dump(obj, f)
    os.replace(tmp, path)


def _fingerprint(p) -> str:
    """SHA-256 of a problem's small inputs (frequencies, broadening, G list
    and tail, k mesh, band energies, cRPA T), so that a resume with other
    inputs of the same sizes is refused; the plane-wave coefficients are not
    included."""
    import hashlib
    h = hashlib.sha256()
    for a in (p.freq_eV, np.array([p.delta_eV], np.float64), p.gsph, getattr(p, "gtail", None), p.kmesh,
              p.energy_eV, p.T):
        if a is not None:
            a = np.ascontiguousarray(np.asarray(a))
            h.update(str(a.dtype).encode() + str(a.shape).encode())
            h.update(a.tobytes())
    return h.hexdigest()


def run_q_checkpointed(ctx, d: DeviceInputs, out_dir: str, prec: int = _rp.RP_FP64, kbatch: int = 1,
                       every: int = 1, stop_after: Optional[int] = None):
    """run_q with its results kept in out_dir (the per-q result directories
    of the paper's chi calculation): chi.npy, eps_inv.npy, W.npy and, with
    Wannier orbitals, Wij.npy (complex128), then done.json.

    The chi0 accumulation is checkpointed every `every` k batches
    (chi_partial.npy and progress.json with the next k-point); a later call
    with the same out_dir and the same parameters resumes after the last
    checkpoint (rp_chi0_run with accumulate = 1 on the restored chi, the
    same sums in the same order, so the results are those of an
    uninterrupted run), and a finished q-point is read back, not recomputed;
    other parameters or inputs (sizes, or the fingerprint of _fingerprint)
    raise ValueError.
    stop_after (a count of k batches) returns None once that many batches
    have been checkpointed in this call, as an interrupted run would leave
    out_dir.  Returns a dict of host arrays and "source": "computed",
    "resumed" or "files"."""
    import json
    import os

    import torch
    os.makedirs(out_dir, exist_ok=True)
    p = d.prob
    keys = ["chi", "eps_inv", "W"] + (["Wij"] if d.phi is not None else [])
    meta = dict(prec=int(prec), kbatch=int(kbatch), nk=d.nk, ng=d.ng, nfreq=d.nfreq,
                iq=[int(x) for x in p.iq], nocc=int(p.nocc), nemp=int(p.nemp), inputs=_fingerprint(p))
    done = os.path.join(out_dir, "done.json")
    if os.path.exists(done):
        with open(done) as f:
            if json.load(f) != meta:
                raise ValueError(f"{out_dir} holds a q-point computed with other parameters")
        out = {k: np.load(os.path.join(out_dir, k + ".npy")) for k in keys}
        out["source"] = "files"
        return out
    prog = os.path.join(out_dir, "progress.json")
    part = os.path.join(out_dir, "chi_partial.npy")
    chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device=d.device)
    k = 0
    source = "computed"
    if os.path.exists(prog):
        with open(prog) as f:
            saved = json.load(f)
        if {x: saved.get(x) for x in meta} != meta:
            raise ValueError(f"{out_dir} holds a partial chi0 computed with other parameters")
        k = int(saved["k_next"])
        host = np.load(part)
        chi.copy_(torch.from_numpy(np.ascontiguousarray(host).view(np.float64).reshape(chi.shape)))
        source = "resumed"
    step = max(1, every) * kbatch
    batches = 0
    while k < d.nk:
        k1 = min(d.nk, k + step)
        _rp.rp_chi0_run(ctx, batch_problem(d, chi, kbatch, k=(k, k1), accumulate=0 if k == 0 else 1), prec)
        _save_atomic(part, to_complex(chi))
        _save_atomic(prog, dict(meta, k_next=k1))
        k = k1
        batches += 1
        if stop_after is not None and batches >= stop_after and k < d.nk:
            return None
    einv, W = screen(ctx, d, chi)
    res = dict(chi=to_complex(chi), eps_inv=to_complex(einv), W=to_complex(W))
    if d.phi is not None:
        res["Wij"] = to_complex(wannier(ctx, d, einv))
    for key in keys:
        _save_atomic(os.path.join(out_dir, key + ".npy"), res[key])
    _save_atomic(done, meta)
    for f in (part, prog):
        os.remove(f)
    res["source"] = source
    return res


def run_qpoints(ctx, ds, root: str, prec: int = _rp.RP_FP64, kbatch: int = 1, every: int = 1):
    """run_q_checkpointed for several q-points (DeviceInputs), in
    root/q001, root/q002, ...; q-points already finished are read back and
    an interrupted one resumes.  Returns the list of result dicts."""
    import os
    return [run_q_checkpointed(ctx, d, os.path.join(root, f"q{i + 1:03d}"), prec=prec, kbatch=kbatch, every=every)
            for i, d in enumerate(ds)]


def to_complex(t) -> np.ndarray:
    """Device [..., 2] float64 tensor -> host complex128 array."""
    a = t.detach().cpu().numpy()
    return np.ascontiguousarray(a).view(np.complex128)[..., 0]
