"""Autotuner of the library's launch shapes per size class.

Size classes are N_G buckets x FFT-edge buckets.  For each class the tuner
times the candidate launch shapes on synthetic inputs of the class's upper
sizes (random coefficients and energies: only the shapes matter for timing)
and keeps the fastest (the library's default shape unless a candidate beats
it by more than 1%):

* the split-BF16 contraction (chi_kernel form, chi_nw frequencies per
  workgroup, chi_fill workgroups aimed for by slicing the pair steps): timed
  per N_G bucket on one contraction of the samples' first k batch (or of
  about 40 000 pairs with 16 imaginary frequencies for the synthetic classes);
* the u-grid transforms (fft_lines per workgroup): timed per edge bucket
  with the stage timer of the u-grid kernels.

The table goes to a JSON file; Context installs it through rp_set_tuning.
Run on the target GPU:  python -m paper_2001_02351_amd.autotune --out FILE
"""

from __future__ import annotations

import argparse
import json
import math
import time
from typing import Optional

import numpy as np

from . import _rp

# a candidate replaces the library's default shape only when it is faster by
# more than this fraction (timings of equal shapes differ by about that much)
MARGIN = 0.01
CHI_DEFAULT = (0, 2, 1024)
FFT_DEFAULT = 0

NG_BUCKETS = (512, 768, 1024, 1200)
GRID_BUCKETS = (27, 32, 40)
CHI_CANDIDATES = tuple((kern, nw, fill) for kern in (0, 1, 2) for nw in (1, 2)
                       for fill in (0, 256, 512, 1024, 2048, 4096, 8192) if not (kern == 2 and nw == 2))
FFT_CANDIDATES = (0, 4, 8, 16, 32)


class _ClassProblem:
    """Inputs of one size class on a cubic cell (a = 7.2613 bohr x edge/48)."""

    def __init__(self, edge: int, ng: int, nocc: int = 32, nemp: int = 160, kedge: int = 2,
                 nfreq: int = 16, seed: int = 0):
        rng = np.random.default_rng(seed)
        a = 7.261273 * edge / 48.0
        self.lat = np.eye(3) * a
        self.fft = (edge, edge, edge)
        self.kmesh = (kedge, kedge, kedge)
        self.iq = (0, 0, 1)
        self.nocc, self.nemp = nocc, nemp
        self.nk = kedge ** 3
        nband = nocc + nemp
        npw = max(300, int(1.25 * nband))
        ball = _ball(npw)
        self.npw = np.full(self.nk, npw, np.int32)
        self.miller = np.ascontiguousarray(np.broadcast_to(ball, (self.nk, npw, 3)), dtype=np.int32)
        self.mmax = np.abs(ball).max(axis=0).astype(np.int32)
        c = rng.standard_normal((self.nk, nband, npw)) + 1j * rng.standard_normal((self.nk, nband, npw))
        self.coef = (c / math.sqrt(2 * npw)).astype(np.complex128)
        e = np.empty((self.nk, nband))
        e[:, :nocc] = np.sort(rng.uniform(-8.0, -1.0, (self.nk, nocc)), axis=1)
        e[:, nocc:] = np.sort(rng.uniform(1.0, 20.0, (self.nk, nemp)), axis=1)
        self.energy = e
        q = np.array(self.iq, float) / kedge
        cand = _ball(4 * ng)
        order = np.argsort(np.linalg.norm(cand + q, axis=1), kind="stable")
        self.gsph = np.ascontiguousarray(cand[order[:ng]], dtype=np.int32)
        self.freq = 1j * np.concatenate([[0.0], np.geomspace(0.1, 100.0, nfreq - 1)])
        self.ng = ng


def _ball(n: int) -> np.ndarray:
    """The n integer vectors of smallest norm (ties in lexicographic order)."""
    r = int(math.ceil((3.0 * n / (4.0 * math.pi)) ** (1.0 / 3.0))) + 2
    ax = np.arange(-r, r + 1)
    m = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], (m * m).sum(axis=1)))
    return np.ascontiguousarray(m[order[:n]], dtype=np.int32)


class _Device:
    def __init__(self, p: _ClassProblem):
        import torch
        self.p = p
        self.cell = _rp.make_cell(p.lat, p.fft, p.kmesh)
        self.miller = torch.from_numpy(p.miller).cuda()
        self.coef = torch.from_numpy(p.coef.view(np.float64)).cuda()
        self.energy = torch.from_numpy(p.energy).cuda()

    def pair(self, ctx, k0, k1, M, prec):
        p = self.p
        _rp.rp_pair_density(ctx, self.cell, p.iq, p.nocc + p.nemp, p.miller.shape[1], p.npw, p.mmax,
                            self.miller, self.coef, 0, p.nocc, p.nocc, p.nocc + p.nemp, k0, k1, p.ng, p.gsph,
                            prec, M)

    def chi(self, ctx, M, chi, prec):
        p = self.p
        _rp.rp_chi0_accumulate(ctx, self.cell, p.iq, p.nocc + p.nemp, self.energy, None, 0, p.nocc, p.nocc,
                               p.nocc + p.nemp, 0, p.nk, p.ng, M, len(p.freq), p.freq, 0.0,
                               _rp.RP_W_TETRA, prec, 0, chi)


def _timed(ctx, fn, repeats: int) -> float:
    """Median device time (ms) of fn() on the context's stream."""
    import torch
    fn()
    times = []
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(ctx.stream)
        fn()
        b.record(ctx.stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return sorted(times)[len(times) // 2]


def _bucket(v: int, buckets) -> Optional[int]:
    for b in buckets:
        if v <= b:
            return b
    return None


class _Sample:
    """A problem the tuner measures: device inputs of the path's DeviceInputs
    form plus the k batch its contractions use."""

    def __init__(self, d, kbatch: int):
        p = d.prob
        self.d, self.kbatch = d, kbatch
        self.ng, self.nk, self.nfreq = d.ng, d.nk, d.nfreq
        self.npk, self.edge = p.nocc * p.nemp, max(p.fft)
        # real weights (imaginary frequencies, no broadening): the library
        # forms the Hermitian half with the 128 x 128 form whatever is asked
        self.real_w = p.delta_eV == 0.0 and bool(np.all(np.real(p.freq_eV) == 0.0))

    def pair(self, ctx, k0, k1, M, prec):
        d, p = self.d, self.d.prob
        _rp.rp_pair_density(ctx, d.cell, p.iq, d.nband, p.miller.shape[1], p.npw, d.mmax, d.miller, d.coef,
                            0, p.nocc, p.nocc, p.nocc + p.nemp, k0, k1, d.ng, p.gsph, prec, M)

    def chi(self, ctx, k1, M, chi, prec):
        d, p = self.d, self.d.prob
        wm = _rp.RP_W_SAMPLING if d.nk == 1 else _rp.RP_W_TETRA
        _rp.rp_chi0_accumulate(ctx, d.cell, p.iq, d.nband, d.energy, d.T, 0, p.nocc, p.nocc, p.nocc + p.nemp,
                               0, k1, d.ng, M, d.nfreq, p.freq_eV, p.delta_eV, wm, prec, 0, chi)


class _Synthetic:
    """A synthetic class problem in the _Sample form (all k in one batch)."""

    def __init__(self, p: _ClassProblem):
        self.dev = _Device(p)
        self.ng, self.nk, self.nfreq = p.ng, p.nk, len(p.freq)
        self.npk, self.edge, self.kbatch = p.nocc * p.nemp, max(p.fft), p.nk
        self.real_w = True

    def pair(self, ctx, k0, k1, M, prec):
        self.dev.pair(ctx, k0, k1, M, prec)

    def chi(self, ctx, k1, M, chi, prec):
        self.dev.chi(ctx, M, chi, prec)


def autotune(ctx, samples=None, ng_buckets=NG_BUCKETS, grid_buckets=GRID_BUCKETS, repeats: int = 3,
             log=print) -> dict:
    """Measure every candidate per class and keep the fastest; returns the
    table (JSON-ready).

    samples: optional list of (DeviceInputs, kbatch) of the workload to tune
    for; each class then sums the device time of its samples' first k batch
    (contraction) or first two k-points (u-grids).  Without samples, one
    synthetic problem at the class's upper sizes stands for each class."""
    import torch
    prec = _rp.RP_SPLIT_BF16
    big = 10 ** 6
    if samples:
        items = [_Sample(d, kb) for d, kb in samples]
        chi_items = [(_bucket(m.ng, ng_buckets), m) for m in items]
        fft_items = [(_bucket(m.edge, grid_buckets), m) for m in items]
    else:
        chi_items = [(b, _Synthetic(_ClassProblem(edge=32, ng=b))) for b in ng_buckets]
        fft_items = [(b, _Synthetic(_ClassProblem(edge=b, ng=300))) for b in grid_buckets]
    chi_tot = {b: {c: 0.0 for c in CHI_CANDIDATES} for b in ng_buckets}
    for b, smp in chi_items:
        if b is None:
            continue
        k1 = min(smp.nk, smp.kbatch)
        M = torch.empty((k1 * smp.npk, smp.ng, 2), dtype=torch.float64, device="cuda")
        chi = torch.empty((smp.nfreq, smp.ng, smp.ng, 2), dtype=torch.float64, device="cuda")
        _rp.rp_set_tuning(ctx, [])
        smp.pair(ctx, 0, k1, M, prec)
        for c in CHI_CANDIDATES:
            if smp.real_w and c[0] != 0:
                chi_tot[b][c] = float("inf")    # the same launches as form 0
                continue
            _rp.rp_set_tuning(ctx, [dict(ng_max=big, grid_max=big, chi_nw=c[1], chi_fill=c[2], fft_lines=0,
                                         chi_kernel=c[0])])
            chi_tot[b][c] += _timed(ctx, lambda: smp.chi(ctx, k1, M, chi, prec), repeats)
        del M, chi
    chi_pick = {}
    for b in ng_buckets:
        res = chi_tot[b]
        if not any(v for v in res.values() if v != float("inf")):
            continue
        best = min(res, key=res.get)
        if res[CHI_DEFAULT] <= res[best] * (1.0 + MARGIN):
            best = CHI_DEFAULT
        chi_pick[b] = best
        log(f"[autotune] N_G <= {b}: " + ", ".join(f"kernel={k} nw={nw} fill={fill}: {v:.3f} ms"
                                                   for (k, nw, fill), v in res.items()) +
            f" -> kernel={best[0]} nw={best[1]} fill={best[2]}")
    fft_tot = {b: {c: 0.0 for c in FFT_CANDIDATES} for b in grid_buckets}
    for b, smp in fft_items:
        if b is None:
            continue
        k1 = min(2, smp.nk)
        M = torch.empty((k1 * smp.npk, smp.ng, 2), dtype=torch.float64, device="cuda")
        for lines in FFT_CANDIDATES:
            _rp.rp_set_tuning(ctx, [dict(ng_max=big, grid_max=big, chi_nw=0, chi_fill=-1, fft_lines=lines,
                                         chi_kernel=0)])
            smp.pair(ctx, 0, k1, M, prec)
            vals = []
            for _ in range(repeats):
                _rp.rp_profile(ctx, True)
                smp.pair(ctx, 0, k1, M, prec)
                vals.append(_rp.rp_profile_read(ctx)["ugrid"][0])
                _rp.rp_profile(ctx, False)
            fft_tot[b][lines] += sorted(vals)[len(vals) // 2]
        del M
    fft_pick = {}
    for b in grid_buckets:
        res = fft_tot[b]
        if not any(res.values()):
            continue
        best = min(res, key=res.get)
        if res[FFT_DEFAULT] <= res[best] * (1.0 + MARGIN):
            best = FFT_DEFAULT
        fft_pick[b] = best
        log(f"[autotune] edge <= {b}: " + ", ".join(f"lines={k}: {v:.3f} ms" for k, v in res.items()) +
            f" -> lines={best}")
    _rp.rp_set_tuning(ctx, [])
    default_chi = (0, 0, -1)
    entries = [dict(ng_max=nb, grid_max=gb, chi_kernel=chi_pick.get(nb, default_chi)[0],
                    chi_nw=chi_pick.get(nb, default_chi)[1], chi_fill=chi_pick.get(nb, default_chi)[2],
                    fft_lines=fft_pick.get(gb, 0))
               for nb in ng_buckets for gb in grid_buckets]
    return {"device": torch.cuda.get_device_name(0), "ng_buckets": list(ng_buckets),
            "grid_buckets": list(grid_buckets), "entries": entries,
            "tuned_on": "workload samples" if samples else "synthetic class problems",
            "samples": len(samples) if samples else 0,
            "measured_ms": {"chi": {str(b): {f"kernel{c[0]}_nw{c[1]}_fill{c[2]}": round(v, 4)
                                             for c, v in r.items() if v != float("inf")}
                                    for b, r in chi_tot.items()},
                            "ugrid": {str(b): {f"lines{c}": round(v, 4) for c, v in r.items()}
                                      for b, r in fft_tot.items()}},
            "created": time.strftime("%Y-%m-%d %H:%M:%S")}


def merge(*tables) -> dict:
    """One table from several: the classes of every table that measured
    them, ordered by N_G bound then edge bound (a class measured by an
    earlier table is kept)."""
    seen, entries = set(), []
    for t in tables:
        measured = {int(b) for b, r in t["measured_ms"]["chi"].items() if r} | \
                   {int(b) for b, r in t["measured_ms"]["ugrid"].items() if any(r.values())}
        for e in t["entries"]:
            key = (e["ng_max"], e["grid_max"])
            if key in seen or (e["ng_max"] not in measured and e["grid_max"] not in measured):
                continue
            seen.add(key)
            entries.append(e)
    entries.sort(key=lambda e: (e["ng_max"], e["grid_max"]))
    out = dict(tables[0])
    out["entries"] = entries
    out["merged_from"] = [{"tuned_on": t.get("tuned_on"), "samples": t.get("samples"),
                           "ng_buckets": t["ng_buckets"], "grid_buckets": t["grid_buckets"],
                           "measured_ms": t["measured_ms"]} for t in tables]
    out.pop("measured_ms", None)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--repeats", type=int, default=5)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the autotuner needs a GPU")
    ctx = _rp.Context(0, tuning=None)
    table = autotune(ctx, repeats=args.repeats)
    ctx.close()
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"[autotune] wrote {args.out} ({len(table['entries'])} classes)", flush=True)


if __name__ == "__main__":
    main()
