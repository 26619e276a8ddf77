"""Autotuner of the library's launch shapes per size class.

Size classes are N_G buckets x FFT-edge buckets.  For each class the tuner
times the candidate launch shapes on synthetic inputs of the class's upper
sizes (random coefficients and energies: only the shapes matter for timing)
and keeps the fastest:

* the split-BF16 contraction (chi_nw frequencies per workgroup, chi_fill
  workgroups aimed for by slicing the pair steps): timed per N_G bucket on
  one contraction of about 40 000 pairs with 16 imaginary frequencies;
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

import numpy as np

from . import _rp

NG_BUCKETS = (512, 768, 1024, 1200)
GRID_BUCKETS = (27, 32, 40)
CHI_CANDIDATES = tuple((nw, fill) for nw in (1, 2) for fill in (0, 512, 1024, 2048))
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


def autotune(ctx, ng_buckets=NG_BUCKETS, grid_buckets=GRID_BUCKETS, repeats: int = 3, log=print) -> dict:
    """Measure every candidate per class; returns the table (JSON-ready)."""
    import torch
    prec = _rp.RP_SPLIT_BF16
    big = 10 ** 6
    chi_pick, chi_ms = {}, {}
    for ngb in ng_buckets:
        p = _ClassProblem(edge=32, ng=ngb)
        d = _Device(p)
        npair = p.nk * p.nocc * p.nemp
        M = torch.empty((npair, p.ng, 2), dtype=torch.float64, device="cuda")
        chi = torch.empty((len(p.freq), p.ng, p.ng, 2), dtype=torch.float64, device="cuda")
        _rp.rp_set_tuning(ctx, [])
        d.pair(ctx, 0, p.nk, M, prec)
        res = {}
        for nw, fill in CHI_CANDIDATES:
            _rp.rp_set_tuning(ctx, [dict(ng_max=big, grid_max=big, chi_nw=nw, chi_fill=fill, fft_lines=0)])
            res[(nw, fill)] = _timed(ctx, lambda: d.chi(ctx, M, chi, prec), repeats)
        best = min(res, key=res.get)
        chi_pick[ngb] = best
        chi_ms[ngb] = {f"nw{nw}_fill{fill}": round(v, 4) for (nw, fill), v in res.items()}
        log(f"[autotune] N_G <= {ngb} ({npair} pairs, 16 w): " +
            ", ".join(f"nw={nw} fill={fill}: {v:.3f} ms" for (nw, fill), v in res.items()) +
            f" -> nw={best[0]} fill={best[1]}")
        del M, chi
    fft_pick, fft_ms = {}, {}
    for gb in grid_buckets:
        p = _ClassProblem(edge=gb, ng=300)
        d = _Device(p)
        M = torch.empty((2 * p.nocc * p.nemp, p.ng, 2), dtype=torch.float64, device="cuda")
        res = {}
        for lines in FFT_CANDIDATES:
            _rp.rp_set_tuning(ctx, [dict(ng_max=big, grid_max=big, chi_nw=0, chi_fill=-1, fft_lines=lines)])
            d.pair(ctx, 0, 2, M, prec)
            vals = []
            for _ in range(repeats):
                _rp.rp_profile(ctx, True)
                d.pair(ctx, 0, 2, M, prec)
                vals.append(_rp.rp_profile_read(ctx)["ugrid"][0])
                _rp.rp_profile(ctx, False)
            res[lines] = sorted(vals)[len(vals) // 2]
        best = min(res, key=res.get)
        fft_pick[gb] = best
        fft_ms[gb] = {f"lines{k}": round(v, 4) for k, v in res.items()}
        log(f"[autotune] edge <= {gb}: " + ", ".join(f"lines={k}: {v:.3f} ms" for k, v in res.items()) +
            f" -> lines={best}")
    _rp.rp_set_tuning(ctx, [])
    entries = [dict(ng_max=ngb, grid_max=gb, chi_nw=chi_pick[ngb][0], chi_fill=chi_pick[ngb][1],
                    fft_lines=fft_pick[gb]) for ngb in ng_buckets for gb in grid_buckets]
    return {"device": torch.cuda.get_device_name(0), "ng_buckets": list(ng_buckets),
            "grid_buckets": list(grid_buckets), "entries": entries,
            "measured_ms": {"chi": {str(k): v for k, v in chi_ms.items()},
                            "ugrid": {str(k): v for k, v in fft_ms.items()}},
            "created": time.strftime("%Y-%m-%d %H:%M:%S")}


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
