#!/usr/bin/env python
"""chi0 build TFLOP/s and seconds per q-point on one MI355X, split-BF16 and
FP64 side by side, on the SrVO3-shaped workload (48^3 grid, 8^3 k mesh,
40 + 200 bands, N_G = 1500, 20 real frequencies, one q-point).

A step is one q-point through the whole path: pair densities and chi0 for all
512 k (streamed in k batches), eps^-1 and W, and the Wannier projection W_ij.
Inputs are resident in HBM before the timed region.

  value         split-BF16 chi0 build rate F_chi / t_chi0 (TFLOP/s), with
                F_chi = 8 N_G^2 P N_w the algorithmic flops of Eq. chi
                (P = 4 096 000 pairs) and t_chi0 the wall time of the pair
                densities + weights + contraction of one q-point
  fp64          the same for the FP64 path
  split_bf16_x6 the six-product (hi/mid/lo) split form
  roofline      the chi contraction kernel of the split path: algorithmic
                flops per launch / its mean launch time (HIP events on the
                library's stream) against the BF16 dense peak; traffic is the
                HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE
                counters, scaled by what they read for a plain copy, as
                recorded in profiles/k_chi_rows_traffic.md (reported only
                while the kernel source matches the recorded hash), and
                mfma_counter_frac the executed MFMA flops from the BF16
                MOPS counter recorded there
  hbm_a2_a4     HBM bytes of the pair kernel and the u-grid kernels from
                profiles/pair_stage_hbm_counters.md over their stage times,
                with the algorithmic bytes (u-grids once + the
                contraction operands it writes) beside them
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload
  vs_oracle_sample  the GPU's chi0 of that sample (split, x6 and FP64)
                against the oracle's result there, element-wise and in norm

Counter runs use two extra modes: --copy-calibration (a plain 1 GiB device
copy, three times) and --profile-k N (the split chi0 build over the first N
k-points in the launch configuration of the timed legs).

--supercell measures the large-supercell shape (96^3, N_G = 6000, 720 000
pairs over 16 frequencies streamed in blocks of empty bands; rate counts the
full Eq. chi, 8 N_G^2 P N_w).

--tune OUT writes the launch-shape table tuned on both workloads (the
package's tuning_mi355x.json comes from it).

--batch measures the batched uneven workload instead (24 systems x 4
q-points, 16 imaginary frequencies, split-BF16 chi0) through rp_chi0_batch,
one graph launch per step, beside the same problems through per-problem
calls; launch shapes are autotuned on the workload first (one q-point of
every system) and the default shapes are timed beside; its rate counts the Hermitian half of Eq. chi, F = 4 N_G^2 P N_w per
problem (real weights on the imaginary axis).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "χ0 build TFLOP/s + s/q-point, split-BF16 vs FP64, at rel err ≤1e-5 vs oracle"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_chi_rows_traffic.md")
CHI_SOURCE = os.path.join(ROOT, "paper_2001_02351_amd", "csrc", "chi_bf16.hip")


PAIR_FILE = os.path.join(ROOT, "profiles", "pair_stage_hbm_counters.md")


def _sha(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _recorded(path, keys):
    """key: value lines of a committed counter summary (None if absent)."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.strip().strip("`")
            k = line.split(":", 1)[0].strip()
            if ":" in line and k in keys:
                vals[k] = line.split(":", 1)[1].strip()
    return vals


def recorded_traffic():
    """HBM bytes and BF16 MFMA ops per contraction launch from the committed
    counter summary, or None when there is none or the kernel source changed
    since it was taken."""
    vals = _recorded(TRAFFIC_FILE, ("traffic_bytes_per_launch", "mfma_mops_per_launch",
                                    "kernel_source_sha256"))
    if not vals or vals.get("kernel_source_sha256") != _sha(CHI_SOURCE) or \
            "traffic_bytes_per_launch" not in vals:
        return None
    return {k: float(v) for k, v in vals.items() if k != "kernel_source_sha256"}


def recorded_pair_counters():
    """HBM bytes of the pair kernel (per launch = per k-point) and of the u-grid
    kernels (per k-point), or None when the sources changed."""
    vals = _recorded(PAIR_FILE, ("pair_bytes_per_launch", "ugrid_bytes_per_k", "pair_source_sha256",
                                 "fft_source_sha256"))
    csrc = os.path.join(ROOT, "paper_2001_02351_amd", "csrc")
    if not vals or vals.get("pair_source_sha256") != _sha(os.path.join(csrc, "pair.hip")) or \
            vals.get("fft_source_sha256") != _sha(os.path.join(csrc, "fft.hip")):
        return None
    return {k: float(vals[k]) for k in ("pair_bytes_per_launch", "ugrid_bytes_per_k")}


def copy_calibration():
    """A plain device-to-device copy of 1 GiB, three times (counter scale)."""
    import torch
    a = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": a.numel() * 4, "repeats": 3}), flush=True)


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, ng_sample: int = 500):
    """Time the FP64 oracle on a bounded sample of the q-point: k = 0 with all
    occupied x empty bands and all frequencies, on the first `ng_sample`
    vectors of the polarization sphere (pair densities on those vectors,
    tetrahedron weights over the full mesh, chi0 of the sample).  value is the
    sample's chi0 build rate 8 N_G'^2 P N_w / t.  The pair densities of a tenth
    of the sample's pairs on the whole sphere are timed as well, and the
    seconds per q-point are extrapolated from the sample (pair densities and
    weights linearly in the k-points, chi0 also as N_G^2), labelled as an
    extrapolation."""
    from dataclasses import replace

    import numpy as np

    import oracle
    ngs = min(ng_sample, prob.ng)
    sub = replace(prob, gsph=np.ascontiguousarray(prob.gsph[:ngs]))
    o0, o1, e0, e1 = 0, prob.nocc, prob.nocc, prob.nocc + prob.nemp
    t0 = time.perf_counter()
    M = oracle.pair_densities(sub, o0, o1, e0, e1, 0, 1)
    t1 = time.perf_counter()
    w = oracle.prob_weights(prob, o0, o1, e0, e1, 0, 1)
    t2 = time.perf_counter()
    chi_sample = oracle.chi0(M, w)
    t3 = time.perf_counter()
    npair = M.shape[0]
    e_tenth = e0 + max(1, (e1 - e0) // 10)
    oracle.pair_densities(prob, o0, o1, e0, e_tenth, 0, 1)
    t4 = time.perf_counter()
    pair_full = (t4 - t3) * (e1 - e0) / (e_tenth - e0)
    nfreq = len(prob.freq_eV)
    flops = 8.0 * ngs ** 2 * npair * nfreq
    per_q = prob.nk * (pair_full + (t2 - t1) + (t3 - t2) * (prob.ng / ngs) ** 2)
    return {
        "value": flops / (t3 - t0) / 1e12,
        "unit": "TFLOP/s",
        "cores": oracle.threads_used(),
        "cpu_model": _cpu_model(),
        "kind": "oracle",
        "sample": (f"k = 0 of {prob.nk}: all {prob.nocc} x {prob.nemp} bands ({npair} pairs), all {nfreq} "
                   f"frequencies, the first {ngs} of the {prob.ng} sphere vectors: pair densities "
                   f"{t1 - t0:.1f} s, weights {t2 - t1:.1f} s, chi0 {t3 - t2:.1f} s (measured, {t3 - t0:.1f} s); "
                   f"pair densities on all {prob.ng} vectors for a tenth of the pairs {t4 - t3:.1f} s"),
        "seconds": t3 - t0,
        "s_per_qpoint_extrapolated": per_q,
        "extrapolation": (f"{prob.nk} k-points x (pair densities on all {prob.ng} vectors, scaled from a tenth "
                          f"of the pairs; weights; chi0 scaled by ({prob.ng}/{ngs})^2)"),
        "chi_sample": chi_sample,   # the sample's chi0, [nfreq][ngs][ngs] (not part of the JSON line)
    }


def oracle_sample_errors(rp, path, ctx, d, baseline) -> dict:
    """The GPU path's chi0 over the cpu_baseline sample (k = 0, all bands and
    frequencies) against the oracle's, on the sample's leading ngs x ngs block
    of the sphere: per frequency the relative Frobenius norm of the difference
    and max |diff| / max |chi|, the largest over the frequencies."""
    import numpy as np
    import torch
    want = baseline["chi_sample"]
    ngs = want.shape[1]
    chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device=d.device)
    out = {"sample": f"chi0 of k = 0 (all bands, all {d.nfreq} frequencies) on the first {ngs} x {ngs} of the "
                     f"{d.ng} x {d.ng} sphere block, against the cpu_baseline leg's oracle result"}
    for name, prec in (("split_bf16", rp.RP_SPLIT_BF16), ("split_bf16_x6", rp.RP_SPLIT_BF16_X6),
                       ("fp64", rp.RP_FP64)):
        path.chi0(ctx, d, prec=prec, kbatch=1, k0=0, k1=1, chi=chi)
        rp.rp_synchronize(ctx)
        got = path.to_complex(chi[:, :ngs, :ngs].contiguous())
        fro = max(float(np.linalg.norm(got[f] - want[f]) / np.linalg.norm(want[f])) for f in range(d.nfreq))
        ew = max(float(np.abs(got[f] - want[f]).max() / np.abs(want[f]).max()) for f in range(d.nfreq))
        out[name] = {"chi": fro, "chi_max_elementwise": ew}
    return out


def run_leg(rp, path, ctx, d, prec, steps, warmup, kbatch):
    import torch
    npair_total = d.nk * d.prob.nocc * d.prob.nemp
    flops = 8.0 * d.ng ** 2 * npair_total * d.nfreq
    chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device=d.device)
    for i in range(warmup):
        log(f"prec={prec} warmup step {i}")
        c = path.chi0(ctx, d, prec=prec, kbatch=kbatch, chi=chi)
        einv, W = path.screen(ctx, d, c)
        path.wannier(ctx, d, einv)
        rp.rp_synchronize(ctx)
    rp.rp_profile(ctx, True)
    t_chi, t_step = [], []
    for i in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = path.chi0(ctx, d, prec=prec, kbatch=kbatch, chi=chi)
        rp.rp_synchronize(ctx)
        t1 = time.perf_counter()
        einv, W = path.screen(ctx, d, c)
        Wij = path.wannier(ctx, d, einv)
        rp.rp_synchronize(ctx)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_chi.append(t1 - t0)
        t_step.append(t2 - t0)
        log(f"prec={prec} step {i}: chi0 {t1 - t0:.3f} s, step {t2 - t0:.3f} s")
    stages = rp.rp_profile_read(ctx)
    rp.rp_profile(ctx, False)
    tc = sorted(t_chi)[len(t_chi) // 2]
    ts = sorted(t_step)[len(t_step) // 2]
    ms_chi, n_chi = stages["chi"]
    per_launch_pairs = kbatch * d.prob.nocc * d.prob.nemp
    chi_launch_ms = ms_chi / max(1, n_chi)
    res = {
        "chi0_tflops": flops / tc / 1e12,
        "s_per_qpoint": ts,
        "t_chi0_s": tc,
        "gemm_tflops": flops / (ms_chi / steps / 1e3) / 1e12 if ms_chi > 0 else None,
        "chi_kernel_ms_per_launch": chi_launch_ms,
        "chi_kernel_launches_per_step": n_chi // steps,
        "chi_kernel_flops_per_launch": 8.0 * d.ng ** 2 * per_launch_pairs * d.nfreq,
        "stage_ms_per_step": {k: v[0] / steps for k, v in stages.items()},
    }
    return res, chi, einv, Wij


def _line(value, unit, steps, warmup, ms, config, extra):
    """One JSON result line of the bench contract."""
    out = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic", "config": config}
    out.update(extra)
    return out


def _chi_roofline(flops_per_launch, ms_per_launch):
    """Roofline entry of the split-BF16 contraction kernel: algorithmic flops
    per launch over its mean launch time, against the BF16 dense peak."""
    if not ms_per_launch:
        return None
    a = flops_per_launch / (ms_per_launch / 1e3) / 1e12
    return {"bound": "mfma", "achieved": a, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
            "frac": a / PEAK_BF16_TFLOPS, "kernel": "k_chi_rows (chi0 contraction, split-BF16)",
            "flops_per_launch": flops_per_launch, "ms_per_launch": ms_per_launch}


def batch_measure(args, embedded: bool = False) -> dict:
    """The batched uneven workload (24 systems x 4 q-points, 16 imaginary
    frequencies, split-BF16 chi0) through rp_chi0_batch: the graphs captured
    on the first call, args.warmup untimed and args.steps timed batch calls
    (median), then the same problems through per-problem calls with the stage
    timers, whose contraction launches give the roofline (the algorithmic
    Hermitian-half flops 4 N_G^2 P N_w of every problem over the summed
    contraction time).  Standalone (--batch) the launch shapes are autotuned on
    the workload first and the default shapes are timed beside; embedded in
    the default run the package's tuning table is used."""
    import copy

    import torch

    import paper_2001_02351_amd as rp
    from paper_2001_02351_amd import path
    from synth import batch_system_qpoints
    nsys = args.batch_systems
    log(f"generating {nsys} uneven systems x 4 q-points")
    t0 = time.perf_counter()
    probs = []
    for s in range(nsys):
        probs += batch_system_qpoints(s)
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    baseline = None
    if not embedded and not args.no_cpu_baseline and not args.batch_no_graph:
        # the oracle on one problem of the batch (system 21, the fewest pairs
        # per k-point): k = 0, all bands, 16 frequencies, the first 500 sphere vectors
        small = [p for p in probs if p.name == "batch_system_21_q0"]
        if small:
            log("timing the FP64 oracle on a bounded sample of the batch (host cores)")
            baseline = cpu_baseline(small[0])
            baseline["value"] /= 2.0     # Hermitian-half flops, as the batch rate counts them
            log(f"oracle sample: {baseline['sample']}")
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    rp.load()
    mode = "default" if embedded else args.batch_tuning
    ctx = rp.Context(0, tuning=None if mode in ("workload", "none") else mode)
    ds = []
    for i, p in enumerate(probs):
        if i % 4 == 0:
            base = path.DeviceInputs(p)
            ds.append(base)
        else:
            d = copy.copy(base)
            d.prob = p
            ds.append(d)
    chis = [torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device=d.device) for d in ds]
    torch.cuda.synchronize()
    log("batch inputs resident on the device")
    prec = rp.RP_SPLIT_BF16
    # k batches of about 40 000 pairs (at least one k-point)
    descs = []
    for d, c in zip(ds, chis):
        npk = d.prob.nocc * d.prob.nemp
        kb = max(1, min(d.nk, args.batch_pairs // npk))
        descs.append(path.batch_problem(d, c, kb))
    pairs = [d.nk * d.prob.nocc * d.prob.nemp for d in ds]
    f_herm = sum(4.0 * d.ng ** 2 * P * d.nfreq for d, P in zip(ds, pairs))
    table, t_tune = None, None
    if mode == "workload":
        # launch shapes tuned on the workload: one q-point of every system
        from paper_2001_02351_amd import autotune
        t = time.perf_counter()
        table = autotune.autotune(ctx, samples=[(ds[i], descs[i]["kbatch"]) for i in range(0, len(ds), 4)],
                                  log=log)
        t_tune = time.perf_counter() - t
        rp.rp_set_tuning(ctx, table["entries"])
        log(f"autotuned on {len(ds) // 4} samples in {t_tune:.1f} s")
        if args.tuning_out:
            with open(args.tuning_out, "w") as f:
                json.dump(table, f, indent=1)
    elif ctx.tuning is not None:
        table = {"entries": rp.load_tuning(ctx.tuning), "file": os.path.relpath(ctx.tuning, ROOT)}
    if args.batch_no_graph:
        # per-problem calls only (for profilers that do not follow graph launches)
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for d, c, q in zip(ds, chis, descs):
                path.chi0(ctx, d, prec=prec, kbatch=q["kbatch"], chi=c)
            rp.rp_synchronize(ctx)
            log(f"per-problem calls {i}: {time.perf_counter() - t:.3f} s")
        ctx.close()
        return {}
    t = time.perf_counter()
    rp.rp_chi0_batch(ctx, descs, prec)
    rp.rp_synchronize(ctx)
    graphs, nodes = rp.rp_chi0_batch_graphs(ctx)
    log(f"first batch call (capture of {graphs} graphs, {nodes} kernel nodes, + run) "
        f"{time.perf_counter() - t:.2f} s")
    warm = 1 if embedded else args.warmup
    steps = 1 if embedded else args.steps
    for i in range(warm):
        rp.rp_chi0_batch(ctx, descs, prec)
        rp.rp_synchronize(ctx)
    times = []
    for i in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        rp.rp_chi0_batch(ctx, descs, prec)
        rp.rp_synchronize(ctx)
        times.append(time.perf_counter() - t)
        log(f"batch step {i}: {times[-1]:.3f} s")
    tb = sorted(times)[len(times) // 2]
    # the same batch with the library's default launch shapes (no table)
    untuned = None
    if table is not None and not embedded:
        rp.rp_set_tuning(ctx, [])
        rp.rp_chi0_batch(ctx, descs, prec)
        rp.rp_synchronize(ctx)
        ut = []
        for i in range(max(1, args.steps // 2)):
            t = time.perf_counter()
            rp.rp_chi0_batch(ctx, descs, prec)
            rp.rp_synchronize(ctx)
            ut.append(time.perf_counter() - t)
        untuned = sorted(ut)[len(ut) // 2]
        log(f"default launch shapes: {untuned:.3f} s")
        rp.rp_set_tuning(ctx, table["entries"])
    # the same problems through per-problem calls, with per-stage timers
    rp.rp_profile(ctx, True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for d, c, q in zip(ds, chis, descs):
        path.chi0(ctx, d, prec=prec, kbatch=q["kbatch"], chi=c)
    rp.rp_synchronize(ctx)
    tu = time.perf_counter() - t
    stages = rp.rp_profile_read(ctx)
    rp.rp_profile(ctx, False)
    log(f"per-problem calls: {tu:.3f} s")
    ctx.close()
    ms_chi, n_chi = stages["chi"]
    roof = _chi_roofline(f_herm / max(1, n_chi), ms_chi / max(1, n_chi))
    if roof:
        roof["note"] = ("mean over the contraction launches of the per-problem calls; flops per launch = the "
                        "batch's Hermitian-half flops / launches")
    return {
        "value": f_herm / tb / 1e12,
        "unit": "TFLOP/s",
        "s_per_batch": tb,
        "steps": steps,
        "warmup": warm,
        "config": {
            "workload": f"batched uneven systems: {nsys} systems x 4 q-points, grids 24^3-40^3, k meshes "
                        "2^3-6^3, 16-64 + 48-256 bands, N_G 300-1200, 16 imaginary frequencies, delta=0, "
                        "generalized tetrahedron, split-BF16 chi0, one rp_chi0_batch call (a sequence of "
                        "captured graphs) per step",
            "problems": len(ds),
            "pairs": sum(pairs),
            "flops_hermitian_half": f_herm,
            "pairs_per_k_batch": args.batch_pairs,
            "graphs": graphs,
            "kernel_nodes": nodes,
        },
        "roofline": roof,
        "tuning": None if table is None else {"mode": mode, "seconds": t_tune, "entries": table["entries"]},
        "s_per_batch_default_shapes": untuned,
        "per_problem_calls_s": tu,
        "per_problem_stage_ms": {k: v[0] for k, v in stages.items()},
        "per_problem_stage_launches": {k: v[1] for k, v in stages.items()},
        "cpu_baseline": None if baseline is None else {k: baseline[k] for k in
                                                        ("value", "unit", "cores", "cpu_model", "kind",
                                                         "sample")},
    }


def batch_leg(args):
    """--batch: the batched workload as its own JSON line."""
    r = batch_measure(args)
    if not r:
        return
    extra = {k: v for k, v in r.items() if k not in ("value", "unit", "steps", "warmup", "config")}
    print(json.dumps(_line(r["value"], r["unit"], r["steps"], r["warmup"], r["s_per_batch"] * 1e3, r["config"],
                           extra)), flush=True)


def supercell_measure(args) -> dict:
    """The large-supercell shape (96^3, Gamma only, q = 0, 600 + 1200 bands,
    N_G = 6000, 16 real frequencies, 20 Wannier orbitals): split-BF16 chi0
    streamed over blocks of empty bands (one warm-up block, then the timed
    q-point), FP64 eps^-1 and W, W_ij; the contraction launches give the
    roofline."""
    import torch

    import paper_2001_02351_amd as rp
    from paper_2001_02351_amd import path
    from synth import supercell_workload
    log("generating the supercell workload (96^3, 600 + 1200 bands, N_G = 6000)")
    t0 = time.perf_counter()
    p = supercell_workload()
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    rp.load()
    ctx = rp.Context(0)
    d = path.DeviceInputs(p)
    eb = args.sc_emp_block
    nblk = (p.nemp + eb - 1) // eb
    nrun = nblk if args.sc_blocks <= 0 else min(nblk, args.sc_blocks)
    prec = rp.RP_SPLIT_BF16
    chi = torch.empty((d.nfreq, d.ng, d.ng, 2), dtype=torch.float64, device=d.device)
    torch.cuda.synchronize()
    log("supercell inputs resident on the device")

    def block(i, acc):
        # one empty-band block: its pair kernels write the contraction's operands
        e0 = p.nocc + i * eb
        e1 = min(p.nocc + p.nemp, e0 + eb)
        rp.rp_chi0_run(ctx, path.batch_problem(d, chi, 1, o=(0, p.nocc), e=(e0, e1), k=(0, 1), accumulate=acc),
                       prec)

    block(0, 0)                                      # warm-up (kernel loading)
    rp.rp_synchronize(ctx)
    rp.rp_profile(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nrun):
        block(i, 0 if i == 0 else 1)
    rp.rp_synchronize(ctx)
    t_chi = time.perf_counter() - t0
    log(f"supercell chi0 over {nrun} of {nblk} empty-band blocks: {t_chi:.2f} s")
    t0 = time.perf_counter()
    einv, W = path.screen(ctx, d, chi)
    rp.rp_synchronize(ctx)
    t_scr = time.perf_counter() - t0
    t0 = time.perf_counter()
    path.wannier(ctx, d, einv)
    rp.rp_synchronize(ctx)
    t_wan = time.perf_counter() - t0
    stages = rp.rp_profile_read(ctx)
    rp.rp_profile(ctx, False)
    ctx.close()
    pairs = p.nocc * min(p.nemp, nrun * eb)
    flops = 8.0 * d.ng ** 2 * pairs * d.nfreq
    scale = (p.nocc * p.nemp) / pairs
    ms_chi, n_chi = stages["chi"]
    return {
        "value": flops / t_chi / 1e12,
        "unit": "TFLOP/s",
        "s_per_qpoint": t_chi * scale + t_scr + t_wan,
        "config": {
            "workload": "supercell q-point: 96^3 grid, Gamma-only k, q = 0 (G = 0 dropped), 600 + 1200 bands, "
                        "N_G = 6000, 16 real frequencies, delta = 0.1 eV, sampling weights, 20 Wannier orbitals; "
                        f"pair densities streamed in blocks of {eb} empty bands",
            "pairs_timed": pairs,
            "pairs_total": p.nocc * p.nemp,
            "pair_grid": list(rp.rp_pair_grid(d.cell, p.iq, d.mmax, p.gsph, rp.RP_SPLIT_BF16)),
            "ng": d.ng,
            "nfreq": d.nfreq,
        },
        "roofline": _chi_roofline(flops / max(1, n_chi), ms_chi / max(1, n_chi)),
        "t_chi0_s_timed": t_chi,
        "t_chi0_s_per_qpoint": t_chi * scale,
        "t_screen_s": t_scr,
        "t_wannier_s": t_wan,
        "stage_ms": {k: v[0] for k, v in stages.items()},
    }


def supercell_leg(args):
    """--supercell: the supercell shape as its own JSON line."""
    r = supercell_measure(args)
    extra = {k: v for k, v in r.items() if k not in ("value", "unit", "config")}
    print(json.dumps(_line(r["value"], r["unit"], 1, 1, r["s_per_qpoint"] * 1e3, r["config"], extra)), flush=True)


def tune_leg(args):
    """Launch shapes tuned on the 48^3 workload's first k batch and on one
    q-point of every batched system, merged into one table (--tune OUT)."""

    import torch

    import paper_2001_02351_amd as rp
    from paper_2001_02351_amd import autotune, path
    from synth import batch_system_qpoints, srvo3_workload
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    rp.load()
    ctx = rp.Context(0, tuning=None)
    log("tuning on the 48^3 workload (first k batch)")
    d = path.DeviceInputs(srvo3_workload())
    t48 = autotune.autotune(ctx, samples=[(d, args.kbatch)], ng_buckets=(1536,), grid_buckets=(48,), log=log)
    del d
    torch.cuda.empty_cache()
    log(f"tuning on the batched workload ({args.batch_systems} systems, one q-point each)")
    samples = []
    for s in range(args.batch_systems):
        p = batch_system_qpoints(s)[0]
        dd = path.DeviceInputs(p)
        npk = p.nocc * p.nemp
        samples.append((dd, max(1, min(dd.nk, args.batch_pairs // npk))))
    tb = autotune.autotune(ctx, samples=samples, log=log)
    ctx.close()
    table = autotune.merge(tb, t48)
    with open(args.tune, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({"tuning_table": args.tune, "entries": table["entries"]}), flush=True)


def metal_weights_leg(rp, ctx, d, reps: int = 3) -> dict:
    """The weights of one k batch (two k-points, 20 frequencies) of a metal
    shaped like the workload's: 40 + 200 bands on its 8^3 mesh with smooth
    cosine dispersion (bandwidth 2 eV), the three bands 37..39 crossing
    E_F = 0 (the t2g-like bands of the paper's metal), so they appear in both
    band ranges (occupied 0..39, empty 37..239, 16 240 pairs per k-point); the
    same batch with the insulating weights beside it.  Only the tetrahedra
    near the Fermi surface of the crossing bands are cut."""
    import math

    import numpy as np
    import torch
    p = d.prob
    nb = d.nband
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in p.kmesh], indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(11)
    centre = np.concatenate([np.linspace(-8.0, -1.5, 37), [-0.6, 0.0, 0.6], np.linspace(1.5, 20.0, nb - 40)])
    phase = rng.uniform(0.0, 2.0 * math.pi, (nb, 3))
    E = np.stack([centre[n] - (1.0 / 3.0) * np.sum(np.cos(2.0 * math.pi * kf + phase[n]), axis=1)
                  for n in range(nb)], axis=1)
    Ed = torch.from_numpy(np.ascontiguousarray(E)).to(d.device)
    o, e = (0, p.nocc), (p.nocc - 3, nb)
    npair = 2 * (o[1] - o[0]) * (e[1] - e[0])
    w = torch.empty((d.nfreq, npair, 2), dtype=torch.float64, device=d.device)
    out = {}
    rp.rp_set_fermi_level(ctx, 0.0)
    for name, mode in (("insulating", rp.RP_W_TETRA), ("metal", rp.RP_W_TETRA_METAL)):
        args = (ctx, d.cell, p.iq, nb, Ed, None, *o, *e, 0, 2, d.nfreq, p.freq_eV, p.delta_eV, mode, w)
        rp.rp_weights(*args)
        rp.rp_synchronize(ctx)
        rp.rp_profile(ctx, True)
        for _ in range(reps):
            rp.rp_weights(*args)
        out[name + "_ms_per_launch"] = rp.rp_profile_read(ctx)["weights"][0] / reps
        rp.rp_profile(ctx, False)
    rp.rp_set_fermi_level(ctx, float("nan"))
    out.update(fermi_eV=0.0, crossing_bands=3, pairs_x_freq=npair * d.nfreq)
    log(f"weights of one k batch of the metal: insulating {out['insulating_ms_per_launch']:.2f} ms, "
        f"Fermi-level cut {out['metal_ms_per_launch']:.2f} ms")
    return out


def drude_leg(rp, ctx, d, reps: int = 5) -> dict:
    """The intraband plasma tensor (Eq. plasma) of the metal of
    metal_weights_leg (the workload's coefficients on its 8^3 mesh, the cosine
    spectrum with bands 37..39 crossing E_F = 0): diagonal moments of the three
    bands and their Fermi-surface tetrahedron weights, one synchronous call."""
    import math

    import numpy as np
    import torch
    p = d.prob
    nb = d.nband
    kf = np.stack(np.meshgrid(*[np.arange(K) / K for K in p.kmesh], indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(11)
    centre = np.concatenate([np.linspace(-8.0, -1.5, 37), [-0.6, 0.0, 0.6], np.linspace(1.5, 20.0, nb - 40)])
    phase = rng.uniform(0.0, 2.0 * math.pi, (nb, 3))
    E = np.stack([centre[n] - (1.0 / 3.0) * np.sum(np.cos(2.0 * math.pi * kf + phase[n]), axis=1)
                  for n in range(nb)], axis=1)
    Ed = torch.from_numpy(np.ascontiguousarray(E)).to(d.device)
    args = (ctx, d.cell, nb, p.miller.shape[1], p.npw, d.miller, d.coef, Ed, None, 37, 40, 0.0)
    om = rp.rp_plasma_frequency(*args)
    t0 = time.perf_counter()
    for _ in range(reps):
        om = rp.rp_plasma_frequency(*args)
    ms = (time.perf_counter() - t0) / reps * 1e3
    log(f"plasma tensor of the three bands at E_F: {ms:.3f} ms per call, diagonal {np.diag(om).round(3)} eV^2")
    # the q -> 0 head density (k.p transition moments) of two k-points, all 40 x 200 pairs, into column 0
    M = torch.empty((2 * p.nocc * p.nemp, d.ng, 2), dtype=torch.float64, device=d.device)
    hargs = (ctx, d.cell, nb, p.miller.shape[1], p.npw, d.miller, d.coef, d.energy, 0, p.nocc, p.nocc, nb, 0, 2,
             np.array([1.0, 0.0, 0.0]), d.ng, 0, M)
    rp.rp_head_density(*hargs)
    rp.rp_synchronize(ctx)
    rp.rp_profile(ctx, True)
    for _ in range(reps):
        rp.rp_head_density(*hargs)
    hms = rp.rp_profile_read(ctx)["pair"][0] / reps / 2
    rp.rp_profile(ctx, False)
    log(f"q -> 0 head density: {hms:.3f} ms per k-point (8 000 pairs)")
    return {"ms_per_call": ms, "bands": [37, 40], "fermi_eV": 0.0, "omega2_eV2_diag": np.diag(om).tolist(),
            "head_density_ms_per_k": hms}


def unfold_leg(rp, ctx, d, eps_inv, reps: int = 5) -> dict:
    """The symmetry-unfolding gathers at the workload's shape: eps^-1 (N_G^2 x
    N_w, Eq. symeps) and the coefficients of one k-point (all bands, Eq.
    coef-G) moved by the operation x -> (y, z, x) + (1/2, 0, 0) of the cubic
    cell (any operation of the lattice costs the same); algorithmic bytes = one
    read and one write of every element."""
    import numpy as np
    import torch
    p = d.prob
    W = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], np.int32)
    t = np.array([0.5, 0.0, 0.0])
    S = np.rint(np.linalg.inv(W).T).astype(np.int64)
    iq_s = np.array(p.iq)
    iq_t = (S @ iq_s) % np.array(p.kmesh)
    delta = ((iq_t / np.array(p.kmesh)) - S @ (iq_s / np.array(p.kmesh))).round().astype(np.int64)
    gsph_t = np.ascontiguousarray((p.gsph @ S.T - delta).astype(np.int32))
    dst = torch.empty_like(eps_inv)
    rp.rp_unfold_eps_inv(ctx, d.cell, W, t, iq_s, p.gsph, iq_t, gsph_t, eps_inv, dst)
    k0 = 1
    n0 = int(p.npw[k0])
    kf = np.array(np.unravel_index(k0, p.kmesh))
    kt = (S @ kf) % np.array(p.kmesh)
    dk = ((kt / np.array(p.kmesh)) - S @ (kf / np.array(p.kmesh))).round().astype(np.int64)
    mt = np.ascontiguousarray((p.miller[k0, :n0] @ S.T - dk).astype(np.int32))
    cdst = torch.empty_like(d.coef[k0])
    rp.rp_unfold_coef(ctx, d.cell, W, t, kf, p.miller[k0, :n0], d.coef[k0], kt, mt, cdst)
    rp.rp_synchronize(ctx)
    rp.rp_profile(ctx, True)
    for _ in range(reps):
        rp.rp_unfold_eps_inv(ctx, d.cell, W, t, iq_s, p.gsph, iq_t, gsph_t, eps_inv, dst)
    t_eps = rp.rp_profile_read(ctx)["unfold"][0] / reps
    rp.rp_profile(ctx, True)
    for _ in range(reps):
        rp.rp_unfold_coef(ctx, d.cell, W, t, kf, p.miller[k0, :n0], d.coef[k0], kt, mt, cdst)
    t_coef = rp.rp_profile_read(ctx)["unfold"][0] / reps
    rp.rp_profile(ctx, False)
    b_eps = 2.0 * d.nfreq * d.ng ** 2 * 16
    b_coef = 2.0 * d.nband * n0 * 16
    log(f"unfolding: eps^-1 {t_eps:.3f} ms ({b_eps / t_eps / 1e6:.0f} GB/s), coefficients of one k "
        f"{t_coef:.3f} ms ({b_coef / t_coef / 1e6:.0f} GB/s)")
    return {"eps_inv_ms": t_eps, "eps_inv_bytes": b_eps, "eps_inv_GB_s": b_eps / t_eps / 1e6,
            "coef_ms_per_k": t_coef, "coef_bytes_per_k": b_coef, "coef_GB_s": b_coef / t_coef / 1e6,
            "peak_GB_s": PEAK_HBM_GBS, "bound": "hbm"}


def qterm_cpu_baseline(prob, eps_inv_host) -> dict:
    """The oracle's q-term (oracle/qsum.py, as it stands) on a bounded
    sample of the same workload: the home cell R = 0 only (nwan^2 of the
    27 nwan^2 exchange densities, plus the direct densities), all 20
    frequencies; scaled to the 27 cells by the density count."""
    import numpy as np

    import oracle
    from oracle import qsum
    nw = int(prob.phi.shape[0])
    allg = np.concatenate([prob.gsph, prob.gtail])
    R0 = np.zeros((1, 3), np.int32)
    t0 = time.perf_counter()
    n_u = np.stack([qsum.exchange_ntilde(prob.lat, prob.fft, prob.kmesh, prob.iq, prob.phi, prob.centre_frac, R0,
                                         allg)[0, i, i] for i in range(nw)])
    t_u = time.perf_counter() - t0
    n_x = qsum.exchange_ntilde(prob.lat, prob.fft, prob.kmesh, prob.iq, prob.phi, prob.centre_frac, R0, allg)
    qsum.qterm(prob.lat, prob.kmesh, prob.iq, n_u, n_x, int(prob.gsph.shape[0]), eps_inv_host, R0, allg)
    t = time.perf_counter() - t0
    per_density = (t - t_u) / (nw * nw)
    scaled = t_u + per_density * 27 * nw * nw
    return {"value": scaled * 1e3, "unit": "ms per q-point term (27 cells, scaled)", "cores": oracle.threads_used(),
            "cpu_model": _cpu_model(), "kind": "oracle",
            "sample": f"R = 0 only: {nw} direct + {nw * nw} exchange densities, {len(prob.freq_eV)} frequencies, "
                      f"{t:.1f} s; scaled by the exchange-density count to 27 cells"}


def qterm_leg(rp, path, ctx, d, eps_inv, reps: int = 3, cpu: bool = False):
    """One q-point's term of the q-sums of U, J, V, X on the workload's
    orbitals and its eps^-1 (split leg), for the 27 cells R in {-1, 0, 1}^3:
    27 x nwan^2 exchange densities; the FP64 matrix-core quadratic forms take
    8 N_G^2 (exchange densities + nwan) N_w flop."""
    import itertools

    import numpy as np
    import torch
    p = d.prob
    nw = int(p.phi.shape[0])
    R = np.array(list(itertools.product((-1, 0, 1), repeat=3)), np.int32)
    out = dict(U=torch.empty((d.nfreq, len(R), nw, nw, 2), dtype=torch.float64, device=d.device),
               J=torch.empty((d.nfreq, len(R), nw, nw, 2), dtype=torch.float64, device=d.device),
               V=torch.empty((len(R), nw, nw, 2), dtype=torch.float64, device=d.device),
               X=torch.empty((len(R), nw, nw, 2), dtype=torch.float64, device=d.device))
    path.qterm(ctx, d, eps_inv, p.gsph, R, out, 0)
    rp.rp_synchronize(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        path.qterm(ctx, d, eps_inv, p.gsph, R, out, 0)
    rp.rp_synchronize(ctx)
    t = (time.perf_counter() - t0) / reps
    nv = len(R) * nw * nw
    flops = 8.0 * d.ng ** 2 * (nv + nw) * d.nfreq
    log(f"interaction q-term: {t * 1e3:.1f} ms per q-point ({nv} exchange densities)")
    U = torch.view_as_complex(out["U"])
    V = torch.view_as_complex(out["V"])
    res = {"nR": len(R), "nwan": nw, "exchange_densities": nv, "ng": d.ng, "ntail": int(p.gtail.shape[0]),
           "nfreq": d.nfreq, "ms_per_qpoint": t * 1e3, "matrix_core_flop": flops,
           "tflops_whole_call": flops / t / 1e12, "fp64_peak_tflops": PEAK_FP64_TFLOPS,
           "U_00_w0_over_V_00": float((U[0, 13, 0, 0] / V[13, 0, 0]).real), "cpu_baseline": None}
    if cpu:
        log("timing the oracle's q-term on a bounded sample (host cores)")
        res["cpu_baseline"] = qterm_cpu_baseline(p, path.to_complex(eps_inv))
        log(f"oracle q-term sample: {res['cpu_baseline']['sample']}")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--fp64-warmup", type=int, default=1)
    ap.add_argument("--x6-steps", type=int, default=3)
    ap.add_argument("--x6-warmup", type=int, default=1)
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the supercell and batched-workload legs of the default run")
    ap.add_argument("--kbatch", type=int, default=16)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-x6", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-qterm", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--profile-k", type=int, default=0)
    ap.add_argument("--batch", action="store_true")
    ap.add_argument("--batch-systems", type=int, default=24)
    ap.add_argument("--batch-pairs", type=int, default=40000)
    ap.add_argument("--batch-tuning", default="workload",
                    help="workload (autotune on the batch first), none, or a table file")
    ap.add_argument("--tuning-out", default=None)
    ap.add_argument("--batch-no-graph", action="store_true")
    ap.add_argument("--supercell", action="store_true")
    ap.add_argument("--sc-emp-block", type=int, default=100)
    ap.add_argument("--sc-blocks", type=int, default=0, help="empty-band blocks to time (0: all)")
    ap.add_argument("--tune", default=None, metavar="OUT",
                    help="autotune the launch shapes on both workloads and write the table")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.tune:
        tune_leg(args)
        return
    if args.supercell:
        supercell_leg(args)
        return
    if args.batch:
        batch_leg(args)
        return

    from synth import srvo3_workload
    log("generating the SrVO3-shaped workload (48^3, 8^3 k, 40+200 bands, N_G=1500, 20 w)")
    t0 = time.perf_counter()
    prob = srvo3_workload()
    log(f"generated in {time.perf_counter() - t0:.1f} s")

    baseline = None
    if not args.no_cpu_baseline and not args.profile_k:
        log("timing the FP64 oracle on a bounded sample (host cores)")
        baseline = cpu_baseline(prob)
        log(f"oracle sample: {baseline['sample']}")

    import numpy as np
    import torch

    import paper_2001_02351_amd as rp
    from paper_2001_02351_amd import path
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    rp.load()
    ctx = rp.Context(0)
    d = path.DeviceInputs(prob)
    torch.cuda.synchronize()
    log("inputs resident on the device")
    if args.profile_k:
        path.chi0(ctx, d, prec=rp.RP_SPLIT_BF16, kbatch=args.kbatch, k0=0, k1=args.profile_k)
        rp.rp_synchronize(ctx)
        log(f"split chi0 over k < {args.profile_k} done")
        ctx.close()
        return

    split, chi_s, einv_s, wij_s = run_leg(rp, path, ctx, d, rp.RP_SPLIT_BF16, args.steps, args.warmup,
                                          args.kbatch)
    chi_s = chi_s.clone()
    einv_s = einv_s.clone()
    wij_s = wij_s.clone()
    x6 = None
    if not args.no_x6:
        x6, _, _, _ = run_leg(rp, path, ctx, d, rp.RP_SPLIT_BF16_X6, args.x6_steps, args.x6_warmup, args.kbatch)
    fp64 = None
    agree = None
    if not args.no_fp64:
        fp64, chi_d, einv_d, wij_d = run_leg(rp, path, ctx, d, rp.RP_FP64, args.fp64_steps, args.fp64_warmup,
                                             args.kbatch)

        def rel(a, b):
            a = torch.view_as_complex(a)
            b = torch.view_as_complex(b)
            fro = max(float(torch.linalg.norm(a[f] - b[f]) / torch.linalg.norm(b[f])) for f in range(b.shape[0]))
            ew = max(float((a[f] - b[f]).abs().max() / b[f].abs().max()) for f in range(b.shape[0]))
            return fro, ew

        wd = torch.view_as_complex(wij_d)
        (c_f, c_e), (e_f, e_e) = rel(chi_s, chi_d), rel(einv_s, einv_d)
        agree = {
            "reference": "the GPU's FP64 path on the same q-point (its own parity with the oracle, and the "
                         "split path's at this launch shape, are tested in tests/test_gpu_fullsize.py)",
            "chi": c_f,
            "chi_max_elementwise": c_e,
            "eps_inv": e_f,
            "eps_inv_max_elementwise": e_e,
            "W_ij_max_elementwise": float((torch.abs(torch.view_as_complex(wij_s) - wd) / torch.abs(wd)).max()),
        }
    vs_oracle = None if baseline is None else oracle_sample_errors(rp, path, ctx, d, baseline)
    qterm = None if args.no_qterm else qterm_leg(rp, path, ctx, d, einv_s,
                                                 cpu=not args.no_cpu_baseline and not args.profile_k)
    unfold = None if args.no_qterm else unfold_leg(rp, ctx, d, einv_s)
    metal_w = None if args.no_qterm else metal_weights_leg(rp, ctx, d)
    drude_o = None if args.no_qterm else drude_leg(rp, ctx, d)
    ctx.close()
    sc_leg = batch_o = None
    if not args.no_extra_legs:
        # (the 48^3 arrays stay resident: 288 GB of HBM hold all three workloads)
        sc_leg = supercell_measure(args)
        torch.cuda.empty_cache()
        batch_o = batch_measure(args, embedded=True)
        torch.cuda.empty_cache()

    npair_total = d.nk * prob.nocc * prob.nemp
    pair_grid = rp.rp_pair_grid(d.cell, prob.iq, d.mmax, prob.gsph, rp.RP_SPLIT_BF16)
    achieved = split["chi_kernel_flops_per_launch"] / (split["chi_kernel_ms_per_launch"] / 1e3) / 1e12
    rec = recorded_traffic()
    pc = recorded_pair_counters()
    hbm = None
    if pc is not None:
        t_pair = split["stage_ms_per_step"]["pair"] / d.nk / 1e3      # s per k-point (one launch)
        t_ugrid = split["stage_ms_per_step"]["ugrid"] / d.nk / 1e3
        alg = (prob.nocc + prob.nemp) * int(np.prod(pair_grid)) * 8 + prob.nocc * prob.nemp * d.ng * 16
        hbm = {
            "pair_kernel": {"bytes_per_launch": pc["pair_bytes_per_launch"], "ms_per_launch": t_pair * 1e3,
                            "achieved_GB_s": pc["pair_bytes_per_launch"] / t_pair / 1e9,
                            "algorithmic_bytes_per_launch": alg,
                            "algorithmic_GB_s": alg / t_pair / 1e9, "peak_GB_s": PEAK_HBM_GBS},
            "ugrid_kernels": {"bytes_per_k": pc["ugrid_bytes_per_k"], "ms_per_k": t_ugrid * 1e3,
                              "achieved_GB_s": pc["ugrid_bytes_per_k"] / t_ugrid / 1e9,
                              "peak_GB_s": PEAK_HBM_GBS},
        }
    out = {
        "metric": METRIC,
        "value": split["chi0_tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": split["s_per_qpoint"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "SrVO3-shaped q-point: 48^3 grid, 8^3 k mesh, 40+200 bands, N_G=1500, "
                        "20 real frequencies, delta=0.1 eV, generalized tetrahedron, 10 Wannier orbitals",
            "pairs": npair_total,
            "ng": d.ng,
            "nfreq": d.nfreq,
            "kbatch": args.kbatch,
            "pair_grid": list(pair_grid),
            "precision": "split-BF16 chi0 (hi/mid BF16 terms, three-term compensated products, FP32 "
                         "accumulation, FP64 sum; FP32 pair-density grids), FP64 weights, eps^-1 and W_ij",
        },
        "s_per_qpoint": split["s_per_qpoint"],
        "split_bf16": split,
        "split_bf16_x6": x6,
        "fp64": fp64,
        "split_vs_gpu_fp64": agree,
        "vs_oracle_sample": vs_oracle,
        "roofline": {
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_BF16_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_BF16_TFLOPS,
            "traffic": None if rec is None else rec["traffic_bytes_per_launch"],
            "kernel": "k_chi_rows (chi0 contraction, split-BF16)",
            "mfma_executed_frac": 3.0 * achieved / PEAK_BF16_TFLOPS,
            "mfma_counter_frac": None if rec is None or "mfma_mops_per_launch" not in rec else
            rec["mfma_mops_per_launch"] * 512.0 / (split["chi_kernel_ms_per_launch"] / 1e3) / 1e12 /
            PEAK_BF16_TFLOPS,
        },
        "hbm_a2_a4": hbm,
        "interaction_qterm": qterm,
        "symmetry_unfold": unfold,
        "metal_weights": metal_w,
        "drude_plasma": drude_o,
        "supercell": sc_leg,
        "batch": batch_o,
        "cpu_baseline": None if baseline is None else {k: baseline[k] for k in
                                                        ("value", "unit", "cores", "cpu_model", "kind",
                                                         "sample", "seconds", "s_per_qpoint_extrapolated",
                                                         "extrapolation")},
    }
    if fp64 is not None:
        a64 = fp64["chi_kernel_flops_per_launch"] / (fp64["chi_kernel_ms_per_launch"] / 1e3) / 1e12
        out["fp64"]["roofline"] = {"bound": "mfma", "achieved": a64, "peak": PEAK_FP64_TFLOPS,
                                   "unit": "TFLOP/s", "frac": a64 / PEAK_FP64_TFLOPS,
                                   "kernel": "k_chi_f64 (chi0 contraction, FP64)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
