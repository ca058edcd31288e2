"""Benchmark of the Lomb-Scargle periodogram hot path on one MI355X.

Default workload (single_4096): one object with N_t = 4,096 seasonal-cadence
observations, N_f = 500,000 frequencies over [0.5, 24) cycles/day, full FP32
periodogram (2 MB) plus the peak.  One step = one lsp_single call of the FP32
form (prep, main kernel, FP64 fix-up check, combine, peak), inputs resident in
HBM.  The plain FP64 form is timed on the same input for the "vs plain FP64
kernel" comparison, and the two periodograms are compared for peak-bin
agreement.  The oracle (CPU, FP64) is timed on a bounded sample of the same
workload on this host's cores.

``--method generalized`` times the generalized periodogram instead (Section
4.11: per-point errors, floating mean) on the same workload drawn with
photometric errors, and also times the standard periodogram on that input to
report the cost ratio the paper measures (generalized / standard).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LS obs×freq evals/s and objects/s vs plain FP64 kernel at peak-bin agreement"
# FP32 form, algorithmic flops per eval: 4 FMA for the sums (8 flops) plus the
# recurrence, 2 mul + 2 FMA for a rotation (6 flops) or 2 FMA for the
# three-term (Chebyshev) recurrence (4 flops).
FLOPS_PER_EVAL = {"rotation": 14, "chebyshev": 12}
# Generalized FP32 form: 6 FMA for the sums (12 flops) plus the three-term
# recurrence's 2 FMA (4 flops).
FLOPS_PER_EVAL_GEN = 16
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 2.4 GHz x 64 flops/clock/SIMD
# (32 FMA lanes per clock), the published 157.3 TFLOP/s.
PEAK_FP32_TFLOPS = 256 * 4 * 2.4e9 * 64 / 1e12
# VALU instructions per observation and lane in the compiled gfx950 loop, for
# K frequencies per lane: 4K for the sums, the recurrence (4(K-1) for rotations;
# 4 + 2(K-2) for Chebyshev), and 9-10 per-observation instructions (FP64
# phase, cvt, 2 transcendentals, moves).  K = 16 compiles to 133 and 106.
def valu_ops_per_eval(rec, k):
    if rec == "chebyshev":
        return (4 * k + 4 + 2 * (k - 2) + 10) / k
    return (4 * k + 4 * (k - 1) + 9) / k


# Generalized form: 6K for the sums, 4 + 2(K-2) for the recurrence and about
# 12 per observation (the standard form's 10 plus the two seed scalings).
def valu_ops_per_eval_gen(k):
    return (6 * k + 4 + 2 * (k - 2) + 12) / k


KERNEL_SOURCES = {
    "standard": ["paper_2105_04006_amd/csrc/lsp_fp32p.hip", "paper_2105_04006_amd/csrc/lsp_common.h"],
    "generalized": ["paper_2105_04006_amd/csrc/lsp_gen.hip",
                    "paper_2105_04006_amd/csrc/lsp_common.h"],
}
TRAFFIC_FILES = {
    "standard": os.path.join(ROOT, "profiles", "fp32p_single_4096_traffic.json"),
    "generalized": os.path.join(ROOT, "profiles", "gen_fp32p_single_4096_traffic.json"),
    ("standard", "batch_10k"): os.path.join(ROOT, "profiles", "fp32p_batch_10k_traffic.json"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash(method="standard"):
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[method]:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(method="standard", workload="single_4096"):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source and this workload."""
    path = TRAFFIC_FILES.get((method, workload), TRAFFIC_FILES[method])
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash(method) or rec.get("workload_name") != workload:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(w, target_evals, threads, method="standard"):
    """The oracle on a bounded sample of the same workload: every m-th bin of
    the object (one object), or every bin of the first objects (a batch)."""
    import oracle

    oracle.default()
    if w.n_obj == 1:
        stride = max(1, int(round(w.evals / target_evals)))
        bins = np.arange(0, w.n_f, stride, dtype=np.int64)
        objs = np.zeros(len(bins), dtype=np.int64)
        what = f"every {stride}th of the {w.n_f} bins ({len(bins)} bins x {w.n_obs} obs"
    else:
        per_obj = w.n_f * np.diff(w.offsets)
        k = max(1, int(np.searchsorted(np.cumsum(per_obj), target_evals)))
        stride = max(1, int(round(per_obj[:k].sum() / target_evals)))
        bins1 = np.arange(0, w.n_f, stride, dtype=np.int64)
        objs = np.repeat(np.arange(k, dtype=np.int64), len(bins1))
        bins = np.tile(bins1, k)
        what = f"every {stride}th bin of the first {k} objects ({len(bins)} (object, bin) pairs"
    t0 = time.perf_counter()
    if method == "generalized":
        vals = oracle.gen_eval_bins(w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, w.n_f, objs,
                                    bins, threads=threads)
    else:
        vals = oracle.eval_bins(w.offsets, w.t, w.y, w.f_min, w.f_max, w.n_f, objs, bins,
                                threads=threads)
    dt = time.perf_counter() - t0
    n_t = np.diff(w.offsets)
    evals = int(n_t[objs].sum())
    return {"value": evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}, {evals:.3g} evals) of the same workload, {dt:.2f} s wall"}, \
        (objs, bins, vals)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="single_4096")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--recurrence", default="auto", choices=["auto", "rotation", "chebyshev"])
    ap.add_argument("--k", type=int, default=0, help="frequencies per lane (0: library default)")
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--schedule", default="auto", choices=["auto", "grid", "persistent"])
    ap.add_argument("--cpu-evals", type=float, default=6e8,
                    help="oracle evaluations in the CPU-baseline sample (about 10-30 s of CPU work)")
    ap.add_argument("--fp64-steps", type=int, default=0,
                    help="timed steps of the FP64 reference form (default steps // 8, >= 3)")
    ap.add_argument("--mode", default="lsp", choices=["lsp", "copy"],
                    help="copy: time a plain device-to-device copy of --copy-bytes bytes "
                         "(calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--copy-bytes", type=float, default=256 * 2**20)
    ap.add_argument("--launch", default="eager", choices=["eager", "graph"],
                    help="graph: each timed FP32 step replays the call captured once as a HIP "
                         "graph (lsp_plan_*)")
    ap.add_argument("--method", default="standard", choices=["standard", "generalized"],
                    help="generalized: the periodogram with per-point errors and a floating "
                         "mean (Section 4.11), on the workload drawn with errors")
    ap.add_argument("--obs-read", default="auto", choices=["auto", "lds", "direct"],
                    help="FP32 form: observations staged in LDS, or read from global memory "
                         "after a staging pass")
    ap.add_argument("--seed-trig", default="auto", choices=["auto", "hw", "lib", "poly"],
                    help="FP32 form: sin/cos of the reduced seed phases by the hardware, the "
                         "math library's sincospif, or Taylor polynomials")
    ap.add_argument("--recovery", action="store_true",
                    help="asteroid-like population (asteroids_1k): derived vs assigned rotation "
                         "periods and the observation-cutoff curve, standard and generalized, "
                         "FP32 and FP64 forms")
    ap.add_argument("--host-return", action="store_true",
                    help="time the whole batch periodogram returned to host memory: one copy of "
                         "the device periodogram into pageable memory against the pinned-staging "
                         "pipeline (lsp_batch_to_host); PCIe-inclusive, not the headline value")
    ap.add_argument("--learned", action="store_true",
                    help="time the learned band-proposal path on --workload (always on for "
                         "learned_100k)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the periodogram of "
              "independent objects would shard by object across GPUs, which is not "
              "implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.mode == "copy":
        n = int(args.copy_bytes) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(args.warmup):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "ms_per_copy": dt * 1e3, "GB_per_s": 8 * n / dt / 1e9}), flush=True)
        return

    from paper_2105_04006_amd import lsp, synth

    lsp.lib()  # fails loudly if the HIP library is not built
    dev = torch.device("cuda:0")
    if args.workload == "learned_100k" or args.learned:
        return bench_learned(args, torch, dev)
    if args.host_return:
        return bench_host_return(args, torch, dev)
    if args.recovery:
        return bench_recovery(args, torch, dev)
    gen = args.method == "generalized"
    w = synth.make_workload(args.workload, errors=gen)
    single = w.n_obj == 1
    log(f"[bench] workload {w.name}: n_obj={w.n_obj} n_obs={w.n_obs} n_f={w.n_f} "
        f"evals={w.evals:.3e}")
    t = torch.as_tensor(w.t, device=dev)
    y = torch.as_tensor(w.y, device=dev)
    off = None if single else torch.as_tensor(w.offsets, device=dev)
    kw = dict(offsets=off, pgram=single, peaks=True)
    rec = {"auto": lsp.REC_AUTO, "rotation": lsp.REC_ROTATION,
           "chebyshev": lsp.REC_CHEBYSHEV}[args.recurrence]
    sched = {"auto": lsp.SCHED_AUTO, "grid": lsp.SCHED_GRID,
             "persistent": lsp.SCHED_PERSISTENT}[args.schedule]
    if gen:
        kw.update(method="generalized", dy=torch.as_tensor(w.dy, device=dev))
    obs = {"auto": 0, "lds": lsp.OBS_LDS, "direct": lsp.OBS_DIRECT}[args.obs_read]
    trig = {"auto": 0, "hw": lsp.TRIG_HW, "lib": lsp.TRIG_LIB, "poly": lsp.TRIG_POLY}[args.seed_trig]
    variant = obs == lsp.OBS_DIRECT or trig in (lsp.TRIG_LIB, lsp.TRIG_POLY)
    kv = dict(obs_read=obs, seed_trig=trig) if variant else {}
    p32 = lsp.Periodogram(t, y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP32P, schedule=sched,
                          recurrence=rec, k=args.k, waves=args.waves, **kw, **kv)
    p64 = lsp.Periodogram(t, y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP64, **kw)

    def timed(fn, steps):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    step32 = p32.capture() if args.launch == "graph" else p32
    for _ in range(args.warmup):
        step32()
    p64()
    torch.cuda.synchronize()
    log("[bench] warm-up done")
    ms32 = timed(step32, args.steps)
    log(f"[bench] fp32p {ms32:.4f} ms/step ({args.launch})")
    steps64 = args.fp64_steps if args.fp64_steps > 0 else max(3, args.steps // 8)
    ms64 = timed(p64, steps64)
    log(f"[bench] fp64 {ms64:.4f} ms/step ({steps64} steps)")
    std_cost = None
    if gen:
        # the standard periodogram of the same input, for the cost ratio
        kws = dict(offsets=off, pgram=single, peaks=True)  # standard, default variant
        s32 = lsp.Periodogram(t, y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP32P, **kws)
        s64 = lsp.Periodogram(t, y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP64, **kws)
        s32()
        s64()
        ms_s32 = timed(s32, args.steps)
        ms_s64 = timed(s64, steps64)
        std_cost = {"fp32_ms_per_step": ms_s32, "fp64_ms_per_step": ms_s64,
                    "generalized_over_standard_fp32": ms32 / ms_s32,
                    "generalized_over_standard_fp64": ms64 / ms_s64}
        log(f"[bench] standard fp32p {ms_s32:.4f} ms, fp64 {ms_s64:.4f} ms; generalized/standard "
            f"{ms32 / ms_s32:.2f}x (fp32), {ms64 / ms_s64:.2f}x (fp64)")

    # dominant kernel's own device time, from events the library records
    # around the main kernel on its launch stream
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(args.steps)]
    for a, b in pairs:
        a.record()
        b.record()
    torch.cuda.synchronize()
    for a, b in pairs:
        lsp.set_stage_events(a.cuda_event, b.cuda_event)
        p32()
    lsp.set_stage_events(None, None)
    torch.cuda.synchronize()
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in pairs]))
    log(f"[bench] fp32p main kernel {k_ms:.4f} ms/launch")

    pk32, pk64 = p32.peaks(), p64.peaks()
    agree = np.abs(pk32["index"] - pk64["index"]) <= 1
    if single:
        d = (p32.pgram.double() - p64.pgram.double()).abs().max().item()
    else:
        d = float(np.max(np.abs(pk32["power"] - pk64["power"])))

    evals = w.evals
    value = evals / (ms32 * 1e-3)
    rec_name = "rotation" if args.recurrence == "rotation" else "chebyshev"  # auto = chebyshev
    k_lane = args.k if args.k else 16
    flops_eval = FLOPS_PER_EVAL_GEN if gen else FLOPS_PER_EVAL[rec_name]
    achieved = flops_eval * evals / (k_ms * 1e-3) / 1e12
    valu_ops = (valu_ops_per_eval_gen(k_lane) if gen else valu_ops_per_eval(rec_name, k_lane)) \
        * evals / (k_ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_obj": w.n_obj, "n_t": int(w.n_obs) if single else
                   "U{%d..%d}" % (int(w.n_t.min()), int(w.n_t.max())), "n_obs": int(w.n_obs),
                   "n_f": w.n_f, "f_range_cycles_per_day": [w.f_min, w.f_max],
                   "form": "fp32 sums, fp64 phase reduction", "output": "pgram f32 + peak"
                   if single else "peaks", "launch": args.launch,
                   "method": "generalized (errors 1/dy^2, floating mean)" if gen else "standard"},
        "objects_per_s": w.n_obj / (ms32 * 1e-3),
        "pgram_bytes_per_step": (4 * w.n_f * w.n_obj) if single else 0,
        "pgram_write_GBps": (4 * w.n_f * w.n_obj / (ms32 * 1e-3) / 1e9) if single else 0.0,
        "fp64_reference": {"evals_per_s": evals / (ms64 * 1e-3), "ms_per_step": ms64,
                           "objects_per_s": w.n_obj / (ms64 * 1e-3)},
        "speedup_vs_fp64": ms64 / ms32,
        "peak_bin_agreement": float(agree.mean()),
        "generalized_vs_standard": std_cost,
        "max_abs_dpower_vs_fp64": d,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": None if variant else measured_traffic(args.method, w.name),
            "kernel": "gen_fp32p_kernel" if gen else "fp32p_kernel",
            "kernel_ms": k_ms,
            "flops_per_eval": flops_eval,
            "recurrence": rec_name,
            "k_per_lane": k_lane,
            "valu_lane_ops_per_s": None if variant else valu_ops,
            "valu_issue_frac": None if variant else valu_ops / (PEAK_FP32_TFLOPS * 1e12 / 2),
            "obs_read": args.obs_read,
            "seed_trig": args.seed_trig,
            "transcendentals_per_s": 2 * evals / k_lane / (k_ms * 1e-3),
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        threads = min(16, len(os.sched_getaffinity(0)))
        log(f"[bench] oracle baseline on {threads} threads")
        out["cpu_baseline"], (objs, bins, ora_vals) = cpu_baseline(w, args.cpu_evals, threads,
                                                                   args.method)
        # the FP32 form's power at the same (object, bin) pairs, against the
        # oracle: the bench line states its error against the FP64 oracle
        if single:
            got = p32.pgram[0][torch.as_tensor(bins, device=dev)].double().cpu().numpy()
        else:
            k = int(objs.max()) + 1
            sub = lsp.Periodogram(t, y, w.f_min, w.f_max, w.n_f, offsets=off[:k + 1],
                                  form=lsp.FORM_FP32P, schedule=sched, recurrence=rec, k=args.k,
                                  waves=args.waves, method=kw.get("method", "standard"),
                                  dy=kw.get("dy"), pgram=True, peaks=False, **kv)
            sub()
            flat = torch.as_tensor(objs * w.n_f + bins, device=dev)
            got = sub.pgram.view(-1)[flat].double().cpu().numpy()
        out["oracle_check"] = {"pairs": int(len(bins)),
                               "max_abs_dpower_vs_oracle": float(np.max(np.abs(got - ora_vals))),
                               "form": "fp32 (the timed form)"}
    print(json.dumps(out), flush=True)


CUTOFFS = (0, 25, 50, 75, 100, 150, 200, 300, 400, 550)


def recovery_curve(p_rot_true_h, p_lc_days, n_t, tol_h=0.1):
    """Fraction of objects whose derived rotation period (twice the light-curve
    period at the peak) is within tol_h of the assigned one, overall and for
    every observation cutoff (objects with at least that many points)."""
    derived = 2.0 * 24.0 * np.asarray(p_lc_days, dtype=np.float64)
    ok = np.abs(derived - p_rot_true_h) <= tol_h
    curve = []
    for c in CUTOFFS:
        m = n_t >= c
        curve.append({"cutoff": c, "objects": int(m.sum()),
                      "matched": float(ok[m].mean()) if m.any() else None})
    return float(ok.mean()), curve, ok


def bench_recovery(args, torch, dev):
    """Section 4.2's accuracy study on an asteroid-like population: the peak
    of each object's periodogram on the paper's batch grid (rad/day,
    N_f = 200,000) gives the light-curve period; twice it should match the
    assigned rotation period within 0.1 h.  Timed as whole batches."""
    from paper_2105_04006_amd import lsp, synth

    w = synth.make_workload("asteroids_1k")
    n_t = np.diff(w.offsets)
    log(f"[bench] recovery: {w.name} n_obj={w.n_obj} n_obs={w.n_obs} n_f={w.n_f} "
        f"N_t median {int(np.median(n_t))}")
    off = torch.as_tensor(w.offsets, device=dev)
    t = torch.as_tensor(w.t, device=dev)
    y = torch.as_tensor(w.y, device=dev)
    dy = torch.as_tensor(w.dy, device=dev)
    runs = {}
    for name, form, method in (("standard_fp32", lsp.FORM_FP32P, "standard"),
                               ("standard_fp64", lsp.FORM_FP64, "standard"),
                               ("generalized_fp32", lsp.FORM_FP32P, "generalized"),
                               ("generalized_fp64", lsp.FORM_FP64, "generalized")):
        p = lsp.Periodogram(t, y, w.f_min, w.f_max, w.n_f, offsets=off, unit=lsp.ANGULAR,
                            form=form, method=method, dy=dy if method == "generalized" else None,
                            pgram=False, peaks=True)
        p()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 3 if form == lsp.FORM_FP32P else 1
        for _ in range(steps):
            p()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        pk = p.peaks()
        frac, curve, ok = recovery_curve(w.p_rot_hours, pk["period"], n_t)
        runs[name] = {"ms_per_batch": ms, "objects_per_s": w.n_obj / (ms * 1e-3),
                      "matched": frac, "curve": curve, "index": pk["index"]}
        log(f"[bench] {name}: {ms:.2f} ms, matched {frac:.4f}, "
            f"N_t>=50 {curve[2]['matched']:.4f}")
    agree = {
        "standard fp32 vs fp64": float(np.mean(np.abs(runs["standard_fp32"]["index"]
                                                      - runs["standard_fp64"]["index"]) <= 1)),
        "generalized fp32 vs fp64": float(np.mean(np.abs(runs["generalized_fp32"]["index"]
                                                         - runs["generalized_fp64"]["index"])
                                                  <= 1)),
    }
    for r in runs.values():
        del r["index"]
    in_grid = float(np.mean(w.p_rot_hours / 2.0 <= 2 * np.pi / w.f_min * 24.0))
    out = {
        "metric": "recovered rotation periods (within 0.1 h) on an asteroid-like population",
        "value": runs["standard_fp32"]["matched"],
        "unit": "fraction of objects",
        "n_gpus": 1,
        "steps": 3,
        "warmup": 1,
        "ms_per_step": runs["standard_fp32"]["ms_per_batch"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_obj": w.n_obj, "n_obs": int(w.n_obs), "n_f": w.n_f,
                   "grid_rad_per_day": [w.f_min, w.f_max],
                   "n_t": "log-normal, median %d, [%d, %d]" % (int(np.median(n_t)),
                                                                int(n_t.min()), int(n_t.max())),
                   "output": "peaks"},
        "paper_context": "94.9% of ~1,000 synthetic asteroids within 0.1 h; 99% with >= 50 "
                         "observations; 100% for the 45 objects with >= 550 (Section 4.2)",
        "rotation_period_on_grid": in_grid,
        "runs": runs,
        "peak_agreement_within_one_bin": agree,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_host_return(args, torch, dev):
    """Section 3.5: periodograms of a whole batch returned to host memory.

    standard: lsp_batch into a device periodogram, then one device-to-host
    copy into pageable memory (the driver stages it); pipelined: the
    pinned-staging pipeline, chunk by chunk with host copy threads.  Both are end-to-end (kernels + transfer), inputs resident on the
    device, destination pages touched beforehand."""
    from paper_2105_04006_amd import lsp, synth

    gen = args.method == "generalized"
    w = synth.make_workload(args.workload, errors=gen)
    nbytes = 4 * w.n_obj * w.n_f
    log(f"[bench] host return: {w.name} n_obj={w.n_obj} n_f={w.n_f}, {nbytes / 1e9:.2f} GB FP32")
    off = torch.as_tensor(w.offsets, device=dev)
    t = torch.as_tensor(w.t, device=dev)
    y = torch.as_tensor(w.y, device=dev)
    dy = torch.as_tensor(w.dy, device=dev) if gen else None
    method = "generalized" if gen else "standard"
    host_a = np.zeros((w.n_obj, w.n_f), dtype=np.float32)
    host_b = np.zeros((w.n_obj, w.n_f), dtype=np.float32)
    ta = torch.from_numpy(host_a)
    p = lsp.Periodogram(t, y, w.f_min, w.f_max, w.n_f, offsets=off, form=lsp.FORM_FP32P,
                        method=method, dy=dy, pgram=True, peaks=True)
    pipe = lsp.HostPipe()

    def standard():
        p()
        ta.copy_(p.pgram)  # synchronous device-to-pageable copy
        p.peaks()

    def pipelined():
        pipe.batch_to_host(off, t, y, w.f_min, w.f_max, w.n_f, dy=dy, method=method,
                           form=lsp.FORM_FP32P, out=host_b)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    steps = max(1, min(args.steps, 5))
    for _ in range(max(1, args.warmup if args.warmup < 3 else 1)):
        standard()
        pipelined()
    ms_std = timed(standard, steps)
    log(f"[bench] standard (kernels + one copy to pageable memory) {ms_std:.1f} ms")
    ms_pipe = timed(pipelined, steps)
    log(f"[bench] pipelined (pinned staging, copy threads) {ms_pipe:.1f} ms")
    p()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p()
    torch.cuda.synchronize()
    ms_kern = (time.perf_counter() - t0) / steps * 1e3
    same = bool(np.array_equal(host_a, host_b))
    out = {
        "metric": METRIC + " (periodograms returned to host memory, PCIe-inclusive)",
        "value": w.evals / (ms_pipe * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": ms_pipe,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_obj": w.n_obj, "n_obs": int(w.n_obs), "n_f": w.n_f,
                   "output": "pgram f32 to host + peaks", "method": method},
        "host_return": {
            "pgram_bytes": nbytes,
            "standard_ms": ms_std,
            "pipelined_ms": ms_pipe,
            "device_only_ms": ms_kern,
            "speedup_pipelined_vs_standard": ms_std / ms_pipe,
            "standard_GBps": nbytes / (ms_std * 1e-3) / 1e9,
            "pipelined_GBps": nbytes / (ms_pipe * 1e-3) / 1e9,
            "identical_results": same,
            "pipe": "library defaults: 1 lane (kernel + copy stream, two chunk buffers), "
                    "16 MiB pinned staging (two halves), 128 MiB chunks, 12 copy threads",
        },
        "roofline": None,
        "cpu_baseline": None,
    }
    pipe.close()
    print(json.dumps(out), flush=True)


def bench_learned(args, torch, dev):
    """Learned band proposal on a batch workload (learned_100k: 1e5 objects,
    N_t 50..500, N_f 2e5 over [1, 12) cycles/day, 64 bands of 3,125 bins, top 8
    refined; lsst_200k with --learned: 2e5 objects with harmonics and noise).

    Untimed set-up: train the proposal network on 40,000 independent objects
    (labels: whole-grid FP32 peaks), calibrate the fallback thresholds on
    20,000 more for >= 99.9% recovery.  Timed step: features -> network ->
    top bands -> refine -> fallback selection -> whole-grid fallback, ending
    with the peaks of all 1e5 objects.  Compared with the whole-grid FP32 batch
    (same peaks, every bin) and the plain FP64 form."""
    from paper_2105_04006_amd import learned, lsp, synth

    gen = args.method == "generalized"
    method = "generalized" if gen else "standard"

    def tens(w):
        return (torch.as_tensor(w.offsets, device=dev), torch.as_tensor(w.t, device=dev),
                torch.as_tensor(w.y, device=dev))

    def errs(w):
        return torch.as_tensor(w.dy, device=dev) if gen else None

    def full(w, tt, form=lsp.FORM_FP32P):
        return lsp.Periodogram(tt[1], tt[2], w.f_min, w.f_max, w.n_f, offsets=tt[0], form=form,
                               pgram=False, unit=w.unit, method=method, dy=errs(w))

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    name = args.workload
    w = synth.make_workload(name, errors=gen) if name != "asteroids_100k" else \
        synth.make_workload(name)
    geo = learned.BandGeometry(w.n_f, 64)
    log(f"[bench] learned: n_obj={w.n_obj} n_obs={w.n_obs} n_f={w.n_f} "
        f"bands of {geo.band_bins}")
    def make(n_obj, seed):
        if name.startswith("asteroids"):
            return synth.make_workload(name, n_obj=n_obj, seed=seed)
        return synth.make_workload(name, n_obj=n_obj, seed=seed, errors=gen)

    wtr = make(40000, synth.SEED_BASE + 1000)
    ttr = tens(wtr)
    feats = lsp.Features(*ttr, wtr.f_min, wtr.f_max, unit=wtr.unit)()
    ptr = full(wtr, ttr)
    ptr()
    labels = learned.peak_bands(ptr.peaks_raw, wtr.n_obj, geo.band_bins, geo.n_bands)
    net = learned.BandNet(dev, seed=7)
    t0 = time.perf_counter()
    hist = learned.train_proposer(net, feats, labels, epochs=30, batch=512, lr=1e-3,
                                  lr_final=3e-5, augment=0.9)
    log(f"[bench] trained in {time.perf_counter() - t0:.1f} s, loss {hist[0]:.3f} -> "
        f"{hist[-1]:.3f}")
    del feats, ptr, ttr
    wva = make(20000, synth.SEED_BASE + 1001)
    tva = tens(wva)
    lpv = learned.LearnedPeriodogram(net, geo, *tva, wva.f_min, wva.f_max, unit=wva.unit,
                                     method=method, dy=errs(wva))
    lpv.refine_only()
    pva = full(wva, tva)
    pva()
    mass_min, power_min, n_fb = learned.calibrate(lpv.peaks(), pva.peaks(),
                                                  lpv.mass.cpu().numpy(), target=0.999)
    log(f"[bench] calibrated mass_min={mass_min:.4f} power_min={power_min:.4f}: "
        f"{n_fb}/{wva.n_obj} validation fallbacks")
    del lpv, pva, tva

    tt = tens(w)
    lp = learned.LearnedPeriodogram(net, geo, *tt, w.f_min, w.f_max, mass_min=mass_min,
                                    power_min=power_min, unit=w.unit, method=method, dy=errs(w))
    p32 = full(w, tt)
    p64 = full(w, tt, lsp.FORM_FP64)
    for _ in range(max(1, args.warmup)):
        lp()
        p32()
    ms_l = timed(lp, args.steps)
    log(f"[bench] learned {ms_l:.3f} ms/step ({lp.n_fallback} fallbacks)")
    ms_32 = timed(p32, args.steps)
    log(f"[bench] whole-grid fp32 {ms_32:.3f} ms/step")
    ms_64 = timed(p64, max(1, args.fp64_steps))
    log(f"[bench] whole-grid fp64 {ms_64:.3f} ms/step")

    # stage breakdown of one learned step (events on the current stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    lp.propose()
    ev[1].record()
    lp.refine()
    ev[2].record()
    learned.select_fallback(lp.peaks_raw, lp.mass, lp.n_obj, mass_min, power_min, lp.objects,
                            lp.count)
    n = int(lp.count.item())
    if n:
        lp.full.set_rows(lp.objects[:n])
        lp.full()
    ev[3].record()
    torch.cuda.synchronize()
    stages = {"features_network_topk_ms": ev[0].elapsed_time(ev[1]),
              "refine_ms": ev[1].elapsed_time(ev[2]),
              "select_fallback_ms": ev[2].elapsed_time(ev[3])}

    pk, ref32, ref64 = lp.peaks(), p32.peaks(), p64.peaks()
    ok = ref32["status"] == 0
    # proposal quality: does the whole-grid peak's band sit among the 8
    # proposed bands?  Compared with the no-network heuristic that takes the
    # 8 bands with the largest pooled coarse value.
    lp.refine_only()
    net8, _ = learned.top_bands(lp.logits, lp.top)
    torch.cuda.synchronize()
    band = ref32["index"] // geo.band_bins

    def hit(idx):
        return float(np.mean((idx.cpu().numpy() == band[:, None]).any(axis=1)[ok]))

    hit_used, hit_net = hit(lp.idx), hit(net8)
    # diagnostic: coverage if part of the refined bands were the one-day
    # aliases (f +- 1 cycle/day) of the first proposals
    alias_bins = (2 * np.pi if w.unit == 1 else 1.0) / ((w.f_max - w.f_min) / w.n_f)
    used = lp.idx.cpu().numpy().astype(np.int64)

    def alias_cover(n_first, n_alias):
        first = used[:, :n_first]
        cand = [first]
        centre = (first[:, :n_alias] + 0.5) * geo.band_bins
        for sgn in (-1, 1):
            a = np.floor((centre + sgn * alias_bins) / geo.band_bins).astype(np.int64)
            cand.append(np.where((a >= 0) & (a < geo.n_bands), a, -1))
        c = np.concatenate(cand, axis=1)
        return float(np.mean((c == band[:, None]).any(axis=1)[ok]))

    def expand_cover(n_first, n_exp, fn):
        first = used[:, :n_first]
        cand = [first]
        for g in fn:
            a = g(first[:, :n_exp])
            cand.append(np.where((a >= 0) & (a < geo.n_bands), a, -1))
        c = np.concatenate(cand, axis=1)
        return float(np.mean((c == band[:, None]).any(axis=1)[ok]))

    def fband(b, scale):  # band holding scale x the frequency at band b's centre
        f = w.f_min + (b + 0.5) * geo.band_bins * (w.f_max - w.f_min) / w.n_f
        return np.floor((scale * f - w.f_min) / (w.f_max - w.f_min) * w.n_f
                        / geo.band_bins).astype(np.int64)

    alias_hits = {"top4+aliases_of_top2": alias_cover(4, 2), "top6+aliases_of_top1": alias_cover(6, 1),
                  "top2+aliases_of_top2": alias_cover(2, 2), "top8": alias_cover(8, 0),
                  "top4+neighbours_of_top2": expand_cover(4, 2, (lambda b: b - 1, lambda b: b + 1)),
                  "top4+half_double_of_top2": expand_cover(4, 2, (lambda b: fband(b, 0.5),
                                                                  lambda b: fband(b, 2.0))),
                  "top16": float(np.mean((np.argsort(-lp.logits.float().cpu().numpy(), axis=1)
                                          [:, :16] == band[:, None]).any(axis=1)[ok]))}
    log(f"[bench] alias coverage {alias_hits}")
    hit_heur = hit(lp.idx_coarse) if lp.proposal == "hybrid" else None
    refine_only = lp.peaks()
    rec_refine = float(np.mean(np.abs(refine_only["index"][ok] - ref32["index"][ok]) <= 1))
    rec32 = float(np.mean(np.abs(pk["index"][ok] - ref32["index"][ok]) <= 1))
    rec64 = float(np.mean(np.abs(pk["index"][ok] - ref64["index"][ok]) <= 1))
    evals = w.evals
    refine_evals = float(np.sum(np.diff(w.offsets))) * 8 * geo.band_bins
    out = {
        "metric": METRIC, "value": evals / (ms_l * 1e-3), "unit": "evals/s (whole-grid equivalent)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_l,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": w.name, "n_obj": w.n_obj,
                   "n_t": "%d..%d" % (int(np.diff(w.offsets).min()), int(np.diff(w.offsets).max())),
                   "n_obs": int(w.n_obs), "n_f": w.n_f, "f_range": [w.f_min, w.f_max],
                   "unit": "rad/day" if w.unit == 1 else "cycles/day",
                   "bands": geo.n_bands, "band_bins": geo.band_bins, "top": lp.top,
                   "network": "1088-512-256-64 BF16 MFMA", "output": "peaks", "method": method},
        "objects_per_s": w.n_obj / (ms_l * 1e-3),
        "whole_grid_fp32": {"ms_per_step": ms_32, "objects_per_s": w.n_obj / (ms_32 * 1e-3),
                            "evals_per_s": evals / (ms_32 * 1e-3)},
        "fp64_reference": {"ms_per_step": ms_64, "objects_per_s": w.n_obj / (ms_64 * 1e-3),
                           "evals_per_s": evals / (ms_64 * 1e-3)},
        "speedup_vs_whole_grid_fp32": ms_32 / ms_l, "speedup_vs_fp64": ms_64 / ms_l,
        "fallback_objects": lp.n_fallback, "refined_evals": refine_evals,
        "peak_bin_agreement": rec32, "peak_bin_agreement_vs_fp64": rec64,
        "peak_bin_agreement_refine_only": rec_refine,
        "proposal": lp.proposal, "top_network": lp.top_net,
        "alias_coverage_diagnostic": alias_hits,
        "proposal_hit_rate": {"used": hit_used, "network_top8": hit_net,
                              "coarse_power_top8": hit_heur},
        "thresholds": {"mass_min": mass_min, "power_min": power_min},
        "stages": stages, "train_loss": [hist[0], hist[-1]],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
