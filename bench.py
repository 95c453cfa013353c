#!/usr/bin/env python3
"""Throughput of the FP64 log-likelihood + exact gradient on one MI355X.

Workload (default): 4096 parameter draws of a 10-layer stack sharing one
dataset of 400 log-spaced Q points in [0.005, 0.35] 1/A with 5 % dQ/Q
resolution (17 quadrature nodes per point), seeded synthetic inputs.  One
step = one nr_loglik_grad call: per-item constants, quadrature nodes,
wavevectors, interface and phase factors, layer product, smearing,
instrument, chi^2 log-likelihood, adjoint seeds, adjoint re-walk and the
gradient reduction, for every draw.  Inputs are resident in HBM before the
timed region.

Metric unit: layer-steps/s = sum over items of nodes x (L + 1) per second.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("logL+∇ evals/s (sample×Q×layer), FP64 vs plain; % of FP64 VALU peak")
UNIT = "layer-steps/s"

# Algorithmic FP64 operations per layer-step of the forward + reverse sweep
# (operation count of the method; FMA = 2, complex multiply 6, complex add 2,
# abs^2 3; special functions at fixed costs: sqrt 10, divide or reciprocal
# 10, exp 20, sin+cos 40).  Forward: w 1, its complex root 36, the Fresnel
# coefficient 25, the Nevot-Croce factor and r' 76, the phase and its
# reciprocal 79, the state update 40.  Reverse (the adjoint of the scaled
# form): re-formed t 8, the cotangents of e, t, r', the states, r and the
# Nevot-Croce exponent 54, the sigma sum 4, kz terms through the
# Nevot-Croce exponent 16, through the Fresnel coefficient 36, their
# combination 4, the phase and thickness terms 24, the chain rule through the
# root 21.
FLOP_FWD_PER_LAYER_STEP = 257
FLOP_ADJ_PER_LAYER_STEP = 167
FLOP_PER_LAYER_STEP = FLOP_FWD_PER_LAYER_STEP + FLOP_ADJ_PER_LAYER_STEP
# Without packed FP32 instructions (the build turns them off), an FP32 FMA
# issues at the FP64 rate: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz.
VALU_FMA_PEAK = 78.6e12

# rocprofv3 counters of executed vector instructions (per wave) from which the
# executed FLOP are counted: FMA = 2, MUL, ADD and transcendental = 1, times
# the 64 lanes of a wave.
FLOP_COUNTERS = {
    "f64": ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
            "SQ_INSTS_VALU_TRANS_F64"),
    "f32": ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32",
            "SQ_INSTS_VALU_TRANS_F32"),
}


class _Hip:
    """hipEvent helpers through the HIP runtime's C API."""

    def __init__(self):
        self.L = ctypes.CDLL("libamdhip64.so")
        self.L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.L.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def event(self):
        e = ctypes.c_void_p()
        rc = self.L.hipEventCreate(ctypes.byref(e))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed: {rc}")
        return e

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        rc = self.L.hipEventElapsedTime(ctypes.byref(ms), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return float(ms.value)

    def destroy(self, e):
        self.L.hipEventDestroy(e)


KERNEL_SOURCES = ["paper_2509_06924_amd/csrc/nr_kernels.hpp",
                  "paper_2509_06924_amd/csrc/nr_kernels_f64.hip",
                  "paper_2509_06924_amd/csrc/nr_kernels_f32.hip",
                  "paper_2509_06924_amd/csrc/nr_kernels_bucket.hip",
                  "paper_2509_06924_amd/csrc/nr_kernels_scan.hip",
                  "paper_2509_06924_amd/csrc/nr_device.hpp",
                  "paper_2509_06924_amd/csrc/nr_internal.hpp",
                  "paper_2509_06924_amd/build.py"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def _profile_record(name):
    """A committed counter summary (profiles/<name>.json), or None when there
    is none or the kernel sources changed since its counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return rec


def measured_traffic(workload):
    """HBM bytes per step of the layer-product kernels from the committed
    FETCH_SIZE / WRITE_SIZE summary (calibrated on a plain copy), or None when
    there is none or the kernel sources changed since it was taken."""
    rec = _profile_record(f"traffic_{workload}")
    return None if rec is None else rec.get("traffic_bytes_per_step")


def executed_flops(workload, precision):
    """Executed vector FLOP per call of the layer-product kernels (FP64 and
    FP32 separately), from the committed rocprofv3 counter summary
    profiles/flops_<workload>_<precision>.json; None when stale or absent."""
    return _profile_record(f"flops_{workload}_{precision}")


def rate_fields(workload, precision, layer_steps, seconds):
    """Achieved rate and fraction of the vector FMA peak of one call's
    layer-product launches lasting `seconds`: from the executed FLOP counted
    by rocprofv3 when the counters match the kernel sources (FP64 + FP32
    FLOP, both issue at the 78.6 TFLOP/s FMA rate here), beside the rate of
    the 424-FLOP-per-layer-step cost model."""
    model = FLOP_PER_LAYER_STEP * layer_steps
    out = {"frac_model": model / seconds / VALU_FMA_PEAK,
           "flop_per_layer_step_model": FLOP_PER_LAYER_STEP}
    rec = executed_flops(workload, precision)
    if rec is None:
        out.update({"achieved": model / seconds / 1e12, "frac": model / seconds / VALU_FMA_PEAK,
                    "flop_source": "cost model (no counters recorded for these kernel sources)"})
        return out
    flop = rec["fp64_flop_per_call"] + rec["fp32_flop_per_call"]
    out.update({"achieved": flop / seconds / 1e12, "frac": flop / seconds / VALU_FMA_PEAK,
                "flop_per_call": flop, "fp64_flop_per_call": rec["fp64_flop_per_call"],
                "fp32_flop_per_call": rec["fp32_flop_per_call"],
                "flop_per_layer_step_executed": flop / layer_steps,
                "flop_source": f"rocprofv3 executed VALU instructions "
                               f"(profiles/flops_{workload}_{precision}.json)"})
    return out


def record_counters(csv_dir, workload, precision, command):
    """Reads the rocprofv3 --pmc output under csv_dir (one or more
    *counter_collection.csv) of a run of this script on `workload`, sums the
    FLOP counters over the layer-product launches (k_loglik_grad*) and
    divides by the calls (one k_item_consts dispatch per call); writes
    profiles/flops_<workload>_<precision>.json."""
    import csv
    import glob
    vals = {}
    consts = set()
    for path in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            if "k_item_consts" in name:
                consts.add(r["Dispatch_Id"])
            if "k_loglik_grad" in name:
                c = r["Counter_Name"]
                vals[c] = vals.get(c, 0.0) + float(r["Counter_Value"])
    if not consts:
        raise SystemExit(f"no k_item_consts dispatch found under {csv_dir}")
    calls = len(consts)

    def flop(prec):
        fma, mul, add, trans = (vals.get(c) for c in FLOP_COUNTERS[prec])
        if fma is None:
            raise SystemExit(f"counters {FLOP_COUNTERS[prec]} missing under {csv_dir}")
        return 64.0 * (2.0 * fma + mul + add + trans) / calls

    batch, _ = make_workload(workload)
    rec = {"workload": workload, "precision": precision, "calls_counted": calls,
           "kernel_sources_sha256": kernel_sources_sha256(),
           "fp64_flop_per_call": flop("f64"), "fp32_flop_per_call": flop("f32"),
           "layer_steps_per_call": batch.layer_steps(),
           "counters_per_call": {k: v / calls for k, v in sorted(vals.items())},
           "command": command}
    rec["flop_per_layer_step"] = ((rec["fp64_flop_per_call"] + rec["fp32_flop_per_call"])
                                  / rec["layer_steps_per_call"])
    out = os.path.join(ROOT, "profiles", f"flops_{workload}_{precision}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: rec[k] for k in ("workload", "precision", "calls_counted",
                                          "fp64_flop_per_call", "fp32_flop_per_call",
                                          "flop_per_layer_step")}))


def make_workload(name):
    from paper_2509_06924_amd import inputs
    if name == "c2":
        b = inputs.c2_batched()
        cfg = {"workload": "4096 draws x 10-layer stack, 400 log-Q in [0.005,0.35], "
                           "5% dQ/Q with 17-node quadrature, logL + exact gradient",
               "draws": 4096, "layers": 10, "q_points": 400, "quad_nodes": 17,
               "dq_over_q": 0.05}
    elif name == "c1":
        b = inputs.c1_single_film()
        cfg = {"workload": "1 draw x 1-layer film, 200 log-Q in [0.008,0.3], unsmeared",
               "draws": 1, "layers": 1, "q_points": 200, "quad_nodes": 1}
    elif name == "c3":
        b = inputs.c3_cofit()
        cfg = {"workload": "1024 draws x 3 contrasts x 12 layers, Q 250/300/350, 5% dQ/Q",
               "draws": 1024, "contrasts": 3, "layers": 12}
    elif name == "c4":
        b = inputs.c4_ragged()
        cfg = {"workload": "16384 ragged items, L 2..40, nQ 100..1000, dQ/Q 2-8%",
               "items": 16384}
    elif name == "c5":
        b = inputs.c5_vi()
        cfg = {"workload": "8192 VI samples x 20 layers x 1000 Q, 5% dQ/Q", "samples": 8192,
               "layers": 20}
    elif name == "deep":
        b = inputs.microsliced()
        cfg = {"workload": "64 microsliced profiles x 1000 slabs x 200 Q, 5% dQ/Q (scan gradient)",
               "items": 64, "layers": 1000, "q_points": 200}
    else:
        raise SystemExit(f"unknown workload {name}")
    return b, cfg


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, target_s=15.0):
    """The oracle (CPU, FP64, complex-step gradient) on a bounded sample of the
    same workload, all host threads (up to 16); returns layer-steps/s of
    logL + gradient, plus the forward-only logL rate on the same sample and
    the one-thread gradient rate on a smaller one."""
    import numpy as np

    import oracle
    nthreads = max(1, min(oracle.max_threads(), os.cpu_count() or 1, 16))

    def run(items, grad=True, threads=nthreads):
        sub = batch.subset(items)
        t0 = time.perf_counter()
        oracle.loglik_grad_batch(sub.q_off, sub.Q, sub.Robs, sub.Rerr, sub.dq_over_q,
                                 sub.dataset_of_item, sub.row_off, sub.layers, sub.scale,
                                 sub.bkg, want_grad=grad, nthreads=threads)
        return time.perf_counter() - t0, sub.layer_steps()

    t1, _ = run(np.arange(min(nthreads, batch.n_items)))
    per_round = max(t1, 1e-3)
    rounds = max(1, int(target_s / per_round))
    n = min(batch.n_items, rounds * nthreads)
    t, ls = run(np.arange(n))
    tf, lsf = run(np.arange(n), grad=False)
    n1 = max(1, min(batch.n_items, int(0.2 * target_s / per_round)))
    t_1, ls_1 = run(np.arange(n1), threads=1)
    return {"value": ls / t, "unit": UNIT, "cores": nthreads, "kind": "oracle",
            "sample": f"first {n} items of the workload ({ls:.3e} layer-steps, {t:.1f} s, "
                      f"complex-step gradient, OpenMP over items)",
            "forward_only_value": lsf / tf,
            "one_thread_value": ls_1 / t_1,
            "one_thread_sample": f"first {n1} items, {t_1:.1f} s",
            "host": {"cpu": _cpu_model(), "nproc": os.cpu_count()},
            "note": "the complex-step gradient costs about 4x a forward evaluation per "
                    "parameter: a correctness referee, not a tuned CPU gradient"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "deep"],
                    help="c2 (default): the 4096-draw batch the metric is quoted on; the others "
                         "time the single-film, co-fit, ragged, VI and deep-stack batches")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-rows", action="store_true",
                    help="skip the forward-only and per-item (unbatched) rows")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the single-film, co-fit, ragged-HMC and VI rows")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default schedule instead of the autotuned one")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON cache of autotuned schedules (default: the user cache)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe-mib", type=float, default=0.0,
                    help="only run a plain device copy of this size (counter calibration)")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"],
                    help="arithmetic of the timed calls (f64, the default, is the headline; "
                         "f32 serves counter collection of the FP32 variant)")
    ap.add_argument("--record-counters", default=None, metavar="DIR",
                    help="no GPU work: read the rocprofv3 --pmc output under DIR of a run of "
                         "this script on --workload / --precision and write "
                         "profiles/flops_<workload>_<precision>.json")
    ap.add_argument("--counter-command", default="",
                    help="with --record-counters: the command that produced DIR (stored)")
    args = ap.parse_args()

    if args.record_counters:
        record_counters(args.record_counters, args.workload, args.precision,
                        args.counter_command)
        return

    if args.copy_probe_mib > 0:
        import torch
        n = int(args.copy_probe_mib * 2**20 / 8)
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}))
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(items shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2509_06924_amd as nr
    from paper_2509_06924_amd import _native

    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    batch, cfg = make_workload(args.workload)
    prec = nr.NR_F32 if args.precision == "f32" else nr.NR_F64
    schedule = None
    if not args.no_autotune:
        from paper_2509_06924_amd import autotune
        schedule = autotune.tune(batch, precision=prec, device="cuda:0",
                                 cache=args.autotune_cache)
    prob = nr.Problem.from_batch(batch, device="cuda:0", precision=prec, options=schedule)
    hip = _Hip()
    t = time_gradient(nr, prob, args.steps, args.warmup, hip)
    out = t["out"]
    layer_steps = batch.layer_steps()
    wall, kern_s = t["wall_s"], t["kernel_s"]
    ms_per_step = wall / args.steps * 1e3
    value = layer_steps * args.steps / wall
    ok = bool(torch.isfinite(out[0]).all().item() and torch.isfinite(out[1]).all().item())

    roof = rate_fields(args.workload, args.precision, layer_steps, kern_s)
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded stand-in; the paper's datasets are not available)",
        "config": cfg,
        "schedule": schedule or "library default",
        "layer_steps_per_step": layer_steps,
        "draw_q_per_s": batch.data_points() * args.steps / wall,
        "finite": ok,
        "roofline": {
            "bound": "alu",
            "achieved": roof["achieved"],
            "peak": VALU_FMA_PEAK / 1e12,
            "unit": "TFLOP/s",
            "frac": roof["frac"],
            "traffic": measured_traffic(args.workload) if args.precision == "f64" else None,
            "kernel": "k_loglik_grad (layer product, smearing, logL and adjoint)",
            "kernel_ms": kern_s * 1e3,
            **{k: v for k, v in roof.items() if k not in ("achieved", "frac")},
        },
    }
    if args.workload == "c2" and args.precision == "f64" and not args.no_other_workloads:
        rec["co_headline"] = ragged_row(nr, hip, max(3, min(args.steps, 10)))
    if not args.no_extra_rows and args.precision == "f64":
        rec["forward_only"] = forward_only_row(prob, batch, args.steps)
        rec["plain_unbatched"] = plain_unbatched_row(nr, batch)
        rec["fp32"] = fp32_row(nr, batch, args.workload, out, args.steps, hip,
                               None if args.no_autotune else args.autotune_cache or "")
    if not args.no_extra_rows and args.workload == "c2" and not args.no_other_workloads:
        rec["other_workloads"] = other_workloads(nr)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(batch, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


def time_gradient(nr, prob, steps, warmup, hip):
    """Times `steps` nr_loglik_grad calls after `warmup` untimed ones: wall
    time of the whole calls (bracketed by device synchronisations) and the
    average duration of their layer-product launches (HIP events the library
    records on the launch stream around them)."""
    import torch

    from paper_2509_06924_amd import _native
    n = prob.plan.n_items
    out = (torch.empty(n, dtype=torch.float64, device=prob.device), torch.empty_like(prob.layers),
           torch.empty(n, 2, dtype=torch.float64, device=prob.device))
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        prob.loglik_grad(out=out, stream=stream)
    torch.cuda.synchronize()
    evs = [(hip.event(), hip.event()) for _ in range(steps)]
    L = _native.lib()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        _native.check(L.nr_plan_set_timing_events(prob.plan.handle, evs[k][0], evs[k][1]))
        prob.loglik_grad(out=out, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _native.check(L.nr_plan_set_timing_events(prob.plan.handle, None, None))
    kern_ms = [hip.elapsed_ms(a, b) for a, b in evs]
    for a, b in evs:
        hip.destroy(a)
        hip.destroy(b)
    return {"out": out, "wall_s": t1 - t0, "kernel_s": sum(kern_ms) / len(kern_ms) / 1e3}


def ragged_row(nr, hip, steps):
    """The largest single-GPU workload beside the headline: 16384 ragged items
    (L 2..40, nQ 100..1000, dQ/Q 2-8 %), one nr_loglik_grad call per step in
    the library's default schedule, timed like the headline, with its own
    executed-FLOP fraction of the FP64 peak."""
    from paper_2509_06924_amd import inputs
    batch = inputs.c4_ragged()
    prob = nr.Problem.from_batch(batch, device="cuda:0")
    t = time_gradient(nr, prob, steps, 2, hip)
    ls = batch.layer_steps()
    roof = rate_fields("c4", "f64", ls, t["kernel_s"])
    prob.plan.close()
    return {"workload": "16384 ragged items, L 2..40, nQ 100..1000, dQ/Q 2-8%, logL + exact "
                        "gradient (FP64), library default schedule",
            "value": ls * steps / t["wall_s"], "unit": UNIT, "steps": steps,
            "ms_per_step": t["wall_s"] / steps * 1e3, "layer_steps_per_step": ls,
            "roofline": {"bound": "alu", "achieved": roof["achieved"],
                         "peak": VALU_FMA_PEAK / 1e12, "unit": "TFLOP/s", "frac": roof["frac"],
                         "kernel_ms": t["kernel_s"] * 1e3,
                         **{k: v for k, v in roof.items() if k not in ("achieved", "frac")}}}


def forward_only_row(prob, batch, steps):
    """The same workload through nr_loglik (value only, no adjoint)."""
    import torch
    for _ in range(2):
        prob.loglik()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.loglik()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"value": batch.layer_steps() / dt, "unit": UNIT, "ms_per_step": dt * 1e3,
            "what": "nr_loglik on the same batch (forward only)"}


def fp32_row(nr, batch, workload, out64, steps, hip, tune_cache=None):
    """The FP32 variant on the same workload: time, rate, fraction of the FP32
    VALU peak, and its largest deviation from the FP64 path (which matches the
    oracle to 1e-10 / 1e-8), over every item.  tune_cache None: library
    default schedule; else autotuned ("" = the user cache)."""
    import numpy as np
    import torch

    from paper_2509_06924_amd import _native
    schedule = None
    if tune_cache is not None:
        from paper_2509_06924_amd import autotune
        schedule = autotune.tune(batch, precision=nr.NR_F32, device="cuda:0",
                                 cache=tune_cache or None)
    prob = nr.Problem.from_batch(batch, device="cuda:0", precision=nr.NR_F32, options=schedule)
    out = (torch.empty_like(out64[0]), torch.empty_like(out64[1]), torch.empty_like(out64[2]))
    stream = torch.cuda.current_stream()
    for _ in range(2):
        prob.loglik_grad(out=out, stream=stream)
    torch.cuda.synchronize()
    L = _native.lib()
    evs = [(hip.event(), hip.event()) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        _native.check(L.nr_plan_set_timing_events(prob.plan.handle, evs[k][0], evs[k][1]))
        prob.loglik_grad(out=out, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    _native.check(L.nr_plan_set_timing_events(prob.plan.handle, None, None))
    kern_s = sum(hip.elapsed_ms(a, b) for a, b in evs) / len(evs) / 1e3
    for a, b in evs:
        hip.destroy(a)
        hip.destroy(b)
    ll32, ll64 = out[0].cpu().numpy(), out64[0].cpu().numpy()
    units = np.array([1.0, 1e-6, 1e-6, 1.0])
    g32 = out[1].cpu().numpy() * units
    g64 = out64[1].cpu().numpy() * units
    i32 = out[2].cpu().numpy() * np.array([1.0, 1e-7])
    i64 = out64[2].cpu().numpy() * np.array([1.0, 1e-7])
    gerr = 0.0
    for b in range(batch.n_items):
        r0, r1 = batch.row_off[b], batch.row_off[b + 1]
        a = np.concatenate([g32[r0:r1].ravel(), i32[b]])
        o = np.concatenate([g64[r0:r1].ravel(), i64[b]])
        gerr = max(gerr, float(np.max(np.abs(a - o)) / np.max(np.abs(o))))
    roof = rate_fields(workload, "f32", batch.layer_steps(), kern_s)
    return {"value": batch.layer_steps() / dt, "unit": UNIT, "ms_per_step": dt * 1e3,
            "kernel_ms": kern_s * 1e3, "dtype": "f32", "schedule": schedule or "library default",
            "achieved_tflops": roof["achieved"], "peak_tflops": VALU_FMA_PEAK / 1e12,
            "frac": roof["frac"],
            "peak_note": "FP32 and FP64 vector FMAs both issue at 78.6 TFLOP/s without packed "
                         "FP32 instructions, which the build turns off (157.3 needs them)",
            **{k: v for k, v in roof.items() if k not in ("achieved", "frac")},
            "max_rel_err_logL": float(np.max(np.abs(ll32 - ll64) / np.abs(ll64))),
            "max_rel_err_grad": gerr,
            "what": "nr_loglik_grad with NR_F32 (layer product and adjoint in float; "
                    "kz0^2 - 4 pi drho, smearing, chi^2 and accumulation in FP64); errors "
                    "against the FP64 path over every item, gradient in natural units "
                    "relative to each item's largest component"}


NATURAL_UNITS = (1.0, 1e-6, 1e-6, 1.0)  # d, rho_re, rho_im, sigma


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def single_film_row(nr):
    """One draw of the 1-layer film, 200 points, unsmeared: latency of one
    logL + gradient call (back to back; with a host sync per call; and as a
    replayed graph)."""
    import torch

    from paper_2509_06924_amd import inputs
    batch = inputs.c1_single_film()
    prob = nr.Problem.from_batch(batch, device="cuda:0")
    out = prob.loglik_grad()
    stream = torch.cuda.current_stream()
    back = _timed(lambda: prob.loglik_grad(out=out, stream=stream), 500)

    def synced():
        prob.loglik_grad(out=out, stream=stream)
        torch.cuda.synchronize()
    sync = _timed(synced, 200)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        prob.loglik_grad(out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        prob.loglik_grad(out=out)
    graph = _timed(g.replay, 500)
    return {"what": "1 draw x 1-layer film x 200 Q, unsmeared, logL + gradient",
            "us_per_call_back_to_back": back * 1e6, "us_per_call_synced": sync * 1e6,
            "us_per_call_graph_replay": graph * 1e6,
            "layer_steps_per_call": batch.layer_steps()}


def cofit_row(nr, reps=10):
    """1024 draws x 3 contrasts x 12 layers: logL + gradient per item, then the
    tie-sum of the per-contrast gradients onto the 50 shared parameters."""
    import numpy as np
    import torch

    from paper_2509_06924_amd import inputs
    batch = inputs.c3_cofit()
    prob = nr.Problem.from_batch(batch, device="cuda:0")
    rows = int(batch.row_off[1] - batch.row_off[0])
    # the shared parameters of a draw: the 12 layers' d, rho_re, rho_im,
    # sigma, the backing roughness and the background (50); the fronting, the
    # backing SLDs (the contrasts) and the scale are fixed
    per_draw = (rows - 2) * 4 + 2
    nre = batch.layers.size
    tie = -np.ones(nre + 2 * batch.n_items, np.int64)
    for b in range(batch.n_items):
        d = b // 3
        k = 0
        for r in range(1, rows - 1):
            for f in range(4):
                tie[(batch.row_off[b] + r) * 4 + f] = d * per_draw + k
                k += 1
        tie[(batch.row_off[b] + rows - 1) * 4 + 3] = d * per_draw + k
        tie[nre + 2 * b + 1] = d * per_draw + k + 1
    first, src = nr.tie_map_to_csr(tie, (batch.n_items // 3) * per_draw)
    first_t = torch.as_tensor(first, device="cuda:0")
    src_t = torch.as_tensor(src, device="cuda:0")
    out = prob.loglik_grad()
    stream = torch.cuda.current_stream()

    def step():
        prob.loglik_grad(out=out, stream=stream)
        nr.tie_sum(first_t, src_t, torch.cat([out[1].reshape(-1), out[2].reshape(-1)]))
    dt = _timed(step, reps)
    return {"what": "1024 draws x 3 contrasts x 12 layers, Q 250/300/350, 5% dQ/Q: "
                    "logL + gradient + tie-sum onto the shared parameters",
            "ms_per_step": dt * 1e3, "value": batch.layer_steps() / dt, "unit": UNIT,
            "shared_params_per_draw": per_draw}


def ragged_hmc_row(nr, precision, n_steps=10):
    """16384 ragged items (L 2..40, nQ 100..1000, dQ/Q 2-8%): n leapfrog steps
    (half kick, drift, logL + gradient, half kick) captured in one HIP graph,
    dt = 1e-3 in natural units (inverse mass = unit^2)."""
    import numpy as np

    from paper_2509_06924_amd import inputs
    batch = inputs.c4_ragged()
    prob = nr.Problem.from_batch(batch, device="cuda:0", precision=precision)
    rng = np.random.default_rng(7)
    units = np.array(NATURAL_UNITS)
    mom_rows = rng.standard_normal(batch.layers.shape) / units
    mom_inst = rng.standard_normal((batch.n_items, 2)) / np.array([1.0, 1e-7])
    im_rows = np.tile(units ** 2, (batch.layers.shape[0], 1))
    im_inst = np.tile(np.array([1.0, 1e-14]), (batch.n_items, 1))
    st = nr.HmcState(prob, mom_rows, mom_inst, im_rows, im_inst)
    graph = nr.LeapfrogGraph(prob, st, 1e-3, n_steps)
    dt = _timed(graph.launch, 3) / n_steps
    graph.close()
    return {"what": "16384 ragged items, L 2..40, nQ 100..1000, dQ/Q 2-8%: HIP-graph leapfrog "
                    f"({n_steps} steps per graph)",
            "dtype": "f32" if precision == nr.NR_F32 else "f64",
            "ms_per_leapfrog_step": dt * 1e3, "value": batch.layer_steps() / dt, "unit": UNIT,
            "layer_steps_per_step": batch.layer_steps(),
            "rate_per_step": rate_fields("c4", "f32" if precision == nr.NR_F32 else "f64",
                                         batch.layer_steps(), dt)}


def hmc_driver_row(nr, n_leapfrog=4):
    """16384 ragged chains (the leapfrog workload above): whole HMC transitions
    of the driver (momentum draws, n leapfrog steps in pre-scaled coordinates,
    Metropolis-Hastings accept) captured in one HIP graph."""
    import numpy as np

    from paper_2509_06924_amd import inputs
    batch = inputs.c4_ragged()
    prob = nr.Problem.from_batch(batch, device="cuda:0")
    R = batch.layers.shape[0]
    # pre-scaled coordinates: z in natural units (d, sigma 1 A; rho 1e-6; bkg 1e-7)
    b_rows = np.tile(np.array(NATURAL_UNITS), (R, 1))
    b_inst = np.tile(np.array([1.0, 1e-7]), (batch.n_items, 1))
    h = nr.HMC(prob, b_rows=b_rows, b_inst=b_inst, step=2e-5, n_leapfrog=n_leapfrog,
               seed=2509).init(from_theta=True)
    graph = h.graph(n_transitions=1)
    dt = _timed(graph.launch, 3)
    graph.close()
    n_acc = int(h.n_accept.sum().item())
    n_tr = int(h.n_accept.numel()) * 4  # the warm-up launch plus three timed ones
    out = {"what": f"16384 ragged chains, L 2..40, nQ 100..1000, dQ/Q 2-8%: HIP-graph HMC "
                   f"transition ({n_leapfrog} leapfrog steps, Philox momenta, MH accept)",
           "ms_per_transition": dt * 1e3,
           "value": n_leapfrog * batch.layer_steps() / dt, "unit": UNIT,
           "accept_rate": n_acc / n_tr,
           "divergent": int(h.n_divergent.sum().item())}
    h.close()
    return out


def deep_stack_row(nr, reps=3):
    """64 microsliced profiles x 1000 slabs x 200 Q, 5% dQ/Q: logL + gradient
    through the parallel-in-layers scan (two waves per data point at this
    depth), and the forward-only value kernel on the same batch."""
    import torch

    from paper_2509_06924_amd import inputs
    batch = inputs.microsliced()
    prob = nr.Problem.from_batch(batch, device="cuda:0")
    out = prob.loglik_grad()
    stream = torch.cuda.current_stream()
    dt = _timed(lambda: prob.loglik_grad(out=out, stream=stream), reps)
    dtf = _timed(lambda: prob.loglik(stream=stream), reps)
    ls = batch.layer_steps()
    return {"what": "64 microsliced profiles x 1000 slabs x 200 Q, 5% dQ/Q: parallel-in-layers "
                    "scan gradient (FP64), two waves per data point",
            "ms_per_step": dt * 1e3, "value": ls / dt, "unit": UNIT,
            "rate_per_step": rate_fields("deep", "f64", ls, dt),
            "forward_only_ms": dtf * 1e3, "layer_steps_per_step": ls}


def resolution_row(nr, reps=10):
    """The 4096-draw batch through nr_loglik_grad_res (the gradient plus
    dlogL/d(dQ/Q) per draw, from dR/dq at every smearing node) beside the
    plain gradient call on the same plan."""
    import torch

    from paper_2509_06924_amd import inputs
    batch = inputs.c2_batched()
    prob = nr.Problem.from_batch(batch, device="cuda:0")
    out = prob.loglik_grad()
    stream = torch.cuda.current_stream()
    dt_res = _timed(lambda: prob.loglik_grad_res(stream=stream), reps)
    dt = _timed(lambda: prob.loglik_grad(out=out, stream=stream), reps)
    ls = batch.layer_steps()
    return {"what": "4096 draws x 10 layers x 400 Q, 5% dQ/Q: logL + gradient + dlogL/d(dQ/Q) "
                    "(nr_loglik_grad_res) beside logL + gradient (nr_loglik_grad), same plan",
            "ms_per_step": dt_res * 1e3, "value": ls / dt_res, "unit": UNIT,
            "frac_model": FLOP_PER_LAYER_STEP * ls / dt_res / VALU_FMA_PEAK,
            "plain_gradient_ms": dt * 1e3}


def vi_mvn_row(nr, reps=5):
    """The full-rank Gaussian VI of the paper's co-fit study: 100 restarts x
    8 draws of a 12-layer stack over 300 Q, 5% dQ/Q, one Adam step each."""
    import numpy as np

    from paper_2509_06924_amd import inputs
    R, S, L = 100, 8, 12
    rng = np.random.default_rng(13)
    template = inputs.draw_stack(rng, L, d=(20.0, 80.0), rho=(0.5e-6, 4.5e-6),
                                 sigma=(2.0, 10.0))
    Q = inputs.log_grid(0.005, 0.3, 300)
    Robs, err = inputs.synthetic_curve(Q, rng)
    batch = inputs._pack("mvn", [(Q, Robs, err, 0.05)], [(0, template, 1.0, 1e-7)] * (R * S),
                         {})
    prob = nr.Problem.from_batch(batch, device="cuda:0")
    nrow = L + 2
    P = 4 * nrow + 2
    kind = np.zeros(P, np.uint8)
    a = np.zeros(P)
    b = np.ones(P)
    for r in range(1, nrow):
        kind[4 * r + 1], b[4 * r + 1] = nr.NR_TF_AFFINE, 1e-6
        kind[4 * r + 3], b[4 * r + 3] = nr.NR_TF_LOGIT, 30.0
        if r < nrow - 1:
            kind[4 * r] = nr.NR_TF_LOG
    kind[P - 2], a[P - 2], b[P - 2] = nr.NR_TF_AFFINE, 1.0, 0.01
    kind[P - 1], b[P - 1] = nr.NR_TF_LOG, 1e-7
    theta = np.concatenate([template.ravel(), [1.0, 1e-7]])
    mu = np.zeros(P)
    for p in np.flatnonzero(kind):
        t = theta[p]
        mu[p] = {nr.NR_TF_AFFINE: lambda: (t - a[p]) / b[p],
                 nr.NR_TF_LOG: lambda: np.log((t - a[p]) / b[p]),
                 nr.NR_TF_LOGIT: lambda: np.log((t - a[p]) / (b[p] - t))}[int(kind[p])]()
    vi = nr.MvnVI(prob, R, S, kind, a, b, theta, mu=np.tile(mu, (R, 1)), sigma0=0.1, lr=0.05,
                  seed=2509)
    graph = vi.graph(n_steps=10)
    dt = _timed(graph.launch, reps) / 10
    graph.close()
    vi.close()
    return {"what": f"{R} restarts x {S} draws, {L} layers x 300 Q, 5% dQ/Q: full-rank Gaussian "
                    "VI, one Adam step (draws, logL + gradient, ELBO gradient, Adam), HIP graph",
            "ms_per_step": dt * 1e3, "value": batch.layer_steps() / dt, "unit": UNIT}


def vi_row(nr, reps=5):
    """8192 mean-field VI samples x 20 layers x 1000 Q, 5% dQ/Q: sampler,
    logL + gradient per sample, and the ELBO gradient reduction."""
    import numpy as np

    from paper_2509_06924_amd import inputs
    batch = inputs.c5_vi()
    mu_rows = batch.meta["mu"]
    L = mu_rows.shape[0] - 2
    P = mu_rows.size + 2
    mu = np.concatenate([mu_rows.reshape(-1), [1.0, 1e-7]])
    mask = np.zeros(P, np.uint8)
    mask[4:4 * (mu_rows.shape[0] - 1)] = 1  # the finite layers' 4 entries
    mask[-2:] = 1
    width = np.maximum(batch.meta["rel_width"] * np.abs(mu), 1e-12)
    omega = np.log(np.expm1(width))
    eps = np.random.default_rng(11).standard_normal((batch.n_items, P))
    import torch
    dev = dict(device="cuda:0")
    mu, omega, eps = (torch.as_tensor(x, dtype=torch.float64, **dev) for x in (mu, omega, eps))
    mask = torch.as_tensor(mask, **dev)
    out = {}
    for prec in (nr.NR_F64, nr.NR_F32):
        prob = nr.Problem.from_batch(batch, device="cuda:0", precision=prec)
        dt = _timed(lambda: prob.vi_elbo_grad(mu, omega, mask, eps), reps)
        out["f32" if prec == nr.NR_F32 else "f64"] = {
            "ms_per_step": dt * 1e3, "value": batch.layer_steps() / dt, "unit": UNIT}
    out["what"] = (f"8192 samples x {L} layers x 1000 Q, 5% dQ/Q: sampler + logL + gradient + "
                   "ELBO gradient, inputs resident on the device")
    return out


def other_workloads(nr):
    return {"single_film": single_film_row(nr), "cofit": cofit_row(nr),
            "ragged_hmc_f64": ragged_hmc_row(nr, nr.NR_F64),
            "ragged_hmc_f32": ragged_hmc_row(nr, nr.NR_F32), "hmc_driver": hmc_driver_row(nr),
            "vi": vi_row(nr), "vi_mvn": vi_mvn_row(nr), "deep_stack": deep_stack_row(nr),
            "resolution_grad": resolution_row(nr)}


def plain_unbatched_row(nr, batch, n_items=64):
    """The same kernels launched once per item (batch of 1), host loop, no
    graph: what a per-evaluation call pattern gets on this GPU."""
    import numpy as np
    import torch
    items = np.arange(min(n_items, batch.n_items))
    probs = [nr.Problem.from_batch(batch.subset([int(b)]), device="cuda:0") for b in items]
    for p in probs:
        p.loglik_grad()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in probs:
        p.loglik_grad()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ls = batch.subset(items).layer_steps()
    return {"value": ls / dt, "unit": UNIT, "items": int(items.size),
            "ms_per_item": dt / items.size * 1e3,
            "what": "nr_loglik_grad per item, batch of 1, host loop"}


if __name__ == "__main__":
    main()
