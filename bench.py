#!/usr/bin/env python3
"""Benchmark of the normal-deviate hot path on one MI355X.

One step = the batched workload (4096 streams, lengths log-uniform on
[1e2, 1e6], per-stream mu, sigma and seed; about 4.45e8 normals per method)
turned into FP32 normals by Box-Muller (Algorithm B1) AND by the Polar method
(Algorithm P), through the C ABI: for each, one tile-table set-up kernel,
then B1's persistent kernel, or Polar's mask, chunk-scan and generate
kernels.  The printed `value` is the whole step's throughput in normals per
second (both methods' normals over the step time), with every input resident
in GPU memory before timing starts.  One kernel is timed inside the timed
steps, by the two events of its own dispatch: the dominant one (the longest
main kernel of the warm-up steps); a breakdown pass after the timed steps
times the other legs.

Alongside, outside the timed region: the measured store-only ceiling (best
of a sweep over plain and nontemporal stores and launch shapes), the
hash-only ceiling, the single-stream fills of 2^30 normals (FP32, BF16, FP16 and the
plain FP64 kernels, the comparison point of the FP32 batched figure), the
graph-replayed repeated fill (64 x 2^28 Polar normals), methods P2 (Section
4), B3 and B2 (Section 3) and Algorithm R (Section 5) on the same batched
workload, and the CPU oracle timed on the host cores.

The default 50 warm-up steps (about 60 ms of load) bring the GPU to its
loaded state: with 3 the timed steps ran about 5% slower, and the step time
levels off from about 20 warm-up steps on.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
                       [--no-cpu] [--only b1|polar|p2|b3|ratio|b2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "normals/s and % HBM write peak, FP32 batched vs plain FP64 (B1, Polar)"
HBM_PEAK_GBS = 8000.0          # MI355X datasheet HBM3E bandwidth
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 lane
# operations/s (the published 157.3 TFLOP/s FP32 vector figure counts an FMA
# as 2 flops on 2 packed values: 157.3 / 4)
VALU_PEAK_TOPS = 39.32
# Algorithmic VALU lane operations per unit of work of each kernel: the
# 32-bit VALU operations of the method's own arithmetic, counted step by
# step in its cheapest form here.  A SplitMix64 hash of a counter inside a
# tile whose counters share the high word of z = c + gamma costs 15 (top
# word: counter add 1, first round on the low word 2, first product 3,
# second round's 64-bit shift and two xors 3, top word of the second product
# 4, final shift and xor 2) or 17 (full hash: the whole second product 4 and
# the final 64-bit xor-shift 4).  Of two consecutive counters whose z are
# even and odd, the odd one's first product is the even one's plus or minus
# the multiplier, one 64-bit add in place of its counter add, first round
# and first product (6): it costs 10 (top word) or 12 (full).  A stream's
# counters go in such pairs, so a candidate or pair of two counters takes one
# of each, and B3's three counters per pair take 1.5 of the cheaper kind.  A
# kernel's re-computation of work another kernel already did (the generate
# kernels' second hash of each accepted candidate) is not the method's work:
# it is listed in IMPL_OVERHEAD_PAIRED and IMPL_OVERHEAD_UNPAIRED.
#   polar_count:    per candidate: top words of the hashes of X 13 and Y 8,
#                   each without the final xor-shift (2; it moves only bit 0,
#                   so S' from these words is within 2^33 of S) + S' - 1 =
#                   X'^2 + (Y'^2 - 1) by two multiply-adds 2 + the unsigned test
#                   1 + the test for S' within 2^34 of 2^62 (64-bit add and
#                   compare) 2; the exact test for such a wave (about one in
#                   10^6 waves) 0
#   polar_generate: per pair: the FP32 radius with the exact complement near
#                   s = 1 (complement and select 5, conversion 4, remainder
#                   and selects 7, log and reciprocal square root 2,
#                   scalings 4) 22 + 2 conversions and 2 FMAs 4
#   b1_batched:     per pair: full hash of u 17 + top-word hash of v 10 +
#                   ln(1 - u) with the exact complement 21 + angle reduction,
#                   conversion, sin, cos 9 + 2 FMAs
#   p2_count:       per candidate: as polar_count, the one-sided test S' < 2^62
#   p2_generate:    per pair: s from the top word 1 + v = (6s - 4)/(4 - 3s) 4 +
#                   degree-9 Horner 9 + split test and select 2 + the library
#                   branch for s > 8/9 (10 operations, taken by 1/9 of the
#                   pairs) 1 + scaling 1 + 2 conversions and 2 FMAs 4
#   b3_batched:     per pair: full hashes of u1 and u2 and the top word of u3
#                   (17 + 17 + 15, less 5 for each of the 1.5 odd counters of
#                   a pair) 41.5 + m = max 3 + conversion 3 + u = m^2 1 + v 4 +
#                   degree-9 Horner 9 + scaling 2 + the library branch's 9
#                   operations for the 1/9 of pairs above 8/9 1 + split test and
#                   select 2 + angle reduction, conversion, sin, cos 8 + 2 FMAs
#   ratio_count:    per candidate: 2 full hashes 17 + 12 + v - 1/2 and 1 - u as
#                   integers 4 + their conversions (signed split 5, unsigned
#                   3) 8 + x = c dv / du 3 + x^2 1 + -4 ln(1 - u) (scale, log,
#                   scale) 3 + the comparison 1 + the FP32 screening band
#                   (difference, sum, FMA, compare) 4; the FP64 test inside
#                   the band (under 1e-4 of candidates) 0
#   ratio_generate: per output: the integer differences 4 + conversions 8 +
#                   x 3 + 1 FMA
#   b2_batched:     per pair: full hash of u 17 + top-word hash of v 10 +
#                   ln(1 - u) with the exact complement 21 + quarter-turn
#                   reduction, conversion and scaling of y 6 + t = y^2 and
#                   the two polynomials (6 FMAs, 1 product) 8 + four
#                   doublings (d = 2s, s' = d c, c' = 1 - d s) 12 + 2 FMAs
ALU_OPS = {"polar_count": 26, "polar_generate": 26, "b1_batched": 59, "p2_count": 26, "p2_generate": 22,
           "b3_batched": 76.5, "ratio_count": 53, "ratio_generate": 16, "b2_batched": 76}
# What the generate kernels compute again per unit, beyond the method's own
# work: the two hashes of the accepted candidate and S (P, P2), or the two
# full hashes (R).  The kernel forms the second hash from the first's
# product when the candidate's counters are an even-odd pair (a stream whose
# z = c + gamma starts even: 15 + 10 + 2 for P and P2, 17 + 12 for R) and in
# full otherwise (15 + 15 + 2, 17 + 17); recomputed_ops() weighs the two by
# the workload's share of pairs in each kind of stream.
IMPL_OVERHEAD_PAIRED = {"polar_generate": 27, "p2_generate": 27, "ratio_generate": 29}
IMPL_OVERHEAD_UNPAIRED = {"polar_generate": 32, "p2_generate": 32, "ratio_generate": 34}
# The same counts by instruction class, for weighting by the measured issue
# cost of each class (extras "valu_issue_cost"): 32-bit multiplies and
# 32 x 32 -> 64-bit multiply-adds (5 in a hash, 3 in the odd counter's),
# 64-bit shifts (1 in a hash), 64-bit adds (the odd counter's product, the
# counter conversion of B1's radius), transcendentals (log, sqrt, rcp, rsq,
# sin, cos), and the rest (FMA-like, cost 1).
ALU_MIX = {
    "polar_count": {"mul": 10, "shr64": 2, "add64": 2, "trans": 0, "other": 12},
    "polar_generate": {"mul": 0, "shr64": 0, "add64": 1, "trans": 2, "other": 23},
    "b1_batched": {"mul": 8, "shr64": 2, "add64": 2, "trans": 4, "other": 43},
    "p2_count": {"mul": 10, "shr64": 2, "add64": 2, "trans": 0, "other": 12},
    "p2_generate": {"mul": 0, "shr64": 0, "add64": 0, "trans": 1, "other": 21},
    "b3_batched": {"mul": 12, "shr64": 3, "add64": 1.5, "trans": 3, "other": 57},
    "ratio_count": {"mul": 8, "shr64": 2, "add64": 1, "trans": 2, "other": 40},
    "ratio_generate": {"mul": 0, "shr64": 0, "add64": 0, "trans": 1, "other": 15},
    "b2_batched": {"mul": 8, "shr64": 2, "add64": 2, "trans": 2, "other": 62},
}
ALU_UNIT = {"polar_count": "candidate", "polar_generate": "output pair", "b1_batched": "output pair",
            "p2_count": "candidate", "p2_generate": "output pair", "b3_batched": "output pair",
            "ratio_count": "candidate", "ratio_generate": "output", "b2_batched": "output pair"}
KERNEL_NAMES = {"polar_count": "polar_mask_kernel<MODE_BATCHED> + polar_scan_kernel",
                "polar_generate": "polar_gen_kernel<float, MODE_BATCHED>",
                "b1_batched": "b1_batched_kernel<float>",
                "p2_count": "polar_mask_kernel<MODE_BATCHED, VM_P2> + polar_scan_kernel",
                "p2_generate": "polar_gen_kernel<float, MODE_BATCHED, VM_P2>",
                "b3_batched": "b1_batched_kernel<float, BM_B3>",
                "ratio_count": "polar_mask_kernel<MODE_BATCHED, VM_R> + polar_scan_kernel",
                "ratio_generate": "polar_gen_kernel<float, MODE_BATCHED, VM_R>",
                "b2_batched": "b1_batched_kernel<float, BM_B2>"}
PROFILES = os.path.join(ROOT, "profiles")


def u64sum(t) -> int:
    return int(t.cpu().numpy().view("uint64").sum(dtype="uint64"))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("nrng_kernels.hpp", "nrng_kernels_p.hip", "nrng_kernels_p2.hip", "nrng_kernels_r.hip",
              "nrng_kernels_b1.hip", "nrng_kernels_b3.hip", "nrng_kernels_b2.hip", "nrng_kernels_misc.hip",
              "nrng_device.hpp", "nrng_p2_poly.hpp", "nrng_b2_poly.hpp",
              "nrng_abi.cpp"):   # the compiled launch defaults pick the variant profiled
        with open(os.path.join(ROOT, "paper_1004_3105_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel, if it was taken on the current kernel source."""
    path = os.path.join(PROFILES, "traffic_%s.txt" % kernel_tag)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_profile_avg(kernel_tag: str):
    """The average duration (ms) of this kernel in the committed rocprofv3
    kernel-trace summary, if it was taken on the current kernel source."""
    path = os.path.join(PROFILES, "avg_%s.txt" % kernel_tag)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["avg_ms"])
    except (KeyError, ValueError):
        return None


def paired_share(cfg) -> float:
    """Share of the workload's outputs in streams whose first z = seed +
    offset + gamma is even (their candidates' two counters are an even-odd
    pair)."""
    import numpy as np
    n = cfg["n"].astype(np.float64)
    z0 = cfg["seed"].astype(np.uint64) + cfg["offset"].astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    even = (z0 & np.uint64(1)) == 0
    return float(n[even].sum() / max(n.sum(), 1.0))


def recomputed_ops(kernel: str, share: float) -> float:
    """Operations per unit the generate kernel computes again (IMPL_OVERHEAD_*),
    weighed by the share of the workload in paired streams."""
    return round(share * IMPL_OVERHEAD_PAIRED[kernel] + (1 - share) * IMPL_OVERHEAD_UNPAIRED[kernel], 2)


def median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--nstreams", type=int, default=4096)
    ap.add_argument("--no-extras", action="store_true", help="skip the side measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", choices=["b1", "polar", "p2", "b3", "ratio", "b2"], default=None,
                    help="time one method only (for profiling runs; p2, b3, ratio and b2 = method P2 of "
                         "Section 4, methods B3 and B2 of Section 3 and Algorithm R of Section 5, which are "
                         "otherwise measured among the extras)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a 1 GiB copy and a 1 GiB store probe once (known traffic, for scaling "
                         "hardware byte counters in profiling runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_1004_3105_amd import binding as nb

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nb.nrng_init()
    stream = torch.cuda.current_stream()

    # ---------------------------------------------------------------- workload
    cfg = synth.batched_streams(nstreams=args.nstreams)
    ns = len(cfg["n"])
    total = cfg["total"]
    D = {
        "seed": torch.from_numpy(cfg["seed"].view(np.int64)).to(dev),
        "offset": torch.from_numpy(cfg["offset"].view(np.int64)).to(dev),
        "n": torch.from_numpy(cfg["n"].view(np.int64)).to(dev),
        "mu": torch.from_numpy(cfg["mu"]).to(dev),
        "sigma": torch.from_numpy(cfg["sigma"]).to(dev),
    }
    methods = [("b1", nb.NRNG_METHOD_B1), ("polar", nb.NRNG_METHOD_POLAR)]
    extra_methods = {"p2": nb.NRNG_METHOD_P2, "b3": nb.NRNG_METHOD_B3, "ratio": nb.NRNG_METHOD_R,
                     "b2": nb.NRNG_METHOD_B2}
    if args.only in extra_methods:
        methods = [(args.only, extra_methods[args.only])]
    elif args.only:
        methods = [m for m in methods if m[0] == args.only]
    outs = {name: torch.empty(total, dtype=torch.float32, device=dev) for name, _ in methods}
    cons = {name: torch.zeros(ns, dtype=torch.int64, device=dev) for name, _ in methods}
    nb.nrng_reserve(total, ns)

    # Each method: plan (set-up kernel), then exec.  Every event costs the
    # stream a few microseconds (a marker, or the profiled dispatch of
    # hipExtLaunchKernel), so the timed steps time one kernel only: the
    # dominant one, the longest main kernel (B1's kernel; Polar's generate
    # kernel) in the warm-up steps.  Its exec dispatches it with two events
    # that take the dispatch's own start and end (nrng_batched_exec_timed).
    # The warm-up steps and the breakdown pass after the timed region launch
    # exec as its two parts with an event before and after each leg (plan,
    # count, main kernel): for Polar part 1 = the mask and scan kernels, part
    # 2 = the generate kernel; for B1 part 1 is empty.
    def step(timed=-1, evs=None):
        for i, (name, m) in enumerate(methods):
            nb.nrng_batched_plan(m, ns, D["n"], None, total, nb.NRNG_F32, stream, cons[name])
            if i == timed:
                nb.nrng_batched_exec_timed(0, m, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"],
                                           outs[name], nb.NRNG_F32, stream, cons[name], evs[0], evs[1])
            else:
                nb.nrng_batched_exec(m, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"],
                                     outs[name], nb.NRNG_F32, stream, cons[name])

    def breakdown_step(evs):
        for i, (name, m) in enumerate(methods):
            evs[4 * i].record(stream)
            nb.nrng_batched_plan(m, ns, D["n"], None, total, nb.NRNG_F32, stream, cons[name])
            for part in (1, 2):
                evs[4 * i + part].record(stream)
                nb.nrng_batched_exec_part(part, m, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"],
                                          outs[name], nb.NRNG_F32, stream, cons[name])
            evs[4 * i + 3].record(stream)

    def new_events(k):
        return [[torch.cuda.Event(enable_timing=True) for _ in range(k)] for _ in range(args.steps)]

    def leg_ms(evs, i, a, b):
        return sum(e[4 * i + a].elapsed_time(e[4 * i + b]) for e in evs) / len(evs)

    nev = 4 * len(methods)
    wu_events = [[torch.cuda.Event(enable_timing=True) for _ in range(nev)] for _ in range(args.warmup)]
    for s in range(args.warmup):
        breakdown_step(wu_events[s])
    torch.cuda.synchronize()
    # the dominant kernel, from the warm-up steps after the first
    probe = len(methods) - 1
    if args.warmup:
        wu = wu_events[1:] if args.warmup > 1 else wu_events
        probe = max(range(len(methods)), key=lambda i: leg_ms(wu, i, 2, 3))
    events = new_events(2)
    for evs in events:
        for e in evs:
            e.record(stream)   # torch creates an event on its first record
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(probe, events[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    normals = total * len(methods) * args.steps
    value = normals / elapsed
    probe_ms = sum(e[0].elapsed_time(e[1]) for e in events) / args.steps

    # breakdown pass (not timed as steps): every leg between events
    bd_events = new_events(nev)
    for s in range(args.steps):
        breakdown_step(bd_events[s])
    torch.cuda.synchronize()

    pairs = int(sum((int(x) + 1) // 2 for x in cfg["n"]))
    per_kernel = {}
    for i, (name, _) in enumerate(methods):
        # the dominant kernel live in the timed steps, the others from the
        # breakdown pass
        gen_ms = probe_ms if i == probe else leg_ms(bd_events, i, 2, 3)
        plan_ms, count_ms = leg_ms(bd_events, i, 0, 1), leg_ms(bd_events, i, 1, 2)
        exec_ms = count_ms + gen_ms
        gbs = 4.0 * total / (exec_ms * 1e-3) / 1e9
        kid = nb.KERNEL_B1_BATCHED if name in ("b1", "b3", "b2") else nb.KERNEL_POLAR
        wg, un, gpc = nb.nrng_tune_get(kid, nb.NRNG_F32)
        per_kernel[name] = {"plan_ms": round(plan_ms, 5), "exec_ms": round(exec_ms, 5),
                            "variant": {"wg": wg, "unroll": un, "grid_per_cu": gpc},
                            "normals_per_s": total / (exec_ms * 1e-3), "write_GBps": round(gbs, 1),
                            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                            "main_kernel_timed_in": "timed steps" if i == probe else "breakdown pass"}
        if name in ("polar", "p2", "ratio"):
            cand = int(u64sum(cons[name])) // 2       # candidates the method evaluates
            per_kernel[name]["count_ms"] = round(count_ms, 5)
            per_kernel[name]["generate_ms"] = round(gen_ms, 5)
            per_kernel[name]["candidates"] = cand
            gen_units = total if name == "ratio" else pairs    # R yields one normal per candidate
            units = {name + "_count": (count_ms, ALU_OPS[name + "_count"] * cand),
                     name + "_generate": (gen_ms, ALU_OPS[name + "_generate"] * gen_units)}
        else:
            units = {name + "_batched": (gen_ms, ALU_OPS[name + "_batched"] * pairs)}
        for k, (ms, ops) in units.items():
            per_kernel[name].setdefault("alu", {})[k] = {
                "ms": round(ms, 5), "Tops_per_s": round(ops / (ms * 1e-3) / 1e12, 2),
                "frac_valu_peak": round(ops / (ms * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4)}
        if name in ("polar", "p2", "ratio"):
            # the method as a whole (count + generate) on its own operations,
            # and the generate kernel's re-computation beside it
            ops = sum(ALU_OPS[k] * (cand if k.endswith("_count") else gen_units) for k in units)
            per_kernel[name]["alu_method"] = {
                "ms": round(exec_ms, 5), "ops": ops,
                "frac_valu_peak": round(ops / (exec_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4),
                "generate_recomputed_ops_per_unit": recomputed_ops(name + "_generate", paired_share(cfg))}

    # dominant kernel (the one timed live, picked in the warm-up steps) ->
    # roofline (ALU-bound: VALU lane operations on the method's own work),
    # with its HBM write rate beside (bytes: the output only, 4 B per FP32
    # normal)
    kern = {k: v for pk in per_kernel.values() for k, v in pk["alu"].items() if not k.endswith("_count")}
    dom = [k for k in per_kernel[methods[probe][0]]["alu"] if not k.endswith("_count")][0]
    traffic = read_traffic("batched_%s_f32" % dom)
    wbytes = 4 * total
    roofline = {"bound": "alu", "achieved": kern[dom]["Tops_per_s"], "peak": VALU_PEAK_TOPS,
                "unit": "Tlane-op/s", "frac": kern[dom]["frac_valu_peak"], "traffic": traffic,
                "kernel": KERNEL_NAMES[dom], "ms_per_launch": kern[dom]["ms"],
                "ops_per_unit": ALU_OPS[dom], "unit_of_work": ALU_UNIT[dom],
                "timed_by": "two HIP events that take this kernel's own dispatch start and end "
                            "(hipExtLaunchKernel) in every timed step, on its launch stream",
                "algorithmic_write_bytes_per_launch": wbytes,
                "hbm": {"achieved_GBps": round(wbytes / (kern[dom]["ms"] * 1e-3) / 1e9, 1), "peak_GBps": HBM_PEAK_GBS,
                        "frac": round(wbytes / (kern[dom]["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    if dom in IMPL_OVERHEAD_PAIRED:
        roofline["recomputed_ops_per_unit"] = recomputed_ops(dom, paired_share(cfg))
    prof = read_profile_avg("batched_%s_f32" % dom)
    if prof is not None:
        roofline["rocprof_avg_ms"] = prof

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "normals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched %d streams, B1 + Polar, FP32 out" % ns if len(methods) == 2 else
                   "batched %d streams, %s only, FP32 out" % (ns, methods[0][0]),
                   "nstreams": ns, "normals_per_method": total,
                   "lengths": "log-uniform on [1e2, 1e6]", "mu": "U(-10, 10)", "sigma": "U(0.1, 5)",
                   "seed_source": "PCG64(0xBA7C4)",
                   "seed_note": "per-stream lengths, mu, sigma and 64-bit seeds are drawn from PCG64 seeded "
                                "0xBA7C4, not seed_j = hash(j)", "parallelism": "single GPU"},
        "hbm_write_frac": round(4.0 * normals / elapsed / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": per_kernel,
        "roofline": roofline,
    }

    if args.calibrate:
        nbytes = 1 << 30
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
        nb.nrng_probe_store(src, nbytes, stream)
        nb.nrng_probe_copy(dst, src, nbytes, stream)
        torch.cuda.synchronize()
        result["calibration"] = {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "store_bytes": nbytes}
        del src, dst
    if not args.no_extras:
        result["extras"] = extras(nb, torch, dev, stream, per_kernel, value)
        for name, m in extra_methods.items():
            if args.only != name:
                result["extras"][name + "_batched"] = extra_batched(nb, torch, stream, D, ns, total, pairs,
                                                                    args.steps, per_kernel, m)
        ceiling = result["extras"]["store_ceiling_GBps"]
        for pk in per_kernel.values():
            pk["frac_store_ceiling"] = round(pk["write_GBps"] / ceiling, 4)
        cost = result["extras"]["valu_issue_cost"]
        w = {"mul": sum(cost[k] for k in ("v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32", "v_mad_i64_i32")) / 4,
             "shr64": cost["v_lshrrev_b64"], "add64": cost["v_lshl_add_u64"],
             "trans": sum(cost[k] for k in ("v_log_f32", "v_sin_f32", "v_sqrt_f32", "v_rcp_f32")) / 4,
             "other": 1.0}
        mix = ALU_MIX[dom]
        wops = sum(mix[c] * w[c] for c in mix)
        frac_w = roofline["frac"] * wops / ALU_OPS[dom]
        roofline["issue_weighted"] = {"ops_per_unit": round(wops, 2), "frac": round(frac_w, 4),
                                      "weights": {k: round(v, 3) for k, v in w.items()}}
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(cfg, [m for m, _ in methods])
    print(json.dumps(result), flush=True)
    return 0


def extra_batched(nb, torch, stream, D, ns, total, pairs, steps, per_kernel, m):
    """Method P2 (Section 4), B3 or B2 (Section 3) or Algorithm R (Section 5) on the
    same batched workload, timed like the step's legs: plan, then exec part 1
    (P2, R: the mask and scan kernels; B3, B2: nothing) and part 2 (the
    generate kernel; the B3 or B2 kernel) between events."""
    out = torch.empty(total, dtype=torch.float32, device=D["n"].device)
    cons = torch.zeros(ns, dtype=torch.int64, device=D["n"].device)

    def once(ev=None):
        if ev is not None:
            ev[0].record(stream)
        nb.nrng_batched_plan(m, ns, D["n"], None, total, nb.NRNG_F32, stream, cons)
        for part in (1, 2):
            if ev is not None:
                ev[part].record(stream)
            nb.nrng_batched_exec_part(part, m, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out,
                                      nb.NRNG_F32, stream, cons)
        if ev is not None:
            ev[3].record(stream)

    for _ in range(3):
        once()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for s in range(steps):
        once(evs[s])
    torch.cuda.synchronize()

    def avg(a, b):
        return sum(evs[s][a].elapsed_time(evs[s][b]) for s in range(steps)) / steps

    plan_ms, count_ms, gen_ms = avg(0, 1), avg(1, 2), avg(2, 3)
    exec_ms = count_ms + gen_ms
    r = {"plan_ms": round(plan_ms, 5), "exec_ms": round(exec_ms, 5), "normals_per_s": total / (exec_ms * 1e-3),
         "write_GBps": round(4.0 * total / (exec_ms * 1e-3) / 1e9, 1), "alu": {}}
    if m == nb.NRNG_METHOD_P2:
        cand = int(u64sum(cons)) // 2
        r.update({"count_ms": round(count_ms, 5), "generate_ms": round(gen_ms, 5), "candidates": cand})
        units = {"p2_count": (count_ms, ALU_OPS["p2_count"] * cand),
                 "p2_generate": (gen_ms, ALU_OPS["p2_generate"] * pairs)}
    elif m == nb.NRNG_METHOD_R:
        cand = int(u64sum(cons)) // 2
        r.update({"count_ms": round(count_ms, 5), "generate_ms": round(gen_ms, 5), "candidates": cand})
        units = {"ratio_count": (count_ms, ALU_OPS["ratio_count"] * cand),
                 "ratio_generate": (gen_ms, ALU_OPS["ratio_generate"] * total)}
    else:
        r["consumed_uniforms"] = int(u64sum(cons))
        key = "b3_batched" if m == nb.NRNG_METHOD_B3 else "b2_batched"
        units = {key: (gen_ms, ALU_OPS[key] * pairs)}
    for k, (ms, ops) in units.items():
        r["alu"][k] = {"ms": round(ms, 5), "Tops_per_s": round(ops / (ms * 1e-3) / 1e12, 2),
                       "frac_valu_peak": round(ops / (ms * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4)}
    ref = "b1" if m in (nb.NRNG_METHOD_B3, nb.NRNG_METHOD_B2) else "polar"
    if ref in per_kernel:
        r["exec_vs_" + ref] = round(per_kernel[ref]["exec_ms"] / exec_ms, 4)
    return r


def extras(nb, torch, dev, stream, per_kernel, batched_value):
    """Side measurements (not part of the timed step)."""
    ex = {}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return median(ts)

    # store-only ceiling: the best of plain and nontemporal 16-byte stores
    # over workgroups per CU and stores per thread per step (4 GiB each)
    nbytes = 4 << 30
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    sweep = {}
    for nt in (0, 1):
        for bpc in (4, 8, 16, 32):
            for unr in (1, 2, 4, 8):
                ms = timed(lambda: nb.nrng_probe_store_variant(buf, nbytes, nt, bpc, unr, stream), 4)
                sweep["%s_wg%d_u%d" % ("nt" if nt else "plain", bpc, unr)] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    best = max(sweep, key=sweep.get)
    ex["store_ceiling_GBps"] = sweep[best]
    ex["store_ceiling_form"] = best
    ex["store_sweep_GBps"] = sweep
    sink = torch.empty(256 * 2048, dtype=torch.int64, device=dev)
    nh = 1 << 33
    ms = timed(lambda: nb.nrng_probe_hash(1, nh, sink, sink.numel(), stream), 5)
    ex["hash_ceiling_per_s"] = nh / (ms * 1e-3)
    # issue cost of single VALU instructions, in units of the peak's lane-op
    # (one FP32 FMA per lane per cycle at 2.4 GHz): whole chip, 8 chains per lane
    cus = nb.nrng_device_cus()
    iters = 4096
    lane_ops = cus * 8 * 256 * 8 * iters
    vsink = torch.empty(cus * 8 * 256, dtype=torch.int32, device=dev)
    ex["valu_issue_cost"] = {}
    for op, name in enumerate(nb.VALU_PROBE_OPS):
        ms = timed(lambda: nb.nrng_probe_valu(op, iters, vsink, vsink.numel(), stream), 5)
        ex["valu_issue_cost"][name] = round(VALU_PEAK_TOPS * 1e12 / (lane_ops / (ms * 1e-3)), 3)

    # single-stream fills of 2^30 normals (FP32 / BF16 / FP16 / plain FP64)
    n = 1 << 30
    single = {}
    for name, dt, nbytes_el in (("f32", nb.NRNG_F32, 4), ("bf16", nb.NRNG_BF16, 2), ("f16", nb.NRNG_F16, 2),
                                ("f64", nb.NRNG_F64, 8)):
        out = torch.empty(n * nbytes_el // 4, dtype=torch.float32, device=dev)
        nb.nrng_reserve(n, 0)
        r = {}
        ms = timed(lambda: nb.nrng_boxmuller(1, 0, n, 0.0, 1.0, out, dt, stream), 5)
        r["b1_normals_per_s"] = n / (ms * 1e-3)
        r["b1_write_GBps"] = round(n * nbytes_el / (ms * 1e-3) / 1e9, 1)
        ms = timed(lambda: nb.nrng_polar(7, 0, n, 0.0, 1.0, out, dt, stream, None), 5)
        r["polar_normals_per_s"] = n / (ms * 1e-3)
        r["polar_write_GBps"] = round(n * nbytes_el / (ms * 1e-3) / 1e9, 1)
        ms = timed(lambda: nb.nrng_polar2(7, 0, n, 0.0, 1.0, out, dt, stream, None), 5)
        r["p2_normals_per_s"] = n / (ms * 1e-3)
        ms = timed(lambda: nb.nrng_b3(1, 0, n, 0.0, 1.0, out, dt, stream), 5)
        r["b3_normals_per_s"] = n / (ms * 1e-3)
        ms = timed(lambda: nb.nrng_ratio(21, 0, n, 0.0, 1.0, out, dt, stream, None), 3)
        r["ratio_normals_per_s"] = n / (ms * 1e-3)
        ms = timed(lambda: nb.nrng_b2(1, 0, n, 0.0, 1.0, out, dt, stream), 5)
        r["b2_normals_per_s"] = n / (ms * 1e-3)
        single[name] = r
        del out
        torch.cuda.empty_cache()
    ex["single_stream_2^30"] = single
    f64 = single["f64"]
    ex["fp32_batched_vs_plain_fp64"] = {
        "b1": per_kernel["b1"]["normals_per_s"] / f64["b1_normals_per_s"] if "b1" in per_kernel else None,
        "polar": per_kernel["polar"]["normals_per_s"] / f64["polar_normals_per_s"] if "polar" in per_kernel else None,
        "step_vs_mean_fp64": batched_value / (0.5 * (f64["b1_normals_per_s"] + f64["polar_normals_per_s"])),
    }

    # the two small parity configurations: B1 FP64 2^20 normals (seed 1) and
    # Polar 2^24 normals (seed 7), FP64 and FP32
    small = {}
    for key, fn, seed, n, dt, el in (("b1_f64_2^20", nb.nrng_boxmuller, 1, 1 << 20, nb.NRNG_F64, 8),
                                     ("polar_f64_2^24", nb.nrng_polar, 7, 1 << 24, nb.NRNG_F64, 8),
                                     ("polar_f32_2^24", nb.nrng_polar, 7, 1 << 24, nb.NRNG_F32, 4)):
        out = torch.empty(n * el // 4, dtype=torch.float32, device=dev)
        if fn is nb.nrng_polar:
            ms = timed(lambda: fn(seed, 0, n, 0.0, 1.0, out, dt, stream, None), 10)
        else:
            ms = timed(lambda: fn(seed, 0, n, 0.0, 1.0, out, dt, stream), 10)
        small[key + "_normals_per_s"] = n / (ms * 1e-3)
        del out
    ex["small_configs"] = small

    # repeated fill: 64 graph replays of a 2^28 FP32 Polar fill
    nf = 1 << 28
    out = torch.empty(nf, dtype=torch.float32, device=dev)
    cursor = torch.zeros(1, dtype=torch.int64, device=dev)
    side = torch.cuda.Stream()
    g = nb.nrng_fillgraph_create(7, cursor, nf, 0.0, 1.0, out, nb.NRNG_F32, side)
    try:
        nb.nrng_fillgraph_launch(g, side)
        side.synchronize()
        cursor.zero_()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(side)
        for _ in range(64):
            nb.nrng_fillgraph_launch(g, side)
        b.record(side)
        side.synchronize()
        ms = a.elapsed_time(b)
    finally:
        nb.nrng_fillgraph_destroy(g)
    ex["graph_fill_64x2^28"] = {"ms_total": round(ms, 3), "normals_per_s": 64 * nf / (ms * 1e-3),
                               "write_GBps": round(64 * nf * 4 / (ms * 1e-3) / 1e9, 1),
                               "cursor_after": int(cursor.item())}
    return ex


def cpu_baseline(cfg, methods):
    """The FP64 oracle over every stream of the same batched workload, one
    oracle call per stream, spread over the host cores."""
    import numpy as np  # noqa: F401
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O
    O.lib()
    cores = os.cpu_count() or 1   # every host core the process sees (nproc)
    ns = len(cfg["n"])
    jobs = [(m, j) for m in methods for j in range(ns)]

    def work(mj):
        m, j = mj
        fn = {"b1": O.b1, "polar": O.polar, "p2": O.polar2, "b3": O.b3, "ratio": O.ratio, "b2": O.b2}[m]
        fn(int(cfg["seed"][j]), int(cfg["offset"][j]), int(cfg["n"][j]), float(cfg["mu"][j]), float(cfg["sigma"][j]))
        return int(cfg["n"][j])

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        done = sum(ex.map(work, jobs, chunksize=8))
    dt = time.perf_counter() - t0
    # the same oracle on one thread, on the two small parity configurations:
    # B1 FP64 seed 1, 2^20 normals; Polar seed 7, 2^24 normals
    single = {}
    for key, fn, seed, n in (("b1_2^20", O.b1, 1, 1 << 20), ("polar_2^24", O.polar, 7, 1 << 24)):
        t1 = time.perf_counter()
        fn(seed, 0, n)
        single[key + "_normals_per_s"] = n / (time.perf_counter() - t1)
    # and on every host core: B1 split into chunks of whole pairs, Polar by a
    # count pass, a prefix of the counts and a generate pass (the same oracle
    # routines as above on disjoint chunks), for the small configurations and
    # the 2^30 single streams
    multi = {}
    for key, fn, seed, n in (("b1_2^20", O.b1_parallel, 1, 1 << 20), ("polar_2^24", O.polar_parallel, 7, 1 << 24),
                             ("b1_2^30", O.b1_parallel, 1, 1 << 30), ("polar_2^30", O.polar_parallel, 7, 1 << 30)):
        piece = max(4096, n // 2 // (4 * cores))   # about four chunks per thread
        kw = {"chunk_pairs": piece} if fn is O.b1_parallel else {"chunk": piece}
        best = None
        for _ in range(2 if n <= 1 << 24 else 1):   # the small ones: best of two
            t1 = time.perf_counter()
            r = fn(seed, 0, n, threads=cores, **kw)
            t2 = time.perf_counter() - t1
            best = t2 if best is None else min(best, t2)
            del r
        multi[key + "_normals_per_s"] = n / best
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = cores
    return {"value": done / dt, "unit": "normals/s", "cores": cores, "nproc_affinity": affinity, "kind": "oracle",
            "sample": "the whole batched workload: %d streams x %s, %d normals, one FP64 oracle call per "
                      "stream on a %d-thread pool (%.1f s wall)" % (ns, "+".join(methods), done, cores, dt),
            "single_thread": single, "host_cores": multi}


if __name__ == "__main__":
    sys.exit(main())
