#!/usr/bin/env python3
"""Benchmark of the Heston Monte Carlo / Longstaff-Schwartz hot path on one MI355X.

One step = one full large risk run: 64 American puts (K=110, T=1, S0=100, r=0.02; each
underlying with its own Heston parameters drawn from the batch ranges), 1,048,576 paths x
252 steps each, QE scheme, Philox seed 5 and stream u for underlying u.  For every underlying
one simr_greeks call: the forward pass writing the path states, the Gram pre-pass, the
cooperative Longstaff-Schwartz induction (the price) and the adjoint sweep (the 7 Greeks).
`value` is path-steps per second of the step (64 x 2^20 x 252 / step time).  Inputs are
generated in-kernel from the counter-based RNG, so nothing is transferred before the timed
region.

Also reported: the pricing pass alone, the bump-and-revalue cost of the same 7 Greeks (15
pricing passes with common random numbers, on the first 4 underlyings), per-kernel-group times
from HIP events the library records on the launch stream, the roofline of every group and of
the dominant one, the single-option American put risk step (131,072 x 252) and the 1,024-option
European batch as secondary workloads, and the FP64 CPU oracle timed on a bounded sample: the
first 65,536 paths of the first underlyings, which the GPU reruns on the same paths for the
error report (a Longstaff-Schwartz price depends on every path of its regression, so the GPU
prices the subsample itself).

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--extra] [--basket]
"""
from __future__ import annotations

import argparse
import ctypes
import gc
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector

# Algorithmic FP32 floating-point operations per path-step (FMA = 2, every other
# arithmetic op or transcendental = 1; the integer Philox work and int->float
# conversions are not counted), QE quadratic branch:
#   uniform map 3 FMA = 6; Box-Muller log2, scale, sqrt, sin, cos, 2 mul = 7;
#   QE variance step 22; log-price update 11.
FLOPS_FORWARD = 46
# Adjoint: recompute of the variance path (uniforms, Box-Muller, QE = 35) plus the
# reverse of the log-price step (23) and of the QE step (63).
FLOPS_ADJOINT = 121
# Longstaff-Schwartz: each date reads every path's (x, v) once: 8 bytes per path-date.
LSM_BYTES_PER_PATH_DATE = 8
SPILL_BYTES_PER_PATH_STEP = 8

# The paper's fastest design per Table 1 shape (programmable-logic multi-kernel, 6 compute units,
# Alveo U280, FP32, random inputs streamed from the host), its Table 3: context only, other
# hardware and a different input path.
PAPER_TABLE1_BEST_MS = {"tiny": 77.81, "small": 98.46, "medium": 221.71, "large": 544.48}

GROUPS = {0: "price", 1: "forward_spill", 2: "lsm_backward", 3: "forward_ckpt", 4: "adjoint", 5: "lsm_gram",
          6: "lsm_factor"}
ALL_GROUPS = (1 << len(GROUPS)) - 1

# Measured per launch, keyed by (group, paths, steps) -- the 1,024-option batch by ("price", "c3")
# -- from rocprofv3 --pmc runs of this script (the summaries under profiles/ give the commands):
#  * HBM bytes: FETCH_SIZE and WRITE_SIZE scaled by what the same counters read for a plain
#    256 MiB device copy (fetch x2.000, write x1.000);
#  * VALU issue quad-cycles: SQ_INSTS_VALU + SQ_INSTS_VALU_TRANS_F32 - SQ_ACTIVE_INST_VALU2, i.e.
#    one quad-cycle per VALU instruction, two for a transcendental (measured on this GPU: a
#    stream of v_log/v_exp/v_sqrt/v_rcp/v_sin issues at half the rate of v_fma_f32), and one
#    for each pair the SIMD issued together (gfx950 co-issues, e.g., v_bitop3_b32 beside an FMA).
# They describe the kernel sources whose digest is given and are reported only while the sources
# match.  At 2^20 paths one induction launch carries two options (the large risk run's pairs).
TRAFFIC_SOURCES_DIGEST = "944137fa530abe2b"
TRAFFIC_BYTES = {
    ('forward_spill', 1048576, 252): 2.1140e+09,
    ('lsm_gram', 1048576, 252): 2.1096e+09,
    ('lsm_backward', 1048576, 252): 4.3070e+09,
    ('adjoint', 1048576, 252): 1.6143e+08,
    ('forward_spill', 131072, 252): 2.6432e+08,
    ('lsm_gram', 131072, 252): 2.6383e+08,
    ('lsm_backward', 131072, 252): 2.7516e+08,
    ('adjoint', 131072, 252): 1.8000e+07,
    ('price', 'c3'): 2.5148e+07,
}
VALU_ISSUE_QUADS = {
    ('forward_spill', 1048576, 252): 3.0258e+08,
    ('lsm_gram', 1048576, 252): 1.5808e+08,
    ('lsm_backward', 1048576, 252): 4.6190e+08,
    ('adjoint', 1048576, 252): 2.6387e+08,
    ('forward_spill', 131072, 252): 3.9521e+07,
    ('lsm_gram', 131072, 252): 1.7041e+07,
    ('lsm_backward', 131072, 252): 3.3121e+07,
    ('adjoint', 131072, 252): 3.8016e+07,
    ('price', 'c3'): 2.3995e+10,
}
# Issue quad-cycles per second of the chip: 256 CUs x 4 SIMDs x 2.4 GHz / 4.  A plain stream of
# independent v_fma_f32 reaches 0.90 of it on this GPU.
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4

def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for p in ("simr_kernels.hip", "simr_device.hpp"):
        with open(os.path.join(ROOT, "paper_2402_12111_amd", "csrc", p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-underlyings", type=int, default=4,
                    help="underlyings whose 65,536-path subsample the oracle prices (about 3 s each on 16 cores)")
    ap.add_argument("--extra", action="store_true",
                    help="also time the c4 Greeks, the schemes, the exact scheme, baskets and the paper's Table 1 shapes")
    ap.add_argument("--basket", action="store_true",
                    help="only the basket workloads (one JSON object; for kernel profiles)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (counter calibration)")
    return ap.parse_args()


def copy_probe(mib):
    """A plain copy of known size: what the HBM counters read for it calibrates them."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3, "ok": bool(torch.equal(src, dst))}))


def read_groups(L, ctx):
    groups = {}
    for gid, name in GROUPS.items():
        ms, n = ctypes.c_double(), ctypes.c_int64()
        L.simr_profile_read(ctx, gid, ctypes.byref(ms), ctypes.byref(n))
        if n.value:
            groups[name] = {"avg_ms": ms.value / n.value, "launches": n.value, "total_ms": ms.value}
    L.simr_profile_reset(ctx)
    return groups


def timed(fn, reps, torch, per_call=None):
    """Milliseconds per call of fn over reps calls, bracketed by device synchronisations.  As
    Python's timeit does, the interpreter's cyclic garbage collector is paused while timing (after
    one collection): a collection pass over the interpreter's objects can take tens of
    milliseconds of host time, during which nothing is enqueued."""
    gc.collect()
    was_enabled = gc.isenabled()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = t0
        for _ in range(reps):
            out = fn()
            if per_call is not None:  # fn synchronises its stream before it returns
                now = time.perf_counter()
                per_call.append((now - t) * 1e3)
                t = now
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, out
    finally:
        if was_enabled:
            gc.enable()


def roofline(name, info, P, N, traffic_current, path_steps=None, key=None, opts_per_launch=1):
    """The roofline of one kernel group: `achieved` is the algorithmic work of one launch (one
    option of P paths x N steps, or `path_steps` in all; the induction's launch carries
    `opts_per_launch` such options side by side) over the group's average launch time, measured
    live."""
    sec = info["avg_ms"] * 1e-3
    if name in ("lsm_backward", "lsm_gram"):
        m = opts_per_launch if name == "lsm_backward" else 1
        work = m * LSM_BYTES_PER_PATH_DATE * P * (N - 1)
        r = {"bound": "hbm", "achieved": work / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "per_launch_work": f"{LSM_BYTES_PER_PATH_DATE} B x {P} paths x {N - 1} dates"}
        if m > 1:
            r["per_launch_work"] = f"{m} options x " + r["per_launch_work"]
    elif name == "lsm_factor":
        r = {"bound": "latency", "achieved": None, "peak": None, "unit": None,
             "per_launch_work": f"{N - 1} FP64 factorisations of 6 x 6 Gram sums"}
    else:
        fl = FLOPS_ADJOINT if name == "adjoint" else FLOPS_FORWARD
        ps = P * N if path_steps is None else path_steps
        r = {"bound": "alu", "achieved": fl * ps / sec / 1e12, "peak": FP32_PEAK_TFLOPS,
             "unit": "TFLOP/s", "per_launch_work": (f"{fl} FLOP x {P} paths x {N} steps" if path_steps is None
                                                    else f"{fl} FLOP x {ps} path-steps")}
        if name == "adjoint":
            r["per_launch_work"] += (" (an upper bound: each path is swept to its exercise index,"
                                     " out-of-the-money paths not at all)")
    r["frac"] = r["achieved"] / r["peak"] if r["achieved"] is not None else None
    key = (name, P, N) if key is None else key
    if traffic_current and key in VALU_ISSUE_QUADS:
        # instruction-issue view: the counted issue quad-cycles of one launch (dynamic, branch
        # divergence included) over the launch time, against the chip's issue quad-cycles
        r["valu_issue_frac"] = VALU_ISSUE_QUADS[key] / sec / VALU_ISSUE_PEAK
        r["valu_issue_quads_per_launch"] = VALU_ISSUE_QUADS[key]
    r["traffic"] = TRAFFIC_BYTES.get(key) if traffic_current else None
    r["kernel"] = name
    r["avg_ms"] = info["avg_ms"]
    if name == "lsm_backward":
        # the induction is one chip-wide exchange per exercise date: its time per date is the
        # figure that bounds it (per date of the launch, all its options)
        r["us_per_date"] = info["avg_ms"] * 1e3 / (N - 1)
        r["options_per_launch"] = opts_per_launch
    return r


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path shards by paths or by option with no collectives, "
              "and runs on more than one GPU are not supported (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2402_12111_amd import simr
    from paper_2402_12111_amd import workloads as W

    L = simr.library()
    ctx = simr.context()
    L.simr_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.simr_profile_groups.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    L.simr_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]
    L.simr_profile_reset.argtypes = [ctypes.c_void_p]
    if args.basket:
        print(json.dumps({"basket": basket_workloads(simr, W, torch)}))
        return

    opts = W.c5_risk()
    P, N = opts[0]["paths"], opts[0]["steps"]
    path_steps = W.path_steps(opts)
    traffic_current = kernel_sources_digest() == TRAFFIC_SOURCES_DIGEST

    def c5_pass():  # the 64 underlyings in one call: one synchronisation per step
        return simr.greeks_batch(opts)

    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            c5_pass()
        simr.price(opts[0])
        torch.cuda.synchronize()

        # ---- one untimed step with every kernel group's launches bracketed by events ---------
        L.simr_profile_reset(ctx)
        L.simr_profile_enable(ctx, 1)
        c5_pass()
        L.simr_profile_enable(ctx, 0)
        groups = read_groups(L, ctx)
        dom = max(groups.items(), key=lambda kv: kv[1]["total_ms"])[0]

        # ---- timed region: K full risk runs, events around the dominant group's launches only
        # (each recorded launch adds two events to the stream; the other groups run unprofiled)
        L.simr_profile_groups(ctx, 1 << {v: k for k, v in GROUPS.items()}[dom])
        L.simr_profile_enable(ctx, 1)
        step_ms = []
        ms_step, res = timed(c5_pass, args.steps, torch, step_ms)
        L.simr_profile_enable(ctx, 0)
        live = read_groups(L, ctx)[dom]
        L.simr_profile_groups(ctx, ALL_GROUPS)

        # ---- pricing pass alone, and bump-and-revalue of the 7 Greeks ---------------------
        ms_price, _ = timed(lambda: simr.price_batch(opts), 2, torch)
        sub = opts[:4]
        ms_price_sub, _ = timed(lambda: simr.price_batch(sub), 2, torch)
        bumped = []
        for o in sub:
            bumped.append(o)
            for name in simr.GREEK_NAMES:
                h = 1e-4 * abs(o[name])
                bumped += [dict(o, **{name: o[name] + h}), dict(o, **{name: o[name] - h})]
        ms_bump_sub, _ = timed(lambda: simr.price_batch(bumped), 1, torch)

        # ---- secondary workloads: the single-option risk step, the European batch --------------
        out["c2_risk_step"] = c2_step(simr, W, torch, L, ctx, args.steps, traffic_current)
        out["c3_batch"] = c3_batch(simr, W, torch, L, ctx, traffic_current)
        if args.extra:
            out["extra"] = extra_workloads(simr, W, torch)

    value = path_steps / (ms_step * 1e-3)
    # consecutive underlyings share the induction's cooperative launch (two of 2^20 paths fit)
    opl = round(len(opts) / groups["lsm_backward"]["launches"])
    rooflines = {name: roofline(name, info, P, N, traffic_current, opts_per_launch=opl)
                 for name, info in groups.items()}
    # the dominant group's roofline from its launches in the timed region
    roof = roofline(dom, live, P, N, traffic_current, opts_per_launch=opl)
    roof["measured_over"] = f"the {live['launches']} launches of the {args.steps} timed steps"

    res_line = {
        "metric": "Heston path-steps/sec and Greeks/sec (adjoint vs bump) at fixed price error",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": statistics.median(step_ms),
        "ms_per_step_range": [min(step_ms), max(step_ms)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (in-kernel Philox4x32-10 draws, seeded; Heston parameters from numpy default_rng(5))",
        "config": {"workload": "large risk run: 64 American puts (K=110, T=1), each with its own Heston "
                               "parameters, 1048576 paths x 252 steps each, LSM price + 7 adjoint Greeks, QE",
                   "underlyings": len(opts), "paths": P, "time_steps": N, "scheme": "QE",
                   "precision": "fp32 paths, fp64 sums/solve"},
        "greeks_per_s": 7.0 * len(opts) / (ms_step * 1e-3),
        "options_per_s": len(opts) / (ms_step * 1e-3),
        "underlying_0": {"price": res[0].price, "price_std_err": res[0].std_err,
                         "greeks": dict(zip(simr.GREEK_NAMES, res[0].grads))},
        "pricing_pass_ms": ms_price,
        "pricing_path_steps_per_s": path_steps / (ms_price * 1e-3),
        "adjoint_ratio": ms_step / ms_price,
        "bump_sample": f"15 CRN pricing passes (the price and +-1e-4 relative bumps of the 7 inputs) of the "
                       f"first {len(sub)} underlyings, against one pricing pass of the same",
        "bump_ms_per_underlying": ms_bump_sub / len(sub),
        "bump_ratio": ms_bump_sub / ms_price_sub,
        "greeks_per_s_bump": 7.0 * len(sub) / (ms_bump_sub * 1e-3),
        "kernel_groups": groups,
        "kernel_groups_measured_over": "one untimed step before the timed region, every group's launches "
                                       "bracketed by events",
        "roofline": roof,
        "kernel_rooflines": rooflines,
    }
    res_line.update(out)
    if not args.no_cpu_baseline:
        res_line["cpu_baseline"], ref = cpu_baseline(opts[:max(1, args.cpu_underlyings)])
        res_line["error_vs_oracle"] = error_vs_oracle(simr, ref)
        res_line["error_vs_oracle_c1"] = c1_errors(simr, W)
    print(json.dumps(res_line))


def c2_step(simr, W, torch, L, ctx, steps, traffic_current):
    """The single-option risk step: American put K=110, 131,072 paths x 252 steps, one
    simr_greeks call, with its own kernel-group times and rooflines."""
    opt = W.c2_american()
    P, N = opt["paths"], opt["steps"]
    simr.greeks(opt)
    L.simr_profile_reset(ctx)
    L.simr_profile_enable(ctx, 1)
    ms, g = timed(lambda: simr.greeks(opt), steps, torch)
    L.simr_profile_enable(ctx, 0)
    groups = read_groups(L, ctx)
    ms_price, _ = timed(lambda: simr.price(opt), steps, torch)
    rl = {name: roofline(name, info, P, N, traffic_current) for name, info in groups.items()}
    return {"paths": P, "time_steps": N, "ms": ms, "path_steps_per_s": P * N / (ms * 1e-3),
            "greeks_per_s": 7.0 / (ms * 1e-3), "pricing_pass_ms": ms_price, "adjoint_ratio": ms / ms_price,
            "price": g.price, "price_std_err": g.std_err, "greeks": dict(zip(simr.GREEK_NAMES, g.grads)),
            "kernel_groups": groups, "kernel_rooflines": rl}


def c3_batch(simr, W, torch, L, ctx, traffic_current):
    """The 1,024-option European batch in one simr_price_batch call (on the bench's stream: the
    captured graph, replayed), then one call with the library's events around the persistent
    kernel (enqueued directly while profiling) for its roofline."""
    opts = W.c3_batch()
    simr.price_batch(opts)  # tunes and captures the graph
    ms, _ = timed(lambda: simr.price_batch(opts), 3, torch)
    ps = W.path_steps(opts)
    L.simr_profile_reset(ctx)
    L.simr_profile_enable(ctx, 1)
    simr.price_batch(opts)
    L.simr_profile_enable(ctx, 0)
    groups = read_groups(L, ctx)
    out = {"options": len(opts), "path_steps": ps, "ms": ms, "path_steps_per_s": ps / (ms * 1e-3),
           "options_per_s": len(opts) / (ms * 1e-3), "tile": simr.get_tile()}
    if "price" in groups:
        out["kernel_ms"] = groups["price"]["avg_ms"]
        out["roofline"] = roofline("price", groups["price"], None, None, traffic_current, path_steps=ps,
                                   key=("price", "c3"))
    return out


GREEK_NAMES_BENCH = ("S0", "v0", "theta", "r", "kappa", "xi", "rho")


def c1_errors(simr, W):
    """The small European call (8192 paths x 64 steps, QE): the GPU price against the FP64
    oracle on the same paths, and both against the characteristic-function closed form."""
    import oracle
    from oracle import heston_cf
    c1 = W.c1_european()
    g = simr.price(c1)
    p, se, _ = oracle.price_european(oracle.Option(**c1))
    cf = heston_cf.call_price(c1["S0"], c1["K"], c1["T"], c1["r"], c1["kappa"], c1["theta"], c1["xi"], c1["rho"],
                              c1["v0"])
    return {"gpu": g.price, "oracle": p, "closed_form": cf, "std_err": se, "gpu_minus_oracle_per_S0": (g.price - p) / c1["S0"],
            "gpu_minus_closed_form_in_std_err": (g.price - cf) / se}


SUBSAMPLE_PATHS = 65536
SINGLE_CORE_PATHS = 8192


def cpu_baseline(opts):
    """The FP64 oracle (LSM price + forward-mode Greeks) on the first 65,536 paths of each of
    `opts`, on all host cores: the reported CPU rate and the reference values of the error
    report."""
    import oracle
    threads = oracle.default_threads()
    refs = []
    t0 = time.perf_counter()
    for o in opts:
        sub = oracle.Option(**dict(o, paths=SUBSAMPLE_PATHS))
        price, se, grads, grad_se = oracle.greeks(sub, nthreads=threads)
        refs.append((o, price, se, [float(x) for x in grads], [float(x) for x in grad_se]))
    dt = time.perf_counter() - t0
    steps = SUBSAMPLE_PATHS * opts[0]["steps"] * len(opts)
    # the same computation on one core, on the first 8,192 paths of the first underlying
    t1 = time.perf_counter()
    oracle.greeks(oracle.Option(**dict(opts[0], paths=SINGLE_CORE_PATHS)), nthreads=1)
    dt1 = time.perf_counter() - t1
    res = {"value": steps / dt, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"LSM price + 7 forward-mode Greeks on the first {SUBSAMPLE_PATHS} of {opts[0]['paths']} "
                     f"paths x {opts[0]['steps']} steps of the first {len(opts)} of the 64 underlyings",
           "seconds": dt, "cpu": cpu_model(),
           "single_core": {"value": SINGLE_CORE_PATHS * opts[0]["steps"] / dt1, "unit": "path-steps/s",
                           "sample": f"the same on the first {SINGLE_CORE_PATHS} paths of the first underlying, "
                                     f"one thread", "seconds": dt1}}
    return res, refs


def cpu_model():
    """The host CPU's model name, as /proc/cpuinfo gives it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def error_vs_oracle(simr, refs):
    """The GPU rerun of each 65,536-path subsample against the FP64 oracle's on the same paths.
    Each side prices with its own in-sample exercise policy (FP32 and FP64 paths), and each
    side's Greeks hold its own policy fixed: the price error in units of S0 and of the standard
    error, each Greek's error relative to its scale max(|g|, s_g), s_g the per-path standard
    deviation.  Then the GPU's exercise policy valued by the oracle on its FP64 paths (the
    stopping rule fixed, so FP32-vs-FP64 near-tie decisions drop out): the GPU's price and
    Greeks against that valuation."""
    import oracle
    out = []
    for o, price, se, grads, grad_se in refs:
        sub = dict(o, paths=SUBSAMPLE_PATHS)
        g = simr.greeks(sub)
        e = {"underlying": o["stream"], "paths": SUBSAMPLE_PATHS,
             "price": {"gpu": g.price, "oracle": price, "per_S0": abs(g.price - price) / o["S0"],
                       "in_std_err": abs(g.price - price) / max(se, 1e-300)},
             "greeks_rel_to_scale": {}}
        for name, a, b_, bse in zip(GREEK_NAMES_BENCH, g.grads, grads, grad_se):
            scale = max(abs(b_), bse * math.sqrt(SUBSAMPLE_PATHS))
            e["greeks_rel_to_scale"][name] = abs(a - b_) / scale
        _, tau, _ = simr.debug_lsm(sub)
        pv, pse, pg, pgse = oracle.greeks_at_tau(oracle.Option(**sub), tau)
        e["gpu_policy_valued_by_oracle"] = {
            "price_per_S0": abs(g.price - pv) / o["S0"],
            "greeks_rel_to_scale": {name: abs(a - b_) / max(abs(b_), bse * math.sqrt(SUBSAMPLE_PATHS))
                                    for name, a, b_, bse in zip(GREEK_NAMES_BENCH, g.grads, pg, pgse)}}
        out.append(e)
    worst = {"price_per_S0": max(e["price"]["per_S0"] for e in out),
             "price_in_std_err": max(e["price"]["in_std_err"] for e in out),
             "greek_rel_to_scale": max(max(e["greeks_rel_to_scale"].values()) for e in out),
             "policy_price_per_S0": max(e["gpu_policy_valued_by_oracle"]["price_per_S0"] for e in out),
             "policy_greek_rel_to_scale": max(max(e["gpu_policy_valued_by_oracle"]["greeks_rel_to_scale"].values())
                                              for e in out)}
    return {"worst": worst, "underlyings": out}


def basket_workloads(simr, W, torch):
    """The 8-asset European call with deltas and cross-gammas (the path kernel timed live by the
    library's HIP events, with its VALU-issue roofline), the 8-asset American put, and the
    paper's Table 1 asset counts as one correlated American basket each."""
    res = {}
    L = simr.library()
    ctx = simr.context()
    eu, am = W.basket_risk()
    for name, bk, fn in (("basket8_european_greeks", eu, simr.basket_greeks),
                         ("basket8_european_risk", eu, simr.basket_risk),
                         ("basket8_american", am, simr.basket_price)):
        fn(bk)
        torch.cuda.synchronize()
        L.simr_profile_reset(ctx)
        L.simr_profile_enable(ctx, 1)
        t0 = time.perf_counter()
        fn(bk)
        torch.cuda.synchronize()
        ms_b = (time.perf_counter() - t0) * 1e3
        L.simr_profile_enable(ctx, 0)
        kms, n = ctypes.c_double(), ctypes.c_int64()
        L.simr_profile_read(ctx, 0, ctypes.byref(kms), ctypes.byref(n))
        L.simr_profile_reset(ctx)
        aps = W.asset_path_steps(bk)
        r = {"assets": len(bk["S0"]), "paths": bk["paths"], "steps": bk["steps"], "ms": ms_b,
             "asset_path_steps_per_s": aps / (ms_b * 1e-3)}
        if n.value:
            r["path_kernel_ms"] = kms.value / n.value
        res[name] = r
    for size in W.TABLE1:
        bk = W.table1_basket(size)
        simr.basket_price(bk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = simr.basket_price(bk)
        torch.cuda.synchronize()
        ms_b = (time.perf_counter() - t0) * 1e3
        res[f"table1_basket_{size}"] = {"assets": len(bk["S0"]), "steps": bk["steps"], "paths": bk["paths"],
                                        "ms": ms_b, "price": r.price,
                                        "asset_path_steps_per_s": W.asset_path_steps(bk) / (ms_b * 1e-3)}
    return res


def extra_workloads(simr, W, torch):
    res = {}
    reps = 3
    opts = W.c3_batch()
    ps = W.path_steps(opts)
    # the same batch under the martingale-corrected QE scheme (one more log per step) and the
    # truncated Gaussian scheme (a table lookup per step, no uniform draw used)
    for name, scheme in (("c3_batch_qe_m", simr.SCHEME_QE_M), ("c3_batch_tg", simr.SCHEME_TG)):
        simr.price_batch(opts, scheme)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            simr.price_batch(opts, scheme)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[name] = {"options": len(opts), "ms": ms, "path_steps_per_s": ps / (ms * 1e-3)}
    # discretisation bias against the exact scheme: the C1 call on 2^20 paths priced by
    # Broadie-Kaya in one step (no bias), and by the other schemes at 64 and 8 steps
    base = W.option(paths=1 << 20)
    simr.price(dict(base, steps=1, paths=4096), simr.SCHEME_BK)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ex = simr.price(dict(base, steps=1), simr.SCHEME_BK)
    torch.cuda.synchronize()
    res["exact_bk_c1"] = {"steps": 1, "paths": base["paths"], "price": ex.price, "std_err": ex.std_err,
                          "ms": (time.perf_counter() - t0) * 1e3}
    for name, scheme in (("qe", simr.SCHEME_QE), ("qe_m", simr.SCHEME_QE_M), ("tg", simr.SCHEME_TG),
                         ("fte", simr.SCHEME_FTE)):
        for steps in (64, 8):
            r = simr.price(dict(base, steps=steps), scheme)
            res[f"bias_{name}_{steps}"] = {"price": r.price, "minus_exact": r.price - ex.price,
                                           "se": math.hypot(r.std_err, ex.std_err)}
    res.update(basket_workloads(simr, W, torch))
    for o in W.c4_greeks():
        simr.greeks(o)  # warm: workspace, pinned staging, and the pricing call's tile and graph
        simr.price(o)
        ms_g, _ = timed(lambda: simr.greeks(o), 5, torch)
        ms_p, _ = timed(lambda: simr.price(o), 5, torch)
        key = "c4_" + ("european" if o["payoff"] < 2 else "american")
        res[key] = {"greeks_ms": ms_g, "price_ms": ms_p, "adjoint_ratio": ms_g / ms_p,
                    "greeks_per_s": 7 / (ms_g * 1e-3)}
        # the extended set (d/dT, and gamma for European options) from the same sweep
        simr.greeks_ext(o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ge = simr.greeks_ext(o)
        torch.cuda.synchronize()
        res[key]["greeks_ext_ms"] = (time.perf_counter() - t0) * 1e3
        res[key]["dprice_dT"] = ge.grads[7]
        res[key]["gamma"] = ge.grads[8] if math.isfinite(ge.grads[8]) else None
    # the C2 risk step (LSM price + 7 adjoint Greeks) under each scheme with adjoint Greeks
    c2 = W.c2_american()
    for name, scheme in (("fte", simr.SCHEME_FTE), ("qe_m", simr.SCHEME_QE_M), ("tg", simr.SCHEME_TG)):
        simr.greeks(c2, scheme)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g = simr.greeks(c2, scheme)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res["c2_risk_" + name] = {"ms": ms, "path_steps_per_s": c2["paths"] * c2["steps"] / (ms * 1e-3),
                                  "price": g.price, "delta": g.grads[0]}
    # the paper's Table 1 shapes as American put batches (LSM), one price_batch call each
    for size in W.TABLE1:
        opts = W.table1_shaped(size)
        simr.price_batch(opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            simr.price_batch(opts)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        ps = W.path_steps(opts)
        res["table1_" + size] = {"options": len(opts), "steps": opts[0]["steps"], "paths": opts[0]["paths"], "ms": ms,
                                 "path_steps_per_s": ps / (ms * 1e-3),
                                 "paper_best_ms_other_hardware": PAPER_TABLE1_BEST_MS[size]}
    return res


if __name__ == "__main__":
    main()
