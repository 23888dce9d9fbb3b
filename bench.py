#!/usr/bin/env python3
"""Benchmark of the Heston Monte Carlo / Longstaff-Schwartz hot path on one MI355X.

One step = one full risk pass of the American put workload (K=110, 131,072
paths x 252 steps, Heston kappa=1.5 theta=0.04 xi=0.3 rho=-0.7 v0=0.04, QE
scheme, Philox seed 7): the forward pass writing the path states, the
Longstaff-Schwartz backward induction (price), and the adjoint sweep (the 7
Greeks), i.e. one simr_greeks call.  `value` is path-steps per second of that
pass (paths x steps / step time).  Inputs are generated in-kernel from the
counter-based RNG, so nothing is transferred before the timed region.

Also reported: the pricing pass alone, the bump-and-revalue cost of the same 7
Greeks (15 pricing passes with common random numbers), per-kernel-group times
from HIP events recorded by the library on the launch stream, the roofline of
the dominant kernel group, and the FP64 CPU oracle timed on a sample of the
same workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--extra]
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

GROUPS = {0: "price", 1: "forward_spill", 2: "lsm_backward", 3: "forward_ckpt", 4: "adjoint", 5: "lsm_gram"}

# HBM bytes per launch of each kernel group on this workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a plain-copy calibration (fetch x2.000, write x1.000).  They describe
# the kernel sources whose digest is given and are reported only while the sources match.
TRAFFIC_SOURCES_DIGEST = "1eb7816434cfb2b5"
TRAFFIC_BYTES = {"forward_spill": 2.643e8, "lsm_gram": 2.641e8 + 1.057e6, "lsm_backward": 2.788e8,
                 "adjoint": 1.802e7}

# VALU instructions per path-step of the forward step loop, counted in the AMD assembly of this
# build (gfx950, -O3): 97, of which 14 transcendental, 15 32x32-bit integer multiplies and 16
# three-input XORs (Philox).  A wave64 VALU instruction occupies a SIMD16 for 4 cycles: issue peak = 1024 SIMDs x
# 2.4 GHz / 4 wave-instructions/s.  (The adjoint sweeps each in-the-money path only up to its
# exercise index, a count the host does not have, so it gets no issue figure.)
VALU_PER_PATH_STEP = {"forward_spill": 97}
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4 * 64  # lane-instructions/s

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
    ap.add_argument("--cpu-sample-paths", type=int, default=131072)
    ap.add_argument("--extra", action="store_true",
                    help="also time the c3 batch, c4 Greeks, c5 risk run and the paper's Table 1 shapes")
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
    L.simr_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]
    L.simr_profile_reset.argtypes = [ctypes.c_void_p]
    if args.basket:
        print(json.dumps({"basket": basket_workloads(simr, W, torch)}))
        return

    opt = W.c2_american()
    P, N = opt["paths"], opt["steps"]
    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            simr.greeks(opt)
            simr.price(opt)
        torch.cuda.synchronize()

        # ---- timed region: K full risk passes -------------------------------------------
        L.simr_profile_reset(ctx)
        L.simr_profile_enable(ctx, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g = simr.greeks(opt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.simr_profile_enable(ctx, 0)
        groups = {}
        for gid, name in GROUPS.items():
            ms, n = ctypes.c_double(), ctypes.c_int64()
            L.simr_profile_read(ctx, gid, ctypes.byref(ms), ctypes.byref(n))
            if n.value:
                groups[name] = {"avg_ms": ms.value / n.value, "launches": n.value}
        L.simr_profile_reset(ctx)
        ms_step = (t1 - t0) * 1e3 / args.steps

        # ---- pricing pass alone, and bump-and-revalue of the 7 Greeks -------------------
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pr = simr.price(opt)
        torch.cuda.synchronize()
        ms_price = (time.perf_counter() - t0) * 1e3 / args.steps
        bumped = [opt]
        for name in simr.GREEK_NAMES:
            h = 1e-4 * abs(opt[name])
            bumped += [dict(opt, **{name: opt[name] + h}), dict(opt, **{name: opt[name] - h})]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for o in bumped:
            simr.price(o)
        torch.cuda.synchronize()
        ms_bump = (time.perf_counter() - t0) * 1e3

        if args.extra:
            out["extra"] = extra_workloads(simr, W, torch)

    path_steps = P * N
    value = path_steps / (ms_step * 1e-3)

    # ---- roofline of every kernel group; the dominant one is `roofline` ----------------------
    def roofline(name, info):
        sec = info["avg_ms"] * 1e-3
        if name in ("lsm_backward", "lsm_gram"):
            work = LSM_BYTES_PER_PATH_DATE * P * (N - 1)
            r = {"bound": "hbm", "achieved": work / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "per_launch_work": f"{LSM_BYTES_PER_PATH_DATE} B x {P} paths x {N - 1} dates"}
        else:
            fl = FLOPS_ADJOINT if name == "adjoint" else FLOPS_FORWARD
            r = {"bound": "alu", "achieved": fl * path_steps / sec / 1e12, "peak": FP32_PEAK_TFLOPS,
                 "unit": "TFLOP/s", "per_launch_work": f"{fl} FLOP x {P} paths x {N} steps"}
            if name == "adjoint":
                r["per_launch_work"] += (" (an upper bound: each path is swept to its exercise index,"
                                         " out-of-the-money paths not at all)")
        r["frac"] = r["achieved"] / r["peak"]
        if name in VALU_PER_PATH_STEP:
            # instruction-issue view: lane-instructions per second against the VALU issue peak
            # (paths that stop early make the adjoint figure an upper bound)
            lane_instr = VALU_PER_PATH_STEP[name] * path_steps / sec
            r["valu_issue_frac"] = lane_instr / VALU_ISSUE_PEAK
            r["valu_per_path_step"] = VALU_PER_PATH_STEP[name]
        r["traffic"] = TRAFFIC_BYTES.get(name) if traffic_current else None
        r["kernel"] = name
        r["avg_ms"] = info["avg_ms"]
        if name == "lsm_backward":
            # the induction is one chip-wide exchange per exercise date: its time per date is the
            # figure that bounds it (a bare 32-block exchange costs about 1.35 us on this GPU)
            r["us_per_date"] = info["avg_ms"] * 1e3 / (N - 1)
        return r

    traffic_current = kernel_sources_digest() == TRAFFIC_SOURCES_DIGEST
    rooflines = {name: roofline(name, info) for name, info in groups.items()}
    dom = max(groups.items(), key=lambda kv: kv[1]["avg_ms"] * kv[1]["launches"])[0]
    roof = rooflines[dom]

    res = {
        "metric": "Heston path-steps/sec and Greeks/sec (adjoint vs bump) at fixed price error",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (in-kernel Philox4x32-10 draws, seeded)",
        "config": {"workload": "american put LSM + 7 adjoint Greeks, 131072 paths x 252 steps, QE",
                   "paths": P, "time_steps": N, "options": 1, "scheme": "QE", "precision": "fp32 paths, fp64 sums/solve"},
        "greeks_per_s": 7.0 / (ms_step * 1e-3),
        "price": g.price, "price_std_err": g.std_err, "greeks": dict(zip(simr.GREEK_NAMES, g.grads)),
        "pricing_pass_ms": ms_price,
        "pricing_path_steps_per_s": path_steps / (ms_price * 1e-3),
        "adjoint_ratio": ms_step / ms_price,
        "bump_ms": ms_bump,
        "bump_ratio": ms_bump / ms_price,
        "greeks_per_s_bump": 7.0 / (ms_bump * 1e-3),
        "kernel_groups": groups,
        "roofline": roof,
        "kernel_rooflines": rooflines,
    }
    res.update(out)
    if not args.no_cpu_baseline:
        res["cpu_baseline"], ref = cpu_baseline(opt, args.cpu_sample_paths)
        err = error_vs_oracle(opt, g, ref)
        if err is not None:
            res["error_vs_oracle"] = err
        res["error_vs_oracle_c1"] = c1_errors(simr, W)
    print(json.dumps(res))


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


def cpu_baseline(opt, sample_paths):
    """The FP64 oracle (LSM price + forward-mode Greeks) on the first `sample_paths`
    paths of the same workload, on all host cores."""
    import oracle
    sample_paths = min(sample_paths, opt["paths"])
    o = oracle.Option(**dict(opt, paths=sample_paths))
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    price, se, grads, grad_se = oracle.greeks(o, nthreads=threads)
    dt = time.perf_counter() - t0
    res = {"value": sample_paths * opt["steps"] / dt, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"LSM price + 7 forward-mode Greeks on {sample_paths} of {opt['paths']} paths x {opt['steps']} steps",
           "seconds": dt}
    return res, (sample_paths, price, se, [float(x) for x in grads], [float(x) for x in grad_se])


def error_vs_oracle(opt, g, ref):
    """The GPU's price and Greeks against the FP64 oracle's on the same paths: the price error in
    units of S0 and of its standard error; each Greek's error relative to its scale
    max(|g|, s_g), s_g the per-path standard deviation.  For an American option each side
    prices with its own in-sample exercise policy (FP32 and FP64 paths), and each side's Greeks
    hold its own policy fixed."""
    paths, price, se, grads, grad_se = ref
    if paths != opt["paths"]:
        return None
    out = {"paths": paths, "price": {"gpu": g.price, "oracle": price, "abs": abs(g.price - price),
                                      "per_S0": abs(g.price - price) / opt["S0"],
                                      "in_std_err": abs(g.price - price) / max(se, 1e-300)}, "greeks": {}}
    for name, a, b, bse in zip(GREEK_NAMES_BENCH, g.grads, grads, grad_se):
        scale = max(abs(b), bse * math.sqrt(paths))
        out["greeks"][name] = {"gpu": a, "oracle": b, "abs": abs(a - b), "rel_to_scale": abs(a - b) / scale}
    return out


# VALU instructions per asset-step of the basket kernel's Greeks step loop (8-asset tile, QE),
# counted in the gfx950 assembly of libsimr.so: 1004 per path-step for 8 assets, the Philox
# blocks, Box-Muller, the correlation triangle, the QE steps and the score sums included.
BASKET_VALU_PER_ASSET_STEP = 1004 / 8


def basket_workloads(simr, W, torch):
    """The 8-asset European call with deltas and cross-gammas (the path kernel timed live by the
    library's HIP events, with its VALU-issue roofline), the 8-asset American put, and the
    paper's Table 1 asset counts as one correlated American basket each."""
    res = {}
    L = simr.library()
    ctx = simr.context()
    eu, am = W.basket_risk()
    for name, bk, fn in (("basket8_european_greeks", eu, simr.basket_greeks),
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
        if name == "basket8_european_greeks" and n.value:
            k_ms = kms.value / n.value
            ach = aps * BASKET_VALU_PER_ASSET_STEP / (k_ms * 1e-3)
            r["roofline"] = {"bound": "valu_issue", "kernel": "basket_path_kernel<QE, 8, Greeks>", "avg_ms": k_ms,
                             "achieved": ach, "peak": VALU_ISSUE_PEAK, "unit": "lane-instructions/s",
                             "frac": ach / VALU_ISSUE_PEAK,
                             "per_launch_work": f"{BASKET_VALU_PER_ASSET_STEP} VALU x {aps} asset-steps"}
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
    opts = W.c3_batch()
    simr.price_batch(opts)  # tunes and captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        simr.price_batch(opts)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    ps = W.path_steps(opts)
    res["c3_batch"] = {"options": len(opts), "path_steps": ps, "ms": ms, "path_steps_per_s": ps / (ms * 1e-3),
                       "options_per_s": len(opts) / (ms * 1e-3), "tile": simr.get_tile()}
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
        simr.greeks(o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        simr.greeks(o)
        torch.cuda.synchronize()
        ms_g = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        simr.price(o)
        torch.cuda.synchronize()
        ms_p = (time.perf_counter() - t0) * 1e3
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
    # c5: 64 American puts, 2^20 paths x 252 steps, LSM price and 7 adjoint Greeks each
    opts = W.c5_risk()
    simr.greeks(opts[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for o in opts:
        simr.greeks(o)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    ps = W.path_steps(opts)
    res["c5_risk"] = {"underlyings": len(opts), "path_steps": ps, "ms": ms, "path_steps_per_s": ps / (ms * 1e-3),
                      "greeks_per_s": 7 * len(opts) / (ms * 1e-3)}
    return res


if __name__ == "__main__":
    main()
