#!/usr/bin/env python3
"""Benchmark of randomized TT-rounding (Randomize-then-Orthogonalize) on one
MI355X.

A step is one whole rounding of one synthetic TT already resident in HBM:
sketch drawn on the device (Definition 3.1), partial contractions
(Algorithm 3), left-to-right orthogonalisation sweep (Algorithm 5) and the
right-to-left truncation to the target rank.  Default workload: N=30,
I=100, rank 200, cores N(0,1)/sqrt(I R), sketch rank 60 (target 50 +
oversampling 10), FP64.

Prints one JSON line.  `value` is milliseconds per rounding (lower is
better).  `roofline` covers the dominant kernel, timed with HIP events on its
own launch stream during a second pass over the same steps.  `cpu_baseline`
times the FP64 numpy oracle on the host on whole roundings of the same input.
On the default workload the line also carries the metric's second half:
`mixed_precision` (the BF16-partial-contraction and FP32 modes on the same
input and on its near-low-rank variant, speedups over FP64 and their accuracy
against the FP64 oracle where it is pinned) and `batched` (64 independent
roundings in FP32 in one graph launch against the same roundings one after
another in FP64).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}  # dense MFMA TFLOP/s (MI355X datasheet)
HBM_PEAK_GBS = 8000.0
# arithmetic of each call site per mode (partial contractions / sweep)
SITE_MATH = {"f64": ("f64", "f64"), "f32": ("f32", "f32"), "bf16": ("bf16", "f32")}
STORE_BYTES = {"f64": 8, "f32": 4, "bf16": 4}
METRIC = "ms per randomized TT-rounding + %MFMA peak; mixed-prec vs FP64 at tol"

# HBM bytes per launch of the roofline kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) over this script's default
# run, each scaled by what the same counter reads for a plain 256 MiB device
# copy (FETCH_SIZE counts half of the copy's reads: x 2.0; WRITE_SIZE x 1.0).
# Source: profiles/wfuse_wchain_single_tt_N30_I100_R200_fp64_pmc_traffic.md.
# Valid for the kernel as measured there; anything else reports null.
# The BF16 entry is the mixed-precision form of the same level (wfuse_bf16_kernel),
# profiles/wfuse_bf16_wchain_single_tt_N30_I100_R200_pmc_traffic.md.
MEASURED_TRAFFIC = {("single_tt", "f64", 6): {"read_bytes": 37.06e6, "write_bytes": 1.63e6},
                    ("single_tt", "bf16", 6): {"read_bytes": 17.67e6, "write_bytes": 0.816e6}}

SITE_NAMES = {0: "wchain_z", 1: "wchain_w", 2: "sweep_y", 3: "sweep_m", 4: "sweep_next",
              5: "trunc", 6: "wchain_fused"}
SITE_KERNEL = {0: "gemm_kernel (V(Y_n) W_n, partial contractions)",
               1: "gemm_kernel (H(Z_n) H(Sk_n)^T, partial contractions)",
               2: "gemm_kernel (Z_n W_n, sketch of the sweep)",
               3: "gemm_kernel (Q^T Z_n, projection)",
               4: "gemm_kernel (M_n H(Y_{n+1}), next core)",
               6: "wfuse_kernel (H(V(Y_n) W_n) H(Sk_n)^T in one kernel, partial contractions)"}
WCHAIN_SITES = (0, 1, 6)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def site_launches(site, dims, ell, summand_ranks, fused=False):
    """(M, N, K) of every product from one call site, in launch order.  With
    `fused` the interior levels of the W chain are one kernel each (site 6,
    two products per launch) and sites 0 and 1 keep only the rest."""
    N = len(dims)
    Rs = [1] + [sum(R[n] for R in summand_ranks) for n in range(1, N)] + [1]
    out = []
    if site == 0:  # V(Z_n) = V(Y_n) W_n, n = N-1..2, per summand
        for n in range(N - 1, 1, -1):
            for R in summand_ranks:
                if not fused:
                    out.append((R[n - 1] * dims[n - 1], ell[n], R[n]))
    elif site == 1:  # W_{N-1}, then W_{n-1} = H(Z_n) H(Sk_n)^T
        for R in summand_ranks:
            out.append((R[N - 1], ell[N - 1], dims[N - 1]))
        for n in range(N - 1, 1, -1):
            for R in summand_ranks:
                if not fused:
                    out.append((R[n - 1], ell[n - 1], dims[n - 1] * ell[n]))
    elif site == 6:  # both products of an interior level, per summand
        for n in range(N - 1, 1, -1):
            for R in summand_ranks:
                if fused:
                    out.append((R[n - 1] * dims[n - 1], ell[n], R[n]))
                    out.append((R[n - 1], ell[n - 1], dims[n - 1] * ell[n]))
    elif site == 2:  # Y_n = Z_n W_n
        for n in range(1, N):
            out.append((ell[n - 1] * dims[n - 1], ell[n], Rs[n]))
    elif site == 3:  # M_n = Q^T Z_n
        for n in range(1, N):
            out.append((ell[n], Rs[n], ell[n - 1] * dims[n - 1]))
    elif site == 4:  # M_n H(Y_{n+1}), per summand
        for n in range(1, N):
            for R in summand_ranks:
                out.append((ell[n], dims[n] * R[n + 1], R[n]))
    else:
        raise ValueError(site)
    return out


def site_flops(site, dims, ell, summand_ranks, fused=False):
    """Algorithmic flops (2 M N K per product) of one step's launches."""
    return sum(2.0 * m * n * k
               for m, n, k in site_launches(site, dims, ell, summand_ranks, fused))


def site_bytes(site, dims, ell, summand_ranks, elem, fused=False, sk_elem=None):
    """Algorithmic HBM bytes of one step's launches: each operand read once,
    the result written once (elem bytes per value; the sketch cores of a fused
    level at sk_elem, 2 for the BF16 sketch).  A fused level reads Y_n, W_n and
    Sk_n and writes W_{n-1}; Z_n never reaches memory."""
    sk_elem = elem if sk_elem is None else sk_elem
    if site != 6:
        return sum(float(elem) * (m * k + k * n + m * n)
                   for m, n, k in site_launches(site, dims, ell, summand_ranks, fused))
    pr = site_launches(site, dims, ell, summand_ranks, fused)
    tot = 0.0
    for (m1, n1, k1), (m2, n2, k2) in zip(pr[0::2], pr[1::2]):
        # (R0 I, L1, R1) then (R0, L0, I L1): Y + W + Sk + W_{n-1}
        tot += float(elem) * (m1 * k1 + k1 * n1 + m2 * n2) + float(sk_elem) * k2 * n2
    return tot


def make_workload(name):
    import tt_inputs as G
    if name == "single_tt":
        w = G.workload_single_tt()
        desc = ("single TT, N=30, I=100, rank 200, cores N(0,1)/sqrt(I*R); sketch rank 60 "
                "(target 50 + oversample 10); truncated to rank 50")
        return dict(kind="single", inputs=w["X"], target=w["target"], over=w["oversample"],
                    seed=w["sketch_seed"], desc=desc)
    if name == "single_tt_lowrank":
        w = G.workload_single_tt()
        X = G.near_low_rank_tt(G.INPUT_SEED_BASE + 1, [100] * 30, 40, 160, 1e-6)
        desc = ("near-low-rank single TT, N=30, I=100, X1 rank 40 + 1e-6 X2 rank 160 (formal "
                "200), cores N(0,1)/sqrt(I*r); sketch rank 60; truncated to rank 50")
        return dict(kind="single", inputs=X, target=w["target"], over=w["oversample"],
                    seed=w["sketch_seed"], desc=desc)
    if name == "small_sum":
        w = G.workload_small_sum()
        return dict(kind="single", inputs=w["X"], target=w["target"], over=w["oversample"],
                    seed=w["sketch_seed"],
                    desc="A+A assembled (N=8, I=10, rank 10 -> formal 20), sketch 15, rank 10")
    if name == "gmres_sum":
        w = G.workload_gmres_sum()
        return dict(kind="sum", inputs=w["summands"], coeffs=w["coeffs"], target=w["target"],
                    over=w["oversample"], seed=w["sketch_seed"],
                    desc="sum of 20 TTs, N=16, I=128, rank 20 each (formal 400), "
                         "coefficients U(-1,1), sketch 70, rank 60")
    raise ValueError(name)


def oracle_rel_errs_to_input(wl, outs):
    """cpu_baseline leg: ||X - Y|| / ||Y|| of GPU results X against the input
    Y, through the oracle's orthogonalised difference TT."""
    import numpy as np

    import oracle as O
    return [O.rel_diff([np.asarray(c) for c in o], wl["inputs"]) for o in outs]


def cpu_baseline(wl, gpu_out, budget_s=12.0, max_reps=30):
    """The FP64 oracle on the host's cores: whole roundings of the same input."""
    import numpy as np

    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    times = []
    ref = None
    t_all = time.perf_counter()
    while len(times) < max_reps and (time.perf_counter() - t_all) < budget_s:
        t0 = time.perf_counter()
        if wl["kind"] == "single":
            ref = O.round_rand(wl["inputs"], wl["target"], wl["over"], seed=wl["seed"])
        else:
            ref = O.round_sum_rand(wl["inputs"], wl["coeffs"], wl["target"], wl["over"],
                                   seed=wl["seed"])
        times.append(time.perf_counter() - t0)
    err = O.rel_diff([np.asarray(c) for c in gpu_out], ref)
    med = statistics.median(times) * 1e3
    return dict(value=round(med, 3), unit="ms", cores=int(cores), kind="oracle",
                sample=f"{len(times)} whole roundings of the benchmark input "
                       f"(median; {sum(times):.1f} s of CPU work)"), err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="single_tt",
                    choices=["single_tt", "single_tt_lowrank", "gmres_sum", "small_sum", "batched"])
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--no-f64-compare", action="store_true",
                    help="with --prec f32/bf16: skip timing the FP64 path for the speedup")
    ap.add_argument("--site", type=int, default=None,
                    help="call site whose kernel the roofline covers (default: 0, V(Y_n) W_n)")
    ap.add_argument("--two-sided", action="store_true",
                    help="single-TT FP64 workloads: also time Two-Sided-Randomization "
                         "(Algorithm 6) to the same output ranks and compare the accuracy")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the mixed-precision and batched measurements")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB ten times (the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * 2**20 // 8
        src = torch.randn(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB ten times ({n * 8} bytes read and written each)")
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the rounding "
              "path has no multi-GPU mode", file=sys.stderr)
        sys.exit(2)

    import ctypes

    import torch

    import paper_2110_04393_amd as tt
    from paper_2110_04393_amd import _lib as L

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "batched":
        return bench_batched(args)
    wl = make_workload(args.workload)
    dev = torch.device("cuda:0")

    def build(prec):
        """Plan, device inputs in the mode's storage type, and one step."""
        store = tt.STORAGE[prec]
        if wl["kind"] == "single":
            cores = [torch.from_numpy(c).to(dev).to(store) for c in wl["inputs"]]
            dims = [int(c.shape[1]) for c in cores]
            ranks = [1] + [int(c.shape[2]) for c in cores]
            plan = tt.RoundPlan(dims, ranks, wl["target"], wl["over"], prec, dev)
            sr = [ranks]

            def step():
                return plan.run(cores, seed=wl["seed"])
        else:
            summ = [[torch.from_numpy(c).to(dev).to(store) for c in t] for t in wl["inputs"]]
            dims = [int(c.shape[1]) for c in summ[0]]
            sr = [[1] + [int(c.shape[2]) for c in t] for t in summ]
            plan = tt.RoundPlan(dims, None, wl["target"], wl["over"], prec, dev,
                                summand_ranks=sr)

            def step():
                return plan.run_sum(summ, wl["coeffs"], seed=wl["seed"])
        return plan, step, dims, sr

    def timed(step, steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return ev0.elapsed_time(ev1) / steps, wall * 1e3 / steps

    two_sided_out = None
    plan, step, dims, summand_ranks = build(args.prec)
    ell = plan.sketch_ranks
    ranks = plan.ranks
    log(f"workload: {wl['desc']}; precision {args.prec}; sketch ranks {ell[:4]}..., "
        f"out ranks {plan.out_ranks[:4]}...")
    log(f"workspace {plan.ws_bytes / 2**20:.1f} MiB")

    # ---- timed region: exactly K steps after W warmup steps
    ms_per_step, wall_ms = timed(step, args.steps, args.warmup)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall_ms:.3f})")

    # ---- per-site kernel timing (second pass, same steps, HIP events on the
    # launch stream around every launch of the site)
    wmath, smath = SITE_MATH[args.prec]
    site_ms = {}
    fused = False
    for site in (6, 0, 1, 2, 3, 4):
        L.check(L.lib().tt_timing_start(site, 4096 * args.steps))
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        tot = ctypes.c_double(0)
        cnt = ctypes.c_int32(0)
        L.check(L.lib().tt_timing_stop(ctypes.byref(tot), ctypes.byref(cnt)))
        if site == 6:
            fused = cnt.value > 0
            if not fused:
                continue
        fl = site_flops(site, dims, ell, summand_ranks, fused) * args.steps
        site_ms[site] = (tot.value, cnt.value, fl)
        log(f"site {SITE_NAMES[site]}: {cnt.value // args.steps} launches/step, "
            f"{tot.value / max(cnt.value, 1) * 1e3:.1f} us avg, {tot.value / args.steps:.3f} ms/step, "
            f"{fl / (tot.value * 1e-3) / 1e12 if tot.value else 0:.2f} TFLOP/s")
    # the roofline covers the partial contractions of one interior level (the fused kernel,
    # else V(Y_n) W_n) unless --site says otherwise: the largest contractions of the method
    site = args.site if args.site is not None else (6 if fused else 0)
    tot_ms, cnt, flops = site_ms[site]
    math_dt = wmath if site in WCHAIN_SITES else smath
    per_launch_us = tot_ms / max(cnt, 1) * 1e3
    if math_dt == "bf16":
        # bandwidth-bound at these shapes: algorithmic bytes against HBM peak
        nbytes = site_bytes(site, dims, ell, summand_ranks, STORE_BYTES[args.prec],
                            fused, sk_elem=2) * args.steps
        achieved = nbytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                        bytes_per_step=nbytes / args.steps)
    else:
        achieved = flops / (tot_ms * 1e-3) / 1e12 if tot_ms > 0 else 0.0
        peak = PEAK[math_dt]
        roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                        frac=round(achieved / peak, 4), traffic=None,
                        flops_per_step=flops / args.steps)
    mt = MEASURED_TRAFFIC.get((args.workload, args.prec, site))
    if mt:
        roofline["traffic"] = mt["read_bytes"] + mt["write_bytes"]
        roofline["traffic_detail"] = dict(mt, unit="bytes per launch",
                                          algorithmic_bytes=site_bytes(
                                              site, dims, ell, summand_ranks,
                                              STORE_BYTES[args.prec], fused,
                                              sk_elem=2 if math_dt == "bf16" else None)
                                          / max(cnt // max(args.steps, 1), 1))
    kname = SITE_KERNEL[site]
    if site == 6 and math_dt == "bf16":
        kname = kname.replace("wfuse_kernel", "wfuse_bf16_kernel")
    roofline.update(kernel=kname, math=math_dt,
                    launches_per_step=cnt // max(args.steps, 1),
                    avg_launch_us=round(per_launch_us, 2),
                    site_ms_per_step={SITE_NAMES[k]: round(v[0] / args.steps, 4)
                                      for k, v in site_ms.items()})

    out = [c.detach().double().cpu().numpy() for c in step()]
    torch.cuda.synchronize()

    res = {
        "metric": METRIC,
        "value": round(ms_per_step, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": wl["desc"], "N": len(dims), "I": dims[0],
                   "rank": max(ranks), "sketch_rank": max(ell), "target_rank": wl["target"],
                   "precision": args.prec},
        "roofline": roofline,
    }
    if args.prec != "f64" and not args.no_f64_compare:
        del plan, step
        _, step64, _, _ = build("f64")
        ms64, _ = timed(step64, args.steps, args.warmup)
        out64 = [c.detach().cpu().numpy() for c in step64()]
        torch.cuda.synchronize()
        # core-by-core relative difference to the FP64 GPU result (same gauge)
        num = sum(float(((a - b) ** 2).sum()) for a, b in zip(out, out64))
        den = sum(float((b ** 2).sum()) for b in out64)
        res["f64_gpu"] = {"ms_per_step": round(ms64, 4), "speedup": round(ms64 / ms_per_step, 3),
                          "core_rel_diff": float(f"{math.sqrt(num / max(den, 1e-300)):.3e}")}
        # gauge-free quality of both roundings: the part of ||Y||^2 kept
        terms = ([(1.0, wl["inputs"])] if wl["kind"] == "single"
                 else list(zip(wl["coeffs"], wl["inputs"])))
        k_mode = kept_norm2(tt, out, terms, dev)
        k_64 = kept_norm2(tt, out64, terms, dev)
        res["f64_gpu"].update(kept_norm2=float(f"{k_mode:.6e}"),
                              kept_norm2_f64=float(f"{k_64:.6e}"))
        log(f"FP64 GPU path: {ms64:.3f} ms/step; {args.prec} speedup {ms64 / ms_per_step:.2f}x; "
            f"kept part of ||Y||^2: {args.prec} {k_mode:.6e}, f64 {k_64:.6e}")
    if args.two_sided and wl["kind"] == "single" and args.prec == "f64":
        cores = [torch.from_numpy(c).to(dev) for c in wl["inputs"]]
        tsp = tt.TwoSidedPlan(dims, ranks, wl["target"], dev)
        ms2, _ = timed(lambda: tsp.run(cores, wl["seed"], wl["seed"] + 1), args.steps,
                       args.warmup)
        out2 = [c.detach().cpu().numpy() for c in tsp.run(cores, wl["seed"], wl["seed"] + 1)]
        res["two_sided"] = {"ms_per_step": round(ms2, 4), "left_ranks": max(tsp.left_ranks),
                            "right_ranks": max(tsp.right_ranks)}
        two_sided_out = out2
        log(f"two-sided (Algorithm 6): {ms2:.3f} ms/rounding to ranks {max(tsp.left_ranks)} "
            f"(right sketch {max(tsp.right_ranks)})")
    extra = None
    if (args.workload == "single_tt" and args.prec == "f64" and not args.no_extras):
        extra = metric_second_half(args, tt, wl, timed, build, dev, out, res)
    if not args.no_cpu_baseline:
        cb, err = cpu_baseline(wl, out, budget_s=args.cpu_budget)
        res["cpu_baseline"] = cb
        res["accuracy"] = {"rel_err_vs_fp64_oracle": float(f"{err:.3e}")}
        log(f"oracle: {cb['value']} ms/rounding on {cb['cores']} threads; GPU rel err {err:.2e}")
        if two_sided_out is not None:
            e_ts, e_rto = oracle_rel_errs_to_input(wl, [two_sided_out, out])
            res["two_sided"].update(rel_err_to_input=float(f"{e_ts:.6e}"),
                                    rto_rel_err_to_input=float(f"{e_rto:.6e}"))
            log(f"||X - Y||/||Y||: two-sided {e_ts:.6e}, RtO {e_rto:.6e}")
        if extra is not None:
            extra_accuracy(extra, res)
    print(json.dumps(res), flush=True)


def metric_second_half(args, tt, wl, timed, build, dev, out64, res):
    """The reduced-precision and batched forms next to the plain FP64 one (the
    metric's second half), on the default run: the mixed (BF16 partial
    contractions) and FP32 modes on the same flat-spectrum input, and on its
    near-low-rank variant (X1 rank 40 + 1e-6 X2 rank 160), where their accuracy
    against the FP64 oracle is pinned (computed in the cpu_baseline leg); the
    64-TT batch in FP32 against the same roundings one after another in FP64."""
    import torch
    mp = {}
    terms = [(1.0, wl["inputs"])]
    k64 = kept_norm2(tt, out64, terms, dev)
    ms64 = res["value"]
    lw = make_workload("single_tt_lowrank")
    low_in = lw["inputs"]
    low_out = {}
    for prec in ("bf16", "f32"):
        _, stp, _, _ = build(prec)
        ms, _ = timed(stp, args.steps, args.warmup)
        o = [c.detach().double().cpu().numpy() for c in stp()]
        torch.cuda.synchronize()
        k = kept_norm2(tt, o, terms, dev)
        mp[prec] = {"ms_per_step": round(ms, 4), "speedup_vs_f64": round(ms64 / ms, 3),
                    "flat_kept_norm2_ratio": float(f"{k / k64:.6f}")}
        del stp
        log(f"{prec}: {ms:.3f} ms/rounding ({ms64 / ms:.2f}x over FP64); kept part of ||Y||^2 "
            f"{k / k64:.6f} of the FP64 rounding's")
    # near-low-rank variant: FP64 and both reduced modes
    low_ms = {}
    for prec in ("f64", "bf16", "f32"):
        store = tt.STORAGE[prec]
        cores = [torch.from_numpy(c).to(dev).to(store) for c in low_in]
        dims = [int(c.shape[1]) for c in cores]
        ranks = [1] + [int(c.shape[2]) for c in cores]
        plan = tt.RoundPlan(dims, ranks, lw["target"], lw["over"], prec, dev)
        stp = (lambda p=plan, c=cores: p.run(c, seed=lw["seed"]))
        ms, _ = timed(stp, max(3, args.steps // 2), 1)
        low_ms[prec] = ms
        low_out[prec] = [c.detach().double().cpu().numpy() for c in stp()]
        torch.cuda.synchronize()
        del plan, cores
    for prec in ("bf16", "f32"):
        mp[prec]["near_low_rank"] = {"ms_per_step": round(low_ms[prec], 4),
                                     "ms_per_step_f64": round(low_ms["f64"], 4),
                                     "speedup_vs_f64": round(low_ms["f64"] / low_ms[prec], 3)}
    log(f"near-low-rank variant: f64 {low_ms['f64']:.3f}, bf16 {low_ms['bf16']:.3f}, "
        f"f32 {low_ms['f32']:.3f} ms/rounding")
    res["mixed_precision"] = mp
    res["deterministic_comparator"] = deterministic_comparator(args, tt, timed, dev)
    # the batched form
    bres, b_outs, b_specs, b_inputs = run_batched(args, "f32", with_f64=True)
    res["batched"] = bres
    return dict(low_in=low_in, low_out=low_out, lw=lw, b_outs=b_outs, b_specs=b_specs,
                b_inputs=b_inputs)


def deterministic_comparator(args, tt, timed, dev):
    """Deterministic rounding (Algorithms 1 and 2, tt_round_svd) next to RtO on
    the largest bond rank the comparator takes: N=30, I=100, rank 96, cores
    N(0,1)/sqrt(I*R), rounded to rank 50 (RtO: sketch rank 60)."""
    import torch

    import tt_inputs as G
    N, I, R = 30, 100, 96
    dims, ranks = G.uniform_tt_shape(N, I, R)
    Y = G.random_tt(G.INPUT_SEED_BASE + 7, dims, ranks, scale="nominal")
    cores = [torch.from_numpy(c).to(dev) for c in Y]
    plan = tt.RoundPlan(dims, ranks, 50, 10, "f64", dev)
    steps = max(3, args.steps // 4)
    ms_rand, _ = timed(lambda: plan.run(cores, seed=2001), steps, 1)
    ms_svd, _ = timed(lambda: tt.round_svd(cores, eps0=0.0, max_rank=50), steps, 1)
    log(f"deterministic comparator at N={N} I={I} R={R} -> 50: tt_round_svd {ms_svd:.3f} ms, "
        f"RtO {ms_rand:.3f} ms ({ms_svd / ms_rand:.2f}x)")
    return {"config": f"N={N}, I={I}, rank {R} -> 50 (RtO sketch 60)",
            "ms_round_svd": round(ms_svd, 4), "ms_round_rand": round(ms_rand, 4),
            "ratio_svd_over_rand": round(ms_svd / ms_rand, 3)}


def extra_accuracy(extra, res):
    """cpu_baseline leg: accuracy of the reduced-precision and batched forms
    against the FP64 oracle (given the same FP32-rounded inputs and sketch
    values), on inputs where it is pinned."""
    import numpy as np

    import oracle as O
    lw = extra["lw"]
    X32 = [O.round_f32(c) for c in extra["low_in"]]
    dims, ranks = O.dims_of(X32), O.ranks_of(X32)
    ell, _ = O.plan_ranks(dims, ranks, lw["target"], lw["over"])
    sk = O.make_sketch(lw["seed"], dims, ell)
    for prec in ("bf16", "f32"):
        skp = [O.round_bf16(c) if prec == "bf16" else O.round_f32(c) for c in sk]
        ref = O.round_rand(X32, lw["target"], lw["over"], sketch=skp)
        err = O.rel_diff(extra["low_out"][prec], ref)
        res["mixed_precision"][prec]["near_low_rank"]["rel_err_vs_fp64_oracle"] = \
            float(f"{err:.3e}")
        log(f"{prec} near-low-rank: rel err vs the FP64 oracle {err:.3e}")
    ref64 = O.round_rand(extra["low_in"], lw["target"], lw["over"], seed=lw["seed"])
    e64 = O.rel_diff(extra["low_out"]["f64"], ref64)
    res["mixed_precision"]["f64_near_low_rank_rel_err_vs_oracle"] = float(f"{e64:.3e}")
    # batch: the four smallest TTs (FP32-rounded inputs and sketch)
    specs, outs, inputs = extra["b_specs"], extra["b_outs"], extra["b_inputs"]
    size = [s["N"] * s["I"] * s["R"] ** 2 for s in specs]
    worst = 0.0
    for b in np.argsort(size)[:4]:
        s = specs[b]
        X = [O.round_f32(c) for c in inputs[b]]
        d, r = O.dims_of(X), O.ranks_of(X)
        el, _ = O.plan_ranks(d, r, s["target"], s["oversample"])
        skb = [O.round_f32(c) for c in O.make_sketch(s["sketch_seed"], d, el)]
        ref = O.round_rand(X, s["target"], s["oversample"], sketch=skb)
        worst = max(worst, O.rel_diff(outs[b], ref))
    res["batched"]["rel_err_vs_fp64_oracle_4_smallest"] = float(f"{worst:.3e}")
    log(f"batched FP32: rel err vs the FP64 oracle on the four smallest TTs {worst:.3e}")


def tt_inner(tt, A, B):
    """<A, B> of two TTs (device FP64 cores, same mode sizes) from the
    library's partial contractions: W_1 = H(A_{2:N}) H(B_{2:N})^T, then the
    first cores."""
    import torch
    if len(A) == 1:
        return float((A[0] * B[0]).sum())
    W = tt.partial_contractions_rl(A, B, prec="f64")
    torch.cuda.synchronize()
    return float(((A[0][0] @ W[1]) * B[0][0]).sum())


def kept_norm2(tt, X, terms, dev):
    """(2 <X, Y> - <X, X>) / <Y, Y> for Y = sum_j c_j Y_j (numpy cores): the
    part of ||Y||^2 the rounding X keeps (gauge-free; when X projects Y it is
    <X, X> / <Y, Y>, and no large terms cancel).  TT inner products through
    the library's FP64 partial contractions."""
    import torch
    D = lambda cores: [torch.from_numpy(c).to(dev).double() for c in cores]
    Xd = D(X)
    Ys = [(c, D(Y)) for c, Y in terms]
    xx = tt_inner(tt, Xd, Xd)
    xy = sum(c * tt_inner(tt, Xd, Y) for c, Y in Ys)
    yy = sum(ci * cj * tt_inner(tt, Yi, Yj) for ci, Yi in Ys for cj, Yj in Ys)
    return (2.0 * xy - xx) / yy


def batch_flops(spec, ell):
    """RtO flops of one TT of the batch (2 M N K per product, same shapes as
    the single-TT path: partial contractions, sweep products, truncation)."""
    N, I, R = spec["N"], spec["I"], spec["R"]
    dims = [I] * N
    ranks = [1] + [R] * (N - 1) + [1]
    f = sum(site_flops(k, dims, ell, [ranks]) for k in range(5))
    return f


def run_batched(args, prec, with_f64=True):
    """64 independent roundings (N ~ U{8..24}, I in {16..256}, R ~ U{8..128},
    target R//2) in one graph launch, timed over args.steps runs; the same
    roundings one after another through the single-TT path (in `prec`, and in
    FP64: the plain form).  Returns (summary, outputs as numpy, specs, numpy
    inputs)."""
    import torch

    import paper_2110_04393_amd as tt
    import tt_inputs as G
    dt = tt.STORAGE[prec]
    specs = G.batched_specs(0, 64)
    tts_np, tts = [], []
    for s in specs:
        dims, ranks = G.uniform_tt_shape(s["N"], s["I"], s["R"])
        X = G.random_tt(s["input_seed"], dims, ranks, scale="nominal")
        tts_np.append(X)
        tts.append([torch.from_numpy(c).to("cuda:0").to(dt) for c in X])
    targets = [s["target"] for s in specs]
    overs = [s["oversample"] for s in specs]
    seeds = [s["sketch_seed"] for s in specs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        bp = tt.BatchPlan(tts, targets, overs, seeds, prec=prec, graph=True, autotune=True,
                          stream=stream)
        torch.cuda.synchronize()
        create_s = time.perf_counter() - t0
        info = bp.info()
        log(f"batch plan: {info}, workspace {bp.ws_bytes / 2**20:.0f} MiB, "
            f"created in {create_s:.2f} s")
        for _ in range(args.warmup):
            bp.run(stream)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            bp.run(stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        batch_ms = ev0.elapsed_time(ev1) / args.steps
        outs = [[c.detach().double().cpu().numpy() for c in o] for o in bp.run(stream)]
        torch.cuda.synchronize()

        def sequential(ts, pr):
            plans = [tt.RoundPlan([int(c.shape[1]) for c in t], [1] + [int(c.shape[2]) for c in t],
                                  tr, ov, pr, "cuda:0") for t, tr, ov in zip(ts, targets, overs)]
            for p, t, sd in zip(plans, ts, seeds):
                p.run(t, seed=sd, stream=stream)
            torch.cuda.synchronize()
            ev0.record(stream)
            for p, t, sd in zip(plans, ts, seeds):
                p.run(t, seed=sd, stream=stream)
            ev1.record(stream)
            torch.cuda.synchronize()
            return ev0.elapsed_time(ev1), plans

        seq_ms, plans = sequential(tts, prec)
        seq64_ms = None
        if with_f64 and prec != "f64":
            seq64_ms, _ = sequential([[c.double() for c in t] for t in tts], "f64")
    flops = 0.0
    for s, p in zip(specs, plans):
        flops += batch_flops(s, p.sketch_ranks)
    achieved = flops / (batch_ms * 1e-3) / 1e12
    peak = PEAK[prec if prec != "bf16" else "f32"]
    log(f"batch of 64: {batch_ms:.3f} ms ({batch_ms / 64:.4f} ms per rounding); "
        f"sequential single-TT path {seq_ms:.3f} ms"
        + (f", FP64 sequential {seq64_ms:.3f} ms" if seq64_ms else "")
        + f"; {achieved:.2f} TFLOP/s")
    summary = {"precision": prec, "ms_per_batch": round(batch_ms, 4),
               "ms_per_rounding": round(batch_ms / 64, 5),
               "sequential_single_tt_ms": round(seq_ms, 3),
               "speedup_vs_sequential": round(seq_ms / batch_ms, 2),
               "sequential_single_tt_f64_ms": round(seq64_ms, 3) if seq64_ms else None,
               "speedup_vs_f64_sequential": round(seq64_ms / batch_ms, 2) if seq64_ms else None,
               "plan_create_s": round(create_s, 2), "tflops": round(achieved, 3),
               "flops_per_batch": flops, "peak_tflops": peak, **info}
    return summary, outs, specs, tts_np


def bench_batched(args):
    """The batched workload as the benchmark line (FP32 unless --prec f64)."""
    prec = args.prec if args.prec != "f64" else "f32"
    if args.prec == "f64" and "--prec" in sys.argv:
        prec = "f64"
    summary, outs, specs, tts_np = run_batched(args, prec, with_f64=True)
    batch_ms = summary["ms_per_batch"]
    res = {
        "metric": METRIC, "value": round(batch_ms / 64, 5), "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(batch_ms, 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": "64 independent roundings, N~U{8..24}, I in {16,32,64,128,256}, "
                               "R~U{8..128}, target R//2, oversample min(10,R-target); one "
                               "hipGraph launch per batch, autotuned GEMM tiles",
                   "batch": 64, "precision": prec},
        "batch": summary,
        "roofline": {"bound": "mfma", "achieved": summary["tflops"],
                     "peak": summary["peak_tflops"], "unit": "TFLOP/s",
                     "frac": round(summary["tflops"] / summary["peak_tflops"], 4),
                     "traffic": None, "kernel": "whole batched run (all grouped launches)",
                     "flops_per_step": summary["flops_per_batch"]},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            cores = os.cpu_count() or 1
        t_all = time.perf_counter()
        done = 0
        while done < 64 and time.perf_counter() - t_all < args.cpu_budget:
            s = specs[done]
            O.round_rand(tts_np[done], s["target"], s["oversample"], seed=s["sketch_seed"])
            done += 1
        el = time.perf_counter() - t_all
        res["cpu_baseline"] = {"value": round(el * 1e3 / max(done, 1), 3), "unit": "ms",
                               "cores": int(cores), "kind": "oracle",
                               "sample": f"TTs 0..{done - 1} of the batch in order ({el:.1f} s), "
                                         "ms per rounding"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
