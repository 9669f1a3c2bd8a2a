"""Benchmark of the MRA log-likelihood hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one mra_loglik call that evaluates the MRA log-likelihood of all
covariance-parameter vectors of the batch (64 by default) over the whole tree:
prior on every level, finest-level factors, folds to the root, final sums.
Workload (batched evaluation at n = 2^20): n = 2^20 locations from a seeded
16-component Gaussian mixture on [0,1]^2, RFF Matern-3/2 values, M = 9, J = 4,
r = 64, theta = 8 ranges (0.02..0.3) x 8 nuggets (1e-3..1e-1), FP64.
Inputs (tree, theta) are resident in HBM before the timed region.

Prints one JSON line (rank 0).  The kernel breakdown goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MRA loglik evals/s at n=2^20,r=64 (FP64 MFMA %); exact evals to MLE vs grid"
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 (vector and matrix), dense


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def canonical_flops(leaf_counts, J, M, p):
    """Flops of the A/omega form of the recursion (prior + fold of every
    non-empty region above the finest level, and every non-empty leaf)."""
    import numpy as np
    n = np.asarray(leaf_counts, dtype=np.float64)
    L = M - 1
    total = float(np.sum(2 * n * p * p * L * L + 2 * n * n * L * p + n ** 3 / 3))
    counts = n
    for m in range(M - 1, 0, -1):
        counts = counts.reshape(-1, J).sum(axis=1)
        total += float(np.count_nonzero(counts)) * 2 * p ** 3 * (m * (m - 1) + 1.0 / 3)
    return total


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, theta, budget_s=12.0):
    """The oracle on whole subtrees of the same tree: first single-threaded
    (the subtree is grown until it takes a bounded time), then the same subtree
    on every host core at once (one oracle call per thread, each with its own
    theta; the oracle is plain sequential C, so this is the all-core
    throughput).  Evals/s is extrapolated from the subtree's share of the
    canonical flops."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as o

    fam = o.MATERN
    t0 = time.time()
    ot = o.Tree(cfg["x"], cfg["y"], cfg["z"], J=cfg["J"], r=cfg["r"], M=cfg["M"], domain=cfg["domain"])
    build_s = time.time() - t0
    off = ot.arrays()["leaf_off"]
    counts = np.diff(off)
    J, M, p = cfg["J"], cfg["M"], ot.rhat
    full = canonical_flops(counts, J, M, p)
    spent, done = 0.0, None
    for level in range(min(6, M), 1, -1):
        per = J ** (M - level)                      # leaves under one region of this level
        sub = counts.reshape(-1, per).sum(axis=1)
        target = counts.sum() / len(sub)
        k = int(np.argmin(np.abs(sub - target)))    # a typical region of this level
        f_sub = canonical_flops(counts[k * per:(k + 1) * per], J, M - level + 1, p)
        t1 = time.time()
        o.subtree_du(ot, theta, level, k, fam, cfg["nu"])
        dt = time.time() - t1
        spent += dt
        done = dict(level=level, k=k, n_obs=int(sub[k]), seconds=dt, flops=f_sub)
        log(f"[cpu_baseline] oracle subtree level {level} region {k}: {int(sub[k])} obs, {dt:.2f} s")
        if dt >= 0.35 * budget_s or spent + 4.5 * dt > budget_s:
            break
    est = done["seconds"] * full / done["flops"]
    # the same subtree on every core: distinct theta (ranges spread over the box)
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    ths = [np.array([1.0, b, theta[2]]) for b in np.exp(np.linspace(np.log(0.02), np.log(0.3), ncores))]
    t1 = time.time()
    with ThreadPoolExecutor(max_workers=ncores) as ex:
        list(ex.map(lambda th: o.subtree_du(ot, th, done["level"], done["k"], fam, cfg["nu"]), ths))
    wall = time.time() - t1
    all_rate = ncores / (wall * full / done["flops"])
    log(f"[cpu_baseline] {ncores} threads: {ncores} subtree evaluations in {wall:.2f} s ({cpu_model()})")
    return {
        "value": all_rate,
        "unit": "evals/s",
        "cores": ncores,
        "kind": "oracle",
        "single_core_value": 1.0 / est,
        "cpu": cpu_model(),
        "sample": (f"the subtree of level-{done['level']} region {done['k']} ({done['n_obs']} of "
                   f"{int(counts.sum())} obs): one theta (alpha=1, range={theta[1]:.3g}, nugget={theta[2]:.3g}) "
                   f"single-threaded in {done['seconds']:.2f} s, then {ncores} theta on {ncores} threads at once in "
                   f"{wall:.2f} s; scaled to the whole tree by canonical flops ({done['flops']:.3g} of {full:.3g}); "
                   f"oracle tree build {build_s:.1f} s not counted"),
    }


KERNEL_SOURCES = ["mra_device.h", "mra_chain.hip", "mra_finish.hip", "mra_gram.hip"]


def kernel_source_digest():
    """SHA-256 (16 hex digits) of the log-likelihood kernels' sources."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1905_00141_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name, level):
    """HBM bytes per launch of a kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy kernel), or None when the
    kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != kernel_source_digest():
        return None
    for k in rec.get("kernels", []):
        if k["name"] == name and k["level"] == level:
            return {"bytes_per_launch": k["bytes_per_launch"], "source": rec["summary"]}
    return None


def bench_predict(mra, synth, torch, dev, reps=3):
    """Kriging throughput at 16384 held-out points of the n = 131072, M = 7,
    r = 64 Matern-3/2 workload (device-resident inputs), and its accuracy
    against the field the data were drawn from."""
    import numpy as np
    c = synth.config2(device="cuda")
    t = mra.Tree(c["x"], c["y"], c["z"], J=c["J"], r=c["r"], M=c["M"], domain=c["domain"])
    th = c["theta"][0]
    px = torch.tensor(c["px"], dtype=torch.float64, device=dev)
    py = torch.tensor(c["py"], dtype=torch.float64, device=dev)
    m, v = t.predict(th, px, py, "matern", 1.5)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m, v = t.predict(th, px, py, "matern", 1.5)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    m, v = m.cpu().numpy(), v.cpu().numpy()
    err = m - c["truth"]
    cover = float(np.mean(np.abs(err) <= 1.96 * np.sqrt(v)))
    log(f"[bench] kriging: {len(px)} points in {1000 * sec:.1f} ms, MSPE {np.mean(err ** 2):.4e}")
    return {"workload": f"{c['name']}_pred{len(px)}", "ms": 1000 * sec, "points_per_s": len(px) / sec,
            "mspe": float(np.mean(err ** 2)), "field_var": float(np.var(c["truth"])),
            "coverage_95": cover}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-theta", type=int, default=64, help="must be a square (ranges x nuggets)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scale", type=int, default=0, help="shrink n by 4^scale and M by scale (quick runs)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the execution-plan autotuner on 4 of the theta before timing (about a minute; "
                         "on this workload it keeps the default plan)")
    ap.add_argument("--no-share", action="store_true",
                    help="compute the prior for every theta (no sharing between theta with the same alpha and range)")
    ap.add_argument("--no-mle", action="store_true",
                    help="skip the MLE searches that follow the timed steps by default on the same tree (32x32 "
                         "profiled grid, Nelder-Mead, trust region, the surrogate's sequential design; exact-"
                         "evaluation counts in the JSON line)")
    ap.add_argument("--mle-pretrained", action="store_true",
                    help="also run the surrogate trained once on 2048 exact evaluations as a Nelder-Mead start")
    ap.add_argument("--predict", action="store_true",
                    help="also time kriging on the n = 131072, M = 7 uniform workload at its 16384 held-out points")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, launch a fill and a plain FP64 copy kernel of MIB MiB each: the "
                         "reference that scales hardware byte counters (FETCH_SIZE, WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the library runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    from paper_1905_00141_amd import mra, synth

    nt = int(round(math.sqrt(args.n_theta)))
    n = (1 << 20) >> (2 * args.scale)
    M = 9 - args.scale
    t0 = time.time()
    cfg = synth.config3(device="cuda", n=n, M=M, n_theta=(nt, nt))
    log(f"[bench] data {cfg['name']} generated in {time.time() - t0:.1f} s")
    t0 = time.time()
    tree = mra.Tree(cfg["x"], cfg["y"], cfg["z"], J=cfg["J"], r=cfg["r"], M=cfg["M"], domain=cfg["domain"])
    # the grid is range-major with nt nuggets per range: the prior (alpha and
    # range only) is shared within each group, so whole groups go to a chunk
    if not args.no_share:
        tree.set_chunk_multiple(nt)
    else:
        os.environ["MRA_SHARE_PRIOR"] = "0"
    info = tree.info
    log(f"[bench] tree built in {time.time() - t0:.1f} s: n_used {info['n_used']}, leaves "
        f"{info['leaf_min']}..{info['leaf_max']} obs, {info['n_gram_regions']} Gram-form regions")
    tune = None
    if args.autotune:
        t0 = time.time()
        tune = tree.autotune(cfg["theta"][::16], cfg["family"], cfg["nu"])
        log(f"[bench] autotune in {time.time() - t0:.1f} s: {tune}")
    theta = torch.tensor(cfg["theta"], dtype=torch.float64, device=dev)
    B = theta.shape[0]
    out = torch.empty(B, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)

    # warmup (the first device-pointer call also captures the launch graph),
    # then one step profiled per launch, in steady state, for the breakdown
    for i in range(max(args.warmup, 1)):
        t1 = time.time()
        tree.loglik(theta, cfg["family"], cfg["nu"], out=out, stream=stream)
        stream.synchronize()
        log(f"[bench] warmup step {i} {time.time() - t1:.3f} s")
    ll = out.cpu().numpy()
    assert np.all(np.isfinite(ll)), ll
    mra.profile_enable(True)
    tree.loglik(theta, cfg["family"], cfg["nu"], out=out, stream=stream)
    stream.synchronize()
    mra.profile_enable(False)
    breakdown = mra.profile_read()
    tot_ms = sum(s["ms"] for s in breakdown)
    log(f"[bench] profiled step: {tot_ms:.1f} ms of kernel time")
    for s in sorted(breakdown, key=lambda s: -s["ms"]):
        tf = s["flops"] / (s["ms"] * 1e-3) / 1e12 if s["ms"] > 0 else 0.0
        log(f"[bench] {s['name']:14s} L{s['level']:<2d} launches {s['launches']:4d} "
            f"{s['ms']:10.3f} ms  {100 * s['ms'] / max(tot_ms, 1e-9):5.1f}%  {tf:7.3f} TF/s")
    dom0 = max(breakdown, key=lambda s: s["ms"])

    # one more step with HIP events around the dominant kernel's launches only
    # (its duration for the roofline); profiling disables graph capture
    mra.profile_enable(True, dom0["name"], dom0["level"])
    tree.loglik(theta, cfg["family"], cfg["nu"], out=out, stream=stream)
    stream.synchronize()
    mra.profile_enable(False)
    stats = mra.profile_read()
    # timed region: repeated device-pointer calls on one stream replay the
    # captured graph of the whole launch sequence (captured by the first call)
    tree.loglik(theta, cfg["family"], cfg["nu"], out=out, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        tree.loglik(theta, cfg["family"], cfg["nu"], out=out, stream=stream)
        stream.synchronize()
        log(f"[bench] step {i} done at {time.perf_counter() - t0:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1000.0 * elapsed / args.steps
    value = B * args.steps / elapsed

    dom = stats[0]
    ach = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    roof = {
        "bound": "mfma",
        "kernel": f"{dom['name']} level {dom['level']}",
        "achieved": ach,
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": ach / FP64_PEAK_TFLOPS,
        "traffic": None,
        "launches": dom["launches"],
        "avg_launch_ms": dom["ms"] / dom["launches"],
        "flops_per_launch": dom["flops"] / dom["launches"],
        "share_of_step": dom["ms"] / ms_step,
        "timing": "HIP events on the library's stream around that kernel's launches in a separate profiled step; "
                  "the timed steps replay the captured graph without events",
    }
    try:
        mp = mra.mfma_peak_tflops()
        roof["measured_peak"] = mp
        roof["frac_of_measured_peak"] = ach / mp
        log(f"[bench] measured FP64 matrix-core rate {mp:.1f} TFLOP/s")
    except mra.MraError as e:
        log(f"[bench] matrix-core rate not measured: {e}")
    all_flops = sum(s["flops"] for s in breakdown)
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": cfg["name"], "n": int(n), "n_used": int(info["n_used"]), "M": M, "J": 4, "r": 64,
            "r_hat": int(info["r_hat"]), "n_theta": int(B), "family": "matern", "nu": 1.5,
            "leaf_obs_min": int(info["leaf_min"]), "leaf_obs_max": int(info["leaf_max"]),
            "whole_path_tflops": all_flops / (ms_step * 1e-3) / 1e12,
            "prior_shared": not args.no_share,
            "distinct_alpha_range": int(len({(float(a), float(b)) for a, b, _ in cfg["theta"]})),
            "plan": None if tune is None else {"fold_max": tune["fold_max"], "small_max": tune["small_max"],
                                               "tile": tune["tile"]},
        },
        "roofline": roof,
    }
    # the recursion's own flop count per evaluation (its A / omega form on
    # this tree), times evaluations per second: the prior work that theta
    # with equal alpha and range share is counted once per theta, as the
    # form defines it, so this is an effective rate, not executed work
    canon = canonical_flops(np.diff(tree.arrays()["leaf_off"]), cfg["J"], cfg["M"], int(info["r_hat"]))
    res["canonical"] = {"flops_per_eval": canon, "tflops": value * canon / 1e12,
                        "frac_of_peak": value * canon / 1e12 / FP64_PEAK_TFLOPS}
    if "measured_peak" in roof:
        res["canonical"]["frac_of_measured_peak"] = value * canon / 1e12 / roof["measured_peak"]
    traffic = measured_traffic(dom["name"], dom["level"])
    if traffic is not None:
        roof["traffic"] = traffic["bytes_per_launch"]
        roof["traffic_source"] = traffic["source"]
    if args.copy_calibration:
        nel = (args.copy_calibration << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: fill and copy of {args.copy_calibration} MiB")
    if args.predict:
        res["predict"] = bench_predict(mra, synth, torch, dev)
    if not args.no_mle:
        from paper_1905_00141_amd import mle
        t0 = time.time()
        res["mle"] = mle.run(tree, cfg["family"], cfg["nu"], n_train=2048, train_steps=3000, log=log,
                             pretrained=args.mle_pretrained)
        res["mle"]["wall_s"] = time.time() - t0
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cfg, cfg["theta"][0])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
