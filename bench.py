"""Benchmark: forest-closeness estimation on one MI355X.

Workload (one "step" = the whole hot path once): Barabasi-Albert graph with
n = 200,000 and m = 5 (999,985 edges), alpha = 1, 4096 uniform spanning trees
of G* rooted at u* sampled with Wilson's algorithm, aggregated into the
estimated diagonal of Omega = (alpha L + I)^{-1}, forest farness and forest
closeness of every vertex.  The CSR is resident in device memory before the
timed region.  Prints one JSON line.

value = trees per second over the timed steps (whole job, one GPU).
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

WORKLOAD = {"workload": "ba_n200000_m5_alpha1_trees4096", "graph": "barabasi_albert",
            "n": 200_000, "m_per_vertex": 5, "alpha": 1.0, "trees": 4096, "seed": 0}

# Algorithmic bytes of Wilson's algorithm per unit of work (what the method
# itself must move with a packed 8-byte per-vertex state word):
#   walk step   : row offsets of v (8) + neighbour id (4) + read state of the
#                 next vertex (8) + write state of v (8)            = 28 B
#   retrace     : read + write the state word of each tree vertex    = 16 B
#   start scan  : read the state word of each start candidate        =  8 B
#   root        : read-modify-write of R[v] (4 + 4)                  =  8 B
BYTES_STEP, BYTES_RETRACE, BYTES_SCAN, BYTES_ROOT = 28, 16, 8, 8
# weighted graphs: a walk step also reads the weighted degree of v and the
# running weight sum of the entry it takes (8 + 8)                  = 44 B
BYTES_STEP_W = 44
HBM_PEAK_GBS = 8000.0

CSRC = os.path.join(ROOT, "paper_2101_06192_amd", "csrc")


def _kernel_hash(sampler: str) -> str:
    """Hash of the sampling kernel's source and the device header it includes."""
    h = hashlib.sha256()
    for name in (f"{sampler}.hip", "fc_device.hpp", "fc_kernels.hpp"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(sampler: str, workload: str = "ba200k"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{sampler}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != _kernel_hash(sampler):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_range(args):
    g, t0, count = args
    import oracle
    t = time.perf_counter()
    r = oracle.sample(g, 1.0, 0, t0, count)
    return time.perf_counter() - t, r.R


def cpu_baseline(g, trees: int) -> dict:
    """The C oracle on the host: one core on trees [0, trees), then every
    core of the host's share as independent processes on disjoint tree
    ranges (integer sums, so the ranges add up exactly).  Runs before the
    process touches the GPU: the workers are forked."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    _oracle_range((g, 0, trees))
    one = time.perf_counter() - t0
    cores = max(1, min(16, os.cpu_count() or 1))
    per = max(1, trees // 2)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_range, [(g, trees + i * per, per) for i in range(cores)])
    wall = time.perf_counter() - t0
    return {"value": cores * per / wall, "unit": "trees/s", "cores": cores, "kind": "oracle",
            "sample": f"trees {trees}..{trees + cores * per - 1} of the same workload as {cores} "
                      f"single-threaded C oracle processes of {per} trees each (Algorithm 3 "
                      f"literal), {wall:.1f} s wall",
            "single_core": {"value": trees / one, "unit": "trees/s",
                            "sample": f"trees 0..{trees - 1}, one process, {one:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-trees", type=int, default=640,
                    help="trees the CPU oracle samples for the baseline (0 = skip)")
    ap.add_argument("--no-eps", action="store_true", help="skip the time-to-eps=0.1 leg")
    ap.add_argument("--sampler", default="auto", choices=["auto", "lane", "coop", "lds", "hyb"])
    ap.add_argument("--config", default="ba200k",
                    choices=["ba200k", "ba200k_w", "er1000", "grid1000", "rmat_batch", "rmat22",
                             "solve", "rank", "group"],
                    help="workload; the default is the headline configuration")
    ap.add_argument("--lds-repop", type=int, default=None, choices=[0, 1, 2],
                    help="LDS sampler: pop re-formed 2-cycles within their round "
                         "(0 never, 1 weighted graphs, 2 always: the library default)")
    ap.add_argument("--coop-repop", type=int, default=None, choices=[0, 1, 2],
                    help="global-counter sampler: the same option (coop_repop)")
    ap.add_argument("--phase-timing", action="store_true",
                    help="report per-phase times of the workgroup sampler (adds clock reads)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.calibrate_copy, "bytes_read": x.numel() * 4,
                          "bytes_written": y.numel() * 4}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the sampler shards by tree id with no exchange "
              "beyond one integer all-reduce, and this build runs on a single MI355X.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2101_06192_amd as fc
    import inputs

    dev = torch.device("cuda:0")
    if args.lds_repop is not None:
        fc.set_option("lds_repop", args.lds_repop, dev)
    if args.coop_repop is not None:
        fc.set_option("coop_repop", args.coop_repop, dev)
    if args.config != "ba200k":
        other_config(args, fc, inputs, dev)
        return
    g = inputs.barabasi_albert(WORKLOAD["n"], WORKLOAD["m_per_vertex"], WORKLOAD["seed"])
    # the CPU leg first: its worker processes are forked before the GPU is used
    cpu = cpu_baseline(g, args.cpu_trees) if args.cpu_trees > 0 else None
    dg = fc.to_device(g, dev)
    trees = WORKLOAD["trees"]
    alpha = WORKLOAD["alpha"]
    if args.phase_timing:
        fc.set_option("phase_timing", 1, dev)
    torch.cuda.synchronize()

    def step():
        return fc.farness(dg, alpha=alpha, seed=WORKLOAD["seed"], tau=trees, device=dev,
                          as_torch=True, sampler=args.sampler)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
        stats.append(out["stats"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = trees / (elapsed / args.steps)

    walk_steps = stats[-1]["walk_steps"]
    roots = stats[-1]["roots"]
    ms_kernel = float(np.mean([s["ms_sample"] for s in stats]))
    n = g.n
    alg_bytes = (BYTES_STEP * walk_steps + (BYTES_RETRACE + BYTES_SCAN) * n * trees
                 + BYTES_ROOT * roots)
    achieved = alg_bytes / (ms_kernel / 1000.0) / 1e9
    sampler = stats[-1]["sampler"]
    traffic = _traffic(sampler)
    # the sampling path's kernels: the LDS sampler may run a first-arrow
    # pre-draw kernel ahead of the tree kernel (both inside ms_sample)
    ms_pre = float(np.mean([s.get("ms_predraw", 0.0) for s in stats]))
    kernels = {f"{sampler}_kernel": ms_kernel - ms_pre}
    if ms_pre > 0.0:
        kernels = {"lds_predraw_kernel": ms_pre, **kernels}

    eps_leg = None
    if not args.no_eps:
        torch.cuda.synchronize()
        te = time.perf_counter()
        o = fc.diag_estimate(dg, alpha=alpha, eps=0.1, delta=0.1, seed=0, device=dev,
                             as_torch=True, sampler=args.sampler)
        torch.cuda.synchronize()
        eps_leg = {"tau": o["tau"], "ms": 1000.0 * (time.perf_counter() - te)}


    # the random-access ceiling the sampler runs against: independent random
    # 4-byte loads and atomic adds over a 4 GiB footprint (far beyond caches)
    ceiling = None
    if not args.no_eps:
        ceiling = {"footprint_bytes": 4 << 30,
                   "random_loads_per_s": fc.probe_random_access(4 << 30, False, dev),
                   "random_atomics_per_s": fc.probe_random_access(4 << 30, True, dev)}

    line = {
        "metric": "USTs/s and walk steps/s (GB/s vs roofline); time to eps=0.1 diag(Omega)",
        "value": value,
        "unit": "trees/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": WORKLOAD,
        "walk_steps_per_s": walk_steps / (ms_per_step / 1000.0),
        "walk_steps_per_tree": walk_steps / trees,
        "trees_in_flight": stats[-1]["trees_in_flight"],
        "time_to_eps0.1_diag": eps_leg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": " + ".join(kernels), "kernel_ms": ms_kernel,
                     "kernels_ms": kernels,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "random_access_ceiling": ceiling},
        "cpu_baseline": cpu,
    }
    if ceiling:
        # the line model of sequential Wilson walks: 3 random lines per walk step
        # plus one line per 8 vertices for the start scan, against the measured
        # rate of independent random loads over 4 GiB
        lines = 3.0 * walk_steps + n * trees / 8.0
        rate = lines / (ms_kernel / 1000.0)
        line["roofline"]["random_gather_model"] = {
            "lines_per_launch": lines, "lines_per_s": rate,
            "ceiling_loads_per_s": ceiling["random_loads_per_s"],
            "frac": rate / ceiling["random_loads_per_s"]}
    if args.phase_timing:
        line["phase_ms_per_workgroup"] = _phases(stats[-1])
    print(json.dumps(line), flush=True)


def _phases(st):
    """Per-phase wall time per workgroup of a workgroup sampler's call."""
    if st["sampler"] == "wilson_lds":
        names = ["first_arrows", "count_and_level0", "peel_wide", "peel_tail",
                 "sweep_and_split", "cycle_scan", "cycles", "output"]
    else:
        names = ["first_arrows", "in_arrows", "peel_level0", "peel_levels", "sweep", "redraw",
                 "output"]
    return dict(zip(names, st["phase_ms"]))


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def other_config(args, fc, inputs, dev):
    """The non-headline workloads (same sampler, other graph families)."""
    import numpy as np
    res = {"metric": "trees/s", "n_gpus": 1, "data": "synthetic", "dtype": "u32",
           "higher_is_better": True, "steps": args.steps, "warmup": args.warmup}
    if args.phase_timing:
        fc.set_option("phase_timing", 1, dev)
    if args.config in ("er1000", "rmat22"):
        if args.config == "er1000":
            g, alpha, trees, name = inputs.erdos_renyi(1000, 0.01, 0), 1.0, 2000, "er_n1000_p0.01_trees2000"
        else:
            g, alpha, trees, name = inputs.rmat(1 << 22, 8, 0), 1.0, 1024, "rmat_n4194304_ef8_trees1024"
        dg = fc.to_device(g, dev)
        per = {}
        samplers = ["lane", "coop", "lds"] if args.config == "er1000" else ["coop", "hyb"]
        for smp in samplers:
            dt, out = _timed(lambda: fc.farness(dg, alpha=alpha, tau=trees, device=dev, as_torch=True,
                                                sampler=smp), args.steps, args.warmup)
            per[smp] = {"trees_per_s": trees / dt, "ms_per_step": 1000 * dt,
                        "walk_steps_per_s": out["stats"]["walk_steps"] / dt,
                        "kernel_ms": out["stats"]["ms_sample"]}
            if args.phase_timing:
                per[smp]["phase_ms"] = out["stats"]["phase_ms"]
        best = max(per, key=lambda k: per[k]["trees_per_s"])
        res.update({"value": per[best]["trees_per_s"], "unit": "trees/s",
                    "config": {"workload": name, "n": g.n, "m": g.m, "alpha": alpha, "trees": trees},
                    "samplers": per})
        if args.config == "rmat22":
            te = time.perf_counter()
            o = fc.diag_estimate(dg, alpha=alpha, eps=0.1, delta=0.1, device=dev, as_torch=True)
            import torch
            torch.cuda.synchronize()
            res["time_to_eps0.1_diag"] = {"tau": o["tau"], "ms": 1000 * (time.perf_counter() - te)}
    elif args.config == "ba200k_w":
        # the headline graph with seeded log-uniform edge weights in [0.1, 10)
        g = inputs.with_weights(inputs.barabasi_albert(200_000, 5, 0), 0)
        dg = fc.to_device(g, dev)
        trees, alpha = 4096, 1.0
        stats = []

        def step():
            out = fc.farness(dg, alpha=alpha, tau=trees, device=dev, as_torch=True,
                             sampler=args.sampler)
            stats.append(out["stats"])
            return out
        dt, out = _timed(step, args.steps, args.warmup)
        st = out["stats"]
        timed = stats[args.warmup:]
        ms_kernel = float(np.mean([s["ms_sample"] for s in timed]))
        ms_pre = float(np.mean([s.get("ms_predraw", 0.0) for s in timed]))
        alg = (BYTES_STEP_W * st["walk_steps"] + (BYTES_RETRACE + BYTES_SCAN) * g.n * trees
               + BYTES_ROOT * st["roots"])
        ach = alg / (ms_kernel / 1000.0) / 1e9
        eps_leg = None
        if not args.no_eps:
            import torch
            torch.cuda.synchronize()
            te = time.perf_counter()
            o = fc.diag_estimate(dg, alpha=alpha, eps=0.1, delta=0.1, device=dev, as_torch=True,
                                 sampler=args.sampler)
            torch.cuda.synchronize()
            eps_leg = {"tau": o["tau"], "ms": 1000 * (time.perf_counter() - te)}
        res.update({"value": trees / dt, "unit": "trees/s", "ms_per_step": 1000 * dt,
                    "config": {"workload": "ba_n200000_m5_logw0.1_10_alpha1_trees4096", "n": g.n,
                               "m": g.m, "alpha": alpha, "trees": trees},
                    "sampler": st["sampler"], "walk_steps_per_tree": st["walk_steps"] / trees,
                    "walk_steps_per_s": st["walk_steps"] / dt,
                    "time_to_eps0.1_diag": eps_leg,
                    "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                 "traffic": _traffic(st["sampler"], "ba200k_w"),
                                 "kernel_ms": ms_kernel,
                                 "kernels_ms": {"lds_predraw_kernel": ms_pre,
                                                f"{st['sampler']}_kernel": ms_kernel - ms_pre},
                                 "algorithmic_bytes_per_launch": alg}})
        if args.phase_timing:
            res["phase_ms_per_workgroup"] = _phases(st)
    elif args.config == "rank":
        # ranking output: the headline graph's closeness ranking and Kendall's tau-b
        # at n = 200000; the KT of eps-estimates against a CG ground truth of every
        # Omega_vv on BA(20000, 5)
        import torch
        g = inputs.barabasi_albert(200_000, 5, 0)
        dg = fc.to_device(g, dev)
        est = fc.farness(dg, alpha=1.0, eps=0.1, delta=0.1, device=dev, as_torch=True)
        clo, diag = est["closeness"], est["diag"]
        dt_rank, _ = _timed(lambda: fc.rank(clo, descending=True, device=dev, as_torch=True),
                            args.steps, args.warmup)
        other = fc.farness(dg, alpha=1.0, eps=0.1, delta=0.1, seed=1, device=dev, as_torch=True)
        dt_kt, kt = _timed(lambda: fc.kendall_tau(diag, other["diag"], device=dev), args.steps,
                           args.warmup)
        fc.set_option("kendall_pairs", 1, dev)
        dt_pairs, kt_pairs = _timed(lambda: fc.kendall_tau(diag, other["diag"], device=dev),
                                    args.steps, args.warmup)
        fc.set_option("kendall_pairs", 0, dev)
        assert kt_pairs["counts"] == kt["counts"]
        n = g.n
        pairs = n * (n - 1) // 2
        # the all-pairs kernel is VALU-bound: 10 instructions per pair (two
        # differences, two v_med3_i32 signs, a product, three multiply-adds, loop
        # share) against 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz int32 lane-ops
        valu_peak = 256 * 4 * 16 * 2.4e9
        gs = inputs.barabasi_albert(20_000, 5, 0)
        dgs = fc.to_device(gs, dev)
        t0 = time.perf_counter()
        truth = torch.empty(gs.n, dtype=torch.float64, device=dev)
        for c0 in range(0, gs.n, 64):
            k = min(64, gs.n - c0)
            B = torch.zeros(gs.n, k, dtype=torch.float64, device=dev)
            B[torch.arange(c0, c0 + k, device=dev), torch.arange(k, device=dev)] = 1.0
            X = fc.solve(dgs, 1.0, B, rtol=1e-9, precision="fp32_refined", device=dev,
                         trusted=True, as_torch=True)["X"]
            truth[c0:c0 + k] = X[torch.arange(c0, c0 + k, device=dev), torch.arange(k, device=dev)]
        torch.cuda.synchronize()
        truth_s = time.perf_counter() - t0
        quality = {}
        for eps in (0.1, 0.3):
            e = fc.diag_estimate(dgs, alpha=1.0, eps=eps, delta=0.1, device=dev, as_torch=True)
            r = fc.kendall_tau(e["diag"], truth, device=dev)
            quality[str(eps)] = {"tau": e["tau"], "kendall_tau_b": r["tau_b"],
                                 "max_abs_err": float((e["diag"] - truth).abs().max())}
        res.update({"metric": "ranking: fc_rank and fc_kendall_tau time at n = 200000; KT vs CG",
                    "value": 1000 * dt_kt, "unit": "ms (fc_kendall_tau, n = 200000)",
                    "higher_is_better": False,
                    "config": {"workload": "ba_n200000_m5_alpha1_eps0.1_rank_kendall", "n": n,
                               "kt_graph": "ba_n20000_m5_alpha1"},
                    "rank_ms": 1000 * dt_rank,
                    "kendall_ms": 1000 * dt_kt,
                    "kendall_all_pairs": {"ms": 1000 * dt_pairs, "pairs_per_s": pairs / dt_pairs,
                                          "roofline": {"bound": "alu",
                                                       "achieved": 10 * pairs / dt_pairs / 1e12,
                                                       "peak": valu_peak / 1e12,
                                                       "unit": "T int32 lane-ops/s",
                                                       "frac": 10 * pairs / dt_pairs / valu_peak}},
                    "kendall_two_estimates_tau_b": kt["tau_b"],
                    "ground_truth_s": truth_s, "kt_vs_cg": quality})
    elif args.config == "group":
        # group forest closeness (Algorithm 2): one dense inverse (k = 1 times it
        # alone), then one downdate pass over the n x n matrix per greedy step
        g = inputs.barabasi_albert(20_000, 5, 0)
        dg = fc.to_device(g, dev)
        k = 50
        t1, _ = _timed(lambda: fc.group_closeness(dg, 1.0, 1, device=dev, trusted=True), args.steps,
                       args.warmup)
        tk, out = _timed(lambda: fc.group_closeness(dg, 1.0, k, device=dev, trusted=True),
                         args.steps, args.warmup)
        N = (g.n + 63) // 64 * 64
        flops = 2.0 * N ** 3  # blocked Gauss-Jordan: n^3 multiply-adds
        step_s = (tk - t1) / (k - 1)
        step_bytes = 16.0 * g.n * g.n  # read and write the n x n binary64 matrix
        res.update({"metric": "greedy group forest closeness time (Algorithm 2)", "value": 1000 * tk,
                    "unit": "ms", "higher_is_better": False,
                    "config": {"workload": "ba_n20000_m5_alpha1_group_k50", "n": g.n, "m": g.m,
                               "k": k},
                    "group_head": out["group"][:8], "farness_first_last": [out["farness"][0],
                                                                           out["farness"][-1]],
                    "inverse": {"ms": 1000 * t1,
                                "roofline": {"bound": "mfma", "achieved": flops / t1 / 1e12,
                                             "peak": 78.6, "unit": "TFLOP/s",
                                             "frac": flops / t1 / 1e12 / 78.6,
                                             "algorithmic_flops": flops,
                                             "note": "k = 1 call: build, inverse, change of ground, one norm pass"}},
                    "greedy_step": {"ms": 1000 * step_s,
                                    "roofline": {"bound": "hbm", "achieved": step_bytes / step_s / 1e9,
                                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                                 "frac": step_bytes / step_s / 1e9 / HBM_PEAK_GBS,
                                                 "algorithmic_bytes": step_bytes}}})
        # the sizes of the paper's group experiment (two citation graphs of 2708 and
        # 3327 vertices, k = 200, 400, 600), as seeded stand-ins of the same n and m
        shapes = []
        for name, gg in (("ba_n2708_m2", inputs.barabasi_albert(2708, 2, 0)),
                         ("er_n3327_m4552", inputs.erdos_renyi(3327, 2 * 4552 / (3327 * 3326), 0))):
            dgg = fc.to_device(gg, dev)
            for kk in (200, 400, 600):
                tt, _ = _timed(lambda: fc.group_closeness(dgg, 1.0, kk, device=dev, trusted=True),
                               args.steps, args.warmup)
                shapes.append({"graph": name, "n": gg.n, "m": gg.m, "k": kk, "ms": 1000 * tt})
        res["paper_sizes"] = shapes
    elif args.config == "grid1000":
        g = inputs.grid_removed(1000, 1000, 0.12, 0)
        dg = fc.to_device(g, dev)
        per = {}
        total_dt = 0.0
        for alpha in (0.5, 1.0, 2.0):
            dt, out = _timed(lambda: fc.farness(dg, alpha=alpha, tau=1024, device=dev, as_torch=True,
                                                sampler=args.sampler), args.steps, args.warmup)
            total_dt += dt
            per[str(alpha)] = {"trees_per_s": 1024 / dt, "walk_steps_per_tree": out["stats"]["walk_steps"] / 1024,
                               "kernel_ms": out["stats"]["ms_sample"], "sampler": out["stats"]["sampler"]}
            if args.phase_timing:
                per[str(alpha)]["phase_ms"] = out["stats"]["phase_ms"]
        res.update({"value": 3 * 1024 / total_dt, "unit": "trees/s",
                    "config": {"workload": "grid_1000x1000_rm0.12_alpha0.5_1_2_trees1024", "n": g.n,
                               "m": g.m}, "per_alpha": per})
    elif args.config == "rmat_batch":
        t0 = time.perf_counter()
        gs = inputs.rmat_batch(256, 8, 0)
        gen_s = time.perf_counter() - t0
        dgs = [fc.to_device(g, dev) for g in gs]
        alphas = (0.1, 1.0, 10.0)
        jobs = [{"graph": dg, "alpha": a, "stream_id": gi * 3 + ai, "tree_count": 512}
                for gi, dg in enumerate(dgs) for ai, a in enumerate(alphas)]
        ntrees = len(jobs) * 512
        t0 = time.perf_counter()
        b = fc.Batch(jobs, seed=0, trusted=False, autotune=True)
        create_s = time.perf_counter() - t0

        def run_batch():
            b.reset()
            return b.run()
        dt, st = _timed(run_batch, args.steps, args.warmup)

        def per_job():
            for j in jobs:
                fc.sample(j["graph"], alpha=j["alpha"], seed=0, tree_count=512,
                          stream_id=j["stream_id"], device=dev, as_torch=True, trusted=True)
        dt_single, _ = _timed(per_job, 1, 0)
        # the Wilson model's bytes (as for the single-graph line) over the batch kernel's time
        vertex_trees = 512 * len(alphas) * int(sum(g.n for g in gs))
        alg = (BYTES_STEP * st["walk_steps"] + (BYTES_RETRACE + BYTES_SCAN) * vertex_trees
               + BYTES_ROOT * st["roots"])
        ach = alg / (st["ms_sample"] / 1000.0) / 1e9
        res.update({"value": ntrees / dt, "unit": "trees/s",
                    "config": {"workload": "rmat_batch_256graphs_alpha0.1_1_10_trees512",
                               "graphs": len(gs), "sum_n": int(sum(g.n for g in gs)),
                               "sum_m": int(sum(g.m for g in gs)), "jobs": len(jobs), "trees": ntrees},
                    "batched": {"ms_per_run": 1000 * dt, "kernel_ms": st["ms_sample"],
                                "launch_shape": st["sampler"], "walk_steps_per_s": st["walk_steps"] / dt,
                                "create_s": create_s,
                                "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                             "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                             "algorithmic_bytes_per_launch": alg,
                                             "kernel": "wilson_lds_kernel (launch groups)"}},
                    "per_job_launches": {"ms_total": 1000 * dt_single, "trees_per_s": ntrees / dt_single},
                    "generation_s": gen_s})
        b.close()
    elif args.config == "solve":
        import torch
        g = inputs.barabasi_albert(2_000_000, 8, 0)
        dg = fc.to_device(g, dev)
        k = 64
        B = torch.from_numpy(inputs.gaussian(g.n * k, 0).reshape(g.n, k)).to(dev)
        legs = {}
        sols = {}
        for prec in ("fp64", "fp32_refined"):
            dt, out = _timed(lambda: fc.solve(dg, 1.0, B, rtol=1e-9, precision=prec, device=dev,
                                              trusted=True, as_torch=True), args.steps, args.warmup)
            sols[prec] = out["X"]
            # bytes of the inner iterations alone (gathered neighbour rows + 12 streamed
            # n x k arrays per iteration: apply, update, direction) over the whole leg,
            # residuals and refinement included in the time: a lower bound on the rate
            es = 8 if prec == "fp64" else 4
            alg = out["iters"] * (2 * g.m * k * es + 12 * g.n * k * es)
            ach = alg / dt / 1e9
            legs[prec] = {"ms": 1000 * dt, "inner_iters": out["iters"],
                          "max_relres": float(out["relres"].max()),
                          "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                       "algorithmic_bytes": alg}}
        diff = (sols["fp32_refined"] - sols["fp64"]).abs().amax(dim=0)
        scale = sols["fp64"].abs().amax(dim=0)
        legs["fp32_refined"]["max_abs_err_vs_fp64_per_column_max"] = float(diff.max())
        legs["fp32_refined"]["max_rel_err_vs_fp64"] = float((diff / scale).max())
        res.update({"metric": "solve time (alpha L + I) X = B to 1e-9", "unit": "ms",
                    "higher_is_better": False, "value": legs["fp32_refined"]["ms"],
                    "config": {"workload": "ba_n2000000_m8_alpha1_rhs64_rtol1e-9", "n": g.n, "m": g.m,
                               "rhs": k}, "legs": legs})
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
