"""Benchmark: forest-closeness estimation on one MI355X.

Workload (one "step" = the whole hot path once): Barabasi-Albert graph with
n = 200,000 and m = 5 (999,985 edges), alpha = 1, 4096 uniform spanning trees
of G* rooted at u* sampled with Wilson's algorithm, aggregated into the
estimated diagonal of Omega = (alpha L + I)^{-1}, forest farness and forest
closeness of every vertex.  The CSR is resident in device memory before the
timed region.  Prints one JSON line.

value = trees per second over the timed steps (whole job, one GPU).

The default line also carries, under "extras", the other sampling workloads
(road-like grid at three alphas, the batch of 256 R-MAT graphs, R-MAT 2^22 on
the hybrid sampler), each with its Wilson-model fraction of the HBM peak and,
where a counter summary taken on the current kernel source exists under
profiles/, its measured HBM traffic.  --config runs one workload alone;
--take-profiles runs rocprofv3 over the committed workloads and writes the
summaries (kernel trace, counters) stamped with the kernel source hash.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import subprocess
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
# int32 VALU lane-ops per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9

CSRC = os.path.join(ROOT, "paper_2101_06192_amd", "csrc")
PROFILE_DIR = os.path.join(ROOT, "profiles")

# Workloads with committed rocprofv3 summaries: bench arguments that run them
# (each label is one launch of the listed kernels, in dispatch order), the
# kernels whose counters are summed, and the sources whose hash stamps them.
PROFILE_SPECS = {
    "wilson_lds_ba200k": {
        "args": ["--config", "ba200k"], "kernels": ["lds_predraw_kernel", "wilson_lds_kernel"],
        "sources": ["wilson_lds.hip"], "labels": ["step"], "counters": True, "timeout": 240,
        "title": "BA(200000, 5), alpha = 1, 4096 trees per step (the headline), LDS-counter "
                 "sampler with its pre-draw kernel"},
    "wilson_lds_ba200k_w": {
        "args": ["--config", "ba200k_w"], "kernels": ["lds_predraw_kernel", "wilson_lds_kernel"],
        "sources": ["wilson_lds.hip"], "labels": ["step"], "counters": True, "timeout": 240,
        "title": "BA(200000, 5) with log-uniform [0.1, 10) edge weights, alpha = 1, 4096 trees"},
    "wilson_tile_grid1000": {
        "args": ["--config", "grid1000"], "kernels": ["tile_predraw_kernel", "wilson_tile_kernel"],
        "sources": ["wilson_tile.hip"], "labels": ["alpha0.5", "alpha1.0", "alpha2.0"],
        "counters": True, "timeout": 240,
        "title": "1000 x 1000 grid, 12% of edges removed, alpha = 0.5, 1, 2, 1024 trees each, "
                 "tile sampler with its pre-draw kernel"},
    "wilson_hyb_rmat22": {
        "args": ["--config", "rmat22", "--sampler", "hyb"], "kernels": ["wilson_hyb_kernel"],
        "sources": ["wilson_hyb.hip"], "labels": ["step"], "counters": True, "timeout": 360,
        "title": "R-MAT n = 2^22, edge factor 8, alpha = 1, 1024 trees, hybrid sampler"},
    "wilson_lds_batch_rmat256": {
        "args": ["--config", "rmat_batch"], "kernels": ["wilson_lds_kernel"],
        "sources": ["wilson_lds.hip", "fc_batch.cpp"], "labels": ["run"], "counters": True,
        "timeout": 420,
        "title": "256 R-MAT graphs (n log-uniform in [2^10, 2^17], edge factor 8) x alpha "
                 "{0.1, 1, 10} x 512 trees, one autotuned batch run (its launch groups)"},
    "wilson_lane_er1000": {
        "args": ["--config", "er1000", "--sampler", "lane"], "kernels": ["wilson_lane_kernel"],
        "sources": ["wilson_lane.hip"], "labels": ["step"], "counters": False, "timeout": 180,
        "title": "Erdos-Renyi n = 1000, p = 0.01, alpha = 1, 2000 trees, lane-per-tree sampler"},
    "cg_ba2m_rhs64": {
        "args": ["--config", "solve"],
        "kernels": ["apply_kernel", "residual_kernel", "update_kernel", "direction_kernel",
                    "correct_kernel", "reduce_kernel", "scalars_kernel", "start_kernel"],
        "sources": ["cg.hip", "fc_solve.cpp"], "labels": None, "counters": True, "timeout": 300,
        "title": "(alpha L + I) X = B on BA(2000000, 8), 64 right-hand sides, rtol 1e-9, "
                 "binary64 then binary32 with binary64 refinement"},
    "group_closeness_ba20k": {
        "args": ["--config", "group"], "kernels": [], "sources": ["group.hip", "fc_group.cpp"],
        "labels": None, "counters": False, "timeout": 300,
        "title": "greedy group forest closeness on BA(20000, 5), k = 1 and k = 50, then the "
                 "paper's group sizes"},
    "fc_rank_kendall_ba200k": {
        "args": ["--config", "rank"], "kernels": [], "sources": ["rank.hip", "fc_rank.cpp"],
        "labels": None, "counters": False, "timeout": 300,
        "title": "closeness ranking and Kendall's tau-b at n = 200000, KT against a CG truth"},
}


def _local_includes(path: str) -> list:
    out = []
    with open(path, encoding="utf-8", errors="replace") as f:
        for line in f:
            m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
            if m:
                out.append(m.group(1))
    return out


def hashed_files(sources) -> list:
    """The named sources and every local header they include (transitively)."""
    todo, seen = list(sources), set()
    while todo:
        name = todo.pop()
        if name in seen or _src_path(name) is None:
            continue
        seen.add(name)
        todo.extend(_local_includes(_src_path(name)))
    return sorted(seen)


def _src_path(name):
    for d in (CSRC, os.path.join(ROOT, "include")):
        p = os.path.join(d, name)
        if os.path.exists(p):
            return p
    return None


def code_tokens(text: str) -> str:
    """C/C++ source without its comments and with whitespace runs collapsed:
    what a profile depends on (a comment or layout edit leaves the hash alone)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":  # string or character literal, kept whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_hash(sources) -> str:
    """sha256[:16] over the code (comments and layout dropped) of the named
    sources and every local header they include, in name order."""
    h = hashlib.sha256()
    for name in hashed_files(sources):
        h.update(name.encode())
        with open(_src_path(name), encoding="utf-8", errors="replace") as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def read_summary(stem: str, kind: str = "traffic"):
    """Key/value lines of profiles/<stem>_<kind>.txt, or None when the file is
    missing or was taken on a different kernel source."""
    path = os.path.join(PROFILE_DIR, f"{stem}_{kind}.txt")
    if not os.path.exists(path) or stem not in PROFILE_SPECS:
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash(PROFILE_SPECS[stem]["sources"]):
        return None
    return vals


def traffic_of(stem: str, label: str = "step"):
    """HBM bytes of one launch (label) from the counter summary, or None."""
    vals = read_summary(stem)
    if vals is None:
        return None
    try:
        return float(vals[f"hbm_bytes_per_launch.{label}"])
    except (KeyError, ValueError):
        return None


def wilson_bytes(walk_steps: int, vertex_trees: int, roots: int, weighted: bool = False) -> int:
    step = BYTES_STEP_W if weighted else BYTES_STEP
    return step * walk_steps + (BYTES_RETRACE + BYTES_SCAN) * vertex_trees + BYTES_ROOT * roots


def roofline_hbm(alg_bytes: float, kernel_ms: float, traffic=None, **extra) -> dict:
    """HBM roofline of one launch: the method's bytes over the launch's HIP-event
    time against 8 TB/s; with a counter summary, the measured traffic too."""
    s = kernel_ms / 1000.0
    ach = alg_bytes / s / 1e9
    d = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel_ms": kernel_ms,
         "algorithmic_bytes_per_launch": alg_bytes}
    if traffic:
        d["traffic_frac"] = traffic / s / 1e9 / HBM_PEAK_GBS
        d["traffic_over_algorithmic"] = traffic / alg_bytes
    d.update(extra)
    return d


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = nproc
    omp = os.environ.get("OMP_NUM_THREADS")
    share = min(aff, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else aff
    return {"cpu_model": model, "nproc": nproc, "affinity_cpus": aff,
            "omp_num_threads": omp, "cores_used": share}


def _oracle_range(args):
    g, t0, count = args
    import oracle
    t = time.perf_counter()
    r = oracle.sample(g, 1.0, 0, t0, count)
    return time.perf_counter() - t, r.R


def cpu_baseline(g, trees: int) -> dict:
    """The C oracle on the host: one core on trees [0, trees), then one process
    per core of this process's CPU share (its affinity set, capped by
    OMP_NUM_THREADS, the share the host gives one GPU) on disjoint tree ranges
    (integer sums, so the ranges add up exactly).  Runs before the process
    touches the GPU: the workers are forked."""
    import multiprocessing as mp
    host = host_info()
    t0 = time.perf_counter()
    _oracle_range((g, 0, trees))
    one = time.perf_counter() - t0
    cores = host["cores_used"]
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
                            "sample": f"trees 0..{trees - 1}, one process, {one:.1f} s"},
            "host": host}


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


def _phases(st):
    """Per-phase wall time per workgroup of a workgroup sampler's call."""
    if st["sampler"] == "wilson_lds":
        names = ["first_arrows", "count_and_level0", "peel_wide", "peel_tail",
                 "sweep_and_split", "cycle_scan", "cycles", "output"]
    elif st["sampler"] == "wilson_tile":
        names = ["tile_load", "count_and_level0", "peel_and_sweep", "cycle_pops", "tile_exits",
                 "exit_graph", "residual", "output"]
    else:
        names = ["first_arrows", "in_arrows", "peel_level0", "peel_levels", "sweep", "redraw",
                 "output"]
    return dict(zip(names, st["phase_ms"]))


def _kernels_ms(st):
    """The sampling call's kernels and their HIP-event times (the pre-draw kernel,
    when one ran, is inside ms_sample)."""
    ms = st["ms_sample"]
    pre = st.get("ms_predraw", 0.0)
    name = f"{st['sampler']}_kernel"
    if pre > 0.0:
        pre_name = "tile_predraw_kernel" if st["sampler"] == "wilson_tile" else "lds_predraw_kernel"
        return {pre_name: pre, name: ms - pre}
    return {name: ms}


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def leg_sampling(fc, dev, g, dg, trees, alpha, steps, warmup, sampler="auto", weighted=False,
                 stem=None, label="step", phase=False, seed=0):
    """`steps` timed calls of farness (sample + estimate) on a resident graph."""
    stats = []

    def step():
        out = fc.farness(dg, alpha=alpha, seed=seed, tau=trees, device=dev, as_torch=True,
                         sampler=sampler)
        stats.append(out["stats"])
        return out
    dt, out = _timed(step, steps, warmup)
    timed = stats[warmup:]
    st = timed[-1]
    kms = sum(s["ms_sample"] for s in timed) / len(timed)
    kernels = {}
    for s in timed:
        for k, v in _kernels_ms(s).items():
            kernels[k] = kernels.get(k, 0.0) + v / len(timed)
    alg = wilson_bytes(st["walk_steps"], g.n * trees, st["roots"], weighted)
    traffic = traffic_of(stem, label) if stem else None
    res = {"trees_per_s": trees / dt, "ms_per_step": 1000 * dt, "sampler": st["sampler"],
           "trees_in_flight": st["trees_in_flight"],
           "walk_steps_per_tree": st["walk_steps"] / trees,
           "walk_steps_per_s": st["walk_steps"] / dt,
           "roofline": roofline_hbm(alg, kms, traffic, kernels_ms=kernels,
                                    kernel=" + ".join(kernels))}
    if phase:
        res["phase_ms_per_workgroup"] = _phases(st)
    return res


def leg_grid(fc, inputs, dev, steps, warmup, sampler="auto", phase=False) -> dict:
    """Road-like grid: 1000 x 1000 with 12% of edges removed, 1024 trees at each
    of alpha = 0.5, 1, 2 (one launch per alpha)."""
    g = inputs.grid_removed(1000, 1000, 0.12, 0)
    dg = fc.to_device(g, dev)
    per, total = {}, 0.0
    for alpha in (0.5, 1.0, 2.0):
        r = leg_sampling(fc, dev, g, dg, 1024, alpha, steps, warmup, sampler,
                         stem="wilson_tile_grid1000", label=f"alpha{alpha}", phase=phase)
        total += r["ms_per_step"] / 1000.0
        per[str(alpha)] = r
    return {"value": 3 * 1024 / total, "unit": "trees/s",
            "config": {"workload": "grid_1000x1000_rm0.12_alpha0.5_1_2_trees1024", "n": g.n,
                       "m": g.m}, "per_alpha": per}


def leg_batch(fc, inputs, dev, steps, warmup, side=True) -> dict:
    """256 R-MAT graphs x alpha {0.1, 1, 10} x 512 trees as one autotuned batch,
    against the same 768 jobs as separate fc_sample calls."""
    t0 = time.perf_counter()
    gs = inputs.rmat_batch(256, 8, 0)
    gen_s = time.perf_counter() - t0
    dgs = [fc.to_device(g, dev) for g in gs]
    alphas = (0.1, 1.0, 10.0)
    jobs = [{"graph": dg, "alpha": a, "stream_id": gi * 3 + ai, "tree_count": 512}
            for gi, dg in enumerate(dgs) for ai, a in enumerate(alphas)]
    ntrees = len(jobs) * 512
    fc.set_option("lds_repop", 3, dev)  # the tuner also times re-pops on and off
    t0 = time.perf_counter()
    b = fc.Batch(jobs, seed=0, trusted=False, autotune=True)
    create_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    b2 = fc.Batch(jobs, seed=0, trusted=False, autotune=True)  # same shapes: the cached choice
    create_cached_s = time.perf_counter() - t0
    b2.close()

    def run_batch():
        b.reset()
        return b.run()
    stats = []

    def run_and_keep():
        st = run_batch()
        stats.append(st)
        return st
    dt, st = _timed(run_and_keep, steps, warmup)
    kms = sum(s["ms_sample"] for s in stats[warmup:]) / steps
    vertex_trees = 512 * len(alphas) * int(sum(g.n for g in gs))
    alg = wilson_bytes(st["walk_steps"], vertex_trees, st["roots"])
    res = {"value": ntrees / dt, "unit": "trees/s",
           "config": {"workload": "rmat_batch_256graphs_alpha0.1_1_10_trees512",
                      "graphs": len(gs), "sum_n": int(sum(g.n for g in gs)),
                      "sum_m": int(sum(g.m for g in gs)), "jobs": len(jobs), "trees": ntrees},
           "batched": {"trees_per_s": ntrees / dt, "ms_per_run": 1000 * dt,
                       "launch_shape": st["sampler"],
                       "walk_steps_per_s": st["walk_steps"] / dt,
                       "create_s": create_s, "create_cached_s": create_cached_s,
                       "roofline": roofline_hbm(alg, kms,
                                                traffic_of("wilson_lds_batch_rmat256", "run"),
                                                kernel="wilson_lds_kernel (launch groups)")},
           "generation_s": gen_s,
           # the launch groups of the last run are the batch's last dispatches
           "profile_last_dispatches": 2 if "+" in st["sampler"] else 1}
    b.close()
    if side:
        def per_job():
            for j in jobs:
                fc.sample(j["graph"], alpha=j["alpha"], seed=0, tree_count=512,
                          stream_id=j["stream_id"], device=dev, as_torch=True, trusted=True)
        dt_single, _ = _timed(per_job, 1, 1)
        res["per_job_launches"] = {"trees_per_s": ntrees / dt_single,
                                   "ms_total": 1000 * dt_single, "launches": len(jobs)}
        res["batched_over_per_job"] = dt_single / dt
    return res


def leg_rmat22(fc, inputs, dev, steps, warmup, samplers=("hyb",), eps=True, phase=False) -> dict:
    """R-MAT n = 2^22, edge factor 8, alpha = 1, 1024 trees; the time to an
    (eps = 0.1, delta = 0.1) estimate of diag(Omega)."""
    import torch
    t0 = time.perf_counter()
    g = inputs.rmat(1 << 22, 8, 0)
    gen_s = time.perf_counter() - t0
    dg = fc.to_device(g, dev)
    per = {}
    for smp in samplers:
        per[smp] = leg_sampling(fc, dev, g, dg, 1024, 1.0, steps, warmup, smp,
                                stem="wilson_hyb_rmat22" if smp == "hyb" else None, phase=phase)
    best = max(per, key=lambda k: per[k]["trees_per_s"])
    res = {"value": per[best]["trees_per_s"], "unit": "trees/s",
           "config": {"workload": "rmat_n4194304_ef8_alpha1_trees1024", "n": g.n, "m": g.m,
                      "alpha": 1.0, "trees": 1024}, "samplers": per, "generation_s": gen_s}
    if eps:
        torch.cuda.synchronize()
        te = time.perf_counter()
        o = fc.diag_estimate(dg, alpha=1.0, eps=0.1, delta=0.1, device=dev, as_torch=True,
                             sampler=samplers[0] if len(samplers) == 1 else "auto")
        torch.cuda.synchronize()
        res["time_to_eps0.1_diag"] = {"tau": o["tau"], "ms": 1000 * (time.perf_counter() - te)}
    return res


def leg_er1000(fc, inputs, dev, steps, warmup, samplers=("lane", "coop", "lds"),
               phase=False) -> dict:
    g = inputs.erdos_renyi(1000, 0.01, 0)
    dg = fc.to_device(g, dev)
    per = {smp: leg_sampling(fc, dev, g, dg, 2000, 1.0, steps, warmup, smp, phase=phase)
           for smp in samplers}
    best = max(per, key=lambda k: per[k]["trees_per_s"])
    return {"value": per[best]["trees_per_s"], "unit": "trees/s",
            "config": {"workload": "er_n1000_p0.01_alpha1_trees2000", "n": g.n, "m": g.m,
                       "alpha": 1.0, "trees": 2000}, "samplers": per}


def leg_weighted(fc, inputs, dev, steps, warmup, sampler="auto", eps=True, phase=False) -> dict:
    """The headline graph with seeded log-uniform edge weights in [0.1, 10)."""
    import torch
    g = inputs.with_weights(inputs.barabasi_albert(200_000, 5, 0), 0)
    dg = fc.to_device(g, dev)
    r = leg_sampling(fc, dev, g, dg, 4096, 1.0, steps, warmup, sampler, weighted=True,
                     stem="wilson_lds_ba200k_w", phase=phase)
    res = {"value": r["trees_per_s"], "unit": "trees/s",
           "config": {"workload": "ba_n200000_m5_logw0.1_10_alpha1_trees4096", "n": g.n,
                      "m": g.m, "alpha": 1.0, "trees": 4096}, **r}
    if eps:
        torch.cuda.synchronize()
        te = time.perf_counter()
        o = fc.diag_estimate(dg, alpha=1.0, eps=0.1, delta=0.1, device=dev, as_torch=True,
                             sampler=sampler)
        torch.cuda.synchronize()
        res["time_to_eps0.1_diag"] = {"tau": o["tau"], "ms": 1000 * (time.perf_counter() - te)}
    return res


def leg_solve(fc, inputs, dev, steps, warmup) -> dict:
    """(alpha L + I) X = B to rtol 1e-9 on BA(2000000, 8) with 64 right-hand sides."""
    import torch
    g = inputs.barabasi_albert(2_000_000, 8, 0)
    dg = fc.to_device(g, dev)
    k = 64
    B = torch.from_numpy(inputs.gaussian(g.n * k, 0).reshape(g.n, k)).to(dev)
    legs, sols = {}, {}
    for prec in ("fp64", "fp32_refined"):
        dt, out = _timed(lambda: fc.solve(dg, 1.0, B, rtol=1e-9, precision=prec, device=dev,
                                          trusted=True, as_torch=True), steps, warmup)
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
    return {"metric": "solve time (alpha L + I) X = B to 1e-9", "unit": "ms",
            "higher_is_better": False, "value": legs["fp32_refined"]["ms"],
            "config": {"workload": "ba_n2000000_m8_alpha1_rhs64_rtol1e-9", "n": g.n, "m": g.m,
                       "rhs": k}, "legs": legs}


def leg_rank(fc, inputs, dev, steps, warmup) -> dict:
    """Ranking output: the headline graph's closeness ranking and Kendall's tau-b
    at n = 200000; the KT of eps-estimates against a CG ground truth of every
    Omega_vv on BA(20000, 5)."""
    import torch
    g = inputs.barabasi_albert(200_000, 5, 0)
    dg = fc.to_device(g, dev)
    est = fc.farness(dg, alpha=1.0, eps=0.1, delta=0.1, device=dev, as_torch=True)
    clo, diag = est["closeness"], est["diag"]
    dt_rank, _ = _timed(lambda: fc.rank(clo, descending=True, device=dev, as_torch=True),
                        steps, warmup)
    other = fc.farness(dg, alpha=1.0, eps=0.1, delta=0.1, seed=1, device=dev, as_torch=True)
    dt_kt, kt = _timed(lambda: fc.kendall_tau(diag, other["diag"], device=dev), steps, warmup)
    fc.set_option("kendall_pairs", 1, dev)
    dt_pairs, kt_pairs = _timed(lambda: fc.kendall_tau(diag, other["diag"], device=dev),
                                steps, warmup)
    fc.set_option("kendall_pairs", 0, dev)
    assert kt_pairs["counts"] == kt["counts"]
    n = g.n
    pairs = n * (n - 1) // 2
    # the all-pairs kernel is VALU-bound: 10 instructions per pair (two
    # differences, two v_med3_i32 signs, a product, three multiply-adds, loop share)
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
    return {"metric": "ranking: fc_rank and fc_kendall_tau time at n = 200000; KT vs CG",
            "value": 1000 * dt_kt, "unit": "ms (fc_kendall_tau, n = 200000)",
            "higher_is_better": False,
            "config": {"workload": "ba_n200000_m5_alpha1_eps0.1_rank_kendall", "n": n,
                       "kt_graph": "ba_n20000_m5_alpha1"},
            "rank_ms": 1000 * dt_rank,
            "kendall_ms": 1000 * dt_kt,
            "kendall_all_pairs": {"ms": 1000 * dt_pairs, "pairs_per_s": pairs / dt_pairs,
                                  "roofline": {"bound": "alu",
                                               "achieved": 10 * pairs / dt_pairs / 1e12,
                                               "peak": VALU_LANE_OPS / 1e12,
                                               "unit": "T int32 lane-ops/s",
                                               "frac": 10 * pairs / dt_pairs / VALU_LANE_OPS}},
            "kendall_two_estimates_tau_b": kt["tau_b"],
            "ground_truth_s": truth_s, "kt_vs_cg": quality}


def leg_group(fc, inputs, dev, steps, warmup, side=True) -> dict:
    """Group forest closeness (Algorithm 2): one dense inverse (the k = 1 call),
    then one downdate pass over the n x n matrix per greedy step."""
    g = inputs.barabasi_albert(20_000, 5, 0)
    dg = fc.to_device(g, dev)
    k = 50
    t1, _ = _timed(lambda: fc.group_closeness(dg, 1.0, 1, device=dev, trusted=True), steps, warmup)
    tk, out = _timed(lambda: fc.group_closeness(dg, 1.0, k, device=dev, trusted=True), steps,
                     warmup)
    # the method's flops: Gauss-Jordan inversion of the n x n matrix, n^3
    # multiply-adds (the kernels pad n to a multiple of 256 and do 2 N^3)
    flops = 2.0 * g.n ** 3
    N = (g.n + 255) // 256 * 256
    inv = {"ms_whole_k1_call": 1000 * t1, "padded_dim": N}
    trace = read_summary("group_closeness_ba20k", "kernel_trace")
    inv_ms = None
    if trace is not None:
        try:
            inv_ms = float(trace["inverse_kernels_ms_per_call"])
        except (KeyError, ValueError):
            inv_ms = None
    t_inv = inv_ms / 1000.0 if inv_ms else t1
    inv["roofline"] = {"bound": "mfma", "achieved": flops / t_inv / 1e12, "peak": 78.6,
                       "unit": "TFLOP/s", "frac": flops / t_inv / 1e12 / 78.6,
                       "algorithmic_flops": flops,
                       "time": ("the inverse's kernels (gemm, gj_*) per call from the kernel "
                                "trace summary" if inv_ms else
                                "the whole k = 1 call (build, inverse, change of ground, norm pass)")}
    step_s = (tk - t1) / (k - 1)
    step_bytes = 16.0 * g.n * g.n  # read and write the n x n binary64 matrix
    res = {"metric": "greedy group forest closeness time (Algorithm 2)", "value": 1000 * tk,
           "unit": "ms", "higher_is_better": False,
           "config": {"workload": "ba_n20000_m5_alpha1_group_k50", "n": g.n, "m": g.m, "k": k},
           "group_head": out["group"][:8],
           "farness_first_last": [out["farness"][0], out["farness"][-1]],
           "inverse": inv,
           "greedy_step": {"ms": 1000 * step_s,
                           "roofline": {"bound": "hbm", "achieved": step_bytes / step_s / 1e9,
                                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": step_bytes / step_s / 1e9 / HBM_PEAK_GBS,
                                        "algorithmic_bytes": step_bytes}}}
    if not side:
        return res
    # the sizes of the paper's group experiment (two citation graphs of 2708 and
    # 3327 vertices, k = 200, 400, 600), as seeded stand-ins of the same n and m
    shapes = []
    for name, gg in (("ba_n2708_m2", inputs.barabasi_albert(2708, 2, 0)),
                     ("er_n3327_m4552", inputs.erdos_renyi(3327, 2 * 4552 / (3327 * 3326), 0))):
        dgg = fc.to_device(gg, dev)
        for kk in (200, 400, 600):
            tt, _ = _timed(lambda: fc.group_closeness(dgg, 1.0, kk, device=dev, trusted=True),
                           steps, warmup)
            shapes.append({"graph": name, "n": gg.n, "m": gg.m, "k": kk, "ms": 1000 * tt})
    res["paper_sizes"] = shapes
    return res


# --------------------------------------------------------------------------
# profiles: rocprofv3 runs of the workloads above, summarised
# --------------------------------------------------------------------------
def _child_json(path):
    last = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{") and line.endswith("}"):
                last = line
    return json.loads(last) if last else None


def _run_pass(cmd, log, timeout_s):
    print("profile pass: " + " ".join(cmd), flush=True)
    with open(log, "w") as f:
        try:
            r = subprocess.run(cmd, stdout=f, stderr=subprocess.STDOUT, timeout=timeout_s,
                               cwd=ROOT)
        except subprocess.TimeoutExpired:
            print(f"profile pass timed out after {timeout_s} s (log {log})", flush=True)
            return 124
    print(f"profile pass exit {r.returncode}", flush=True)
    return r.returncode


def _csv_rows(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    rows = []
    for p in files:
        with open(p, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _short(name):
    """A profiler kernel name without namespaces, return type and parameters."""
    s = name.replace("(anonymous namespace)::", "").split("(")[0].strip()
    s = re.sub(r"^void\s+", "", s)
    return re.sub(r"^[\w:]*::", "", s)


def _matches(name, kernels):
    """One of this library's kernels (namespace fc), by short name."""
    if "fc::" not in name:
        return False
    short = _short(name)
    return any(short == k or short.startswith(k + "<") for k in kernels)


def _dispatch_counters(rows, kernels):
    """{dispatch id: (short kernel name, {counter: value})} for the named kernels."""
    out = {}
    for r in rows:
        if not _matches(r["Kernel_Name"], kernels):
            continue
        d = int(r["Dispatch_Id"])
        ent = out.setdefault(d, (_short(r["Kernel_Name"]), {}))
        ent[1][r["Counter_Name"]] = ent[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def take_profiles(stems, out_dir):
    """rocprofv3 over each workload: a kernel trace (--kernel-trace --stats) and,
    for the sampling kernels, one counter pass each for FETCH_SIZE, WRITE_SIZE,
    TCC hits/misses and the SQ instruction mix, plus a plain 1 GiB copy for the
    byte calibration; summaries stamped with the kernel source hash."""
    raw = os.path.join(out_dir, "raw")
    os.makedirs(raw, exist_ok=True)
    py = "python3"
    me = os.path.relpath(os.path.abspath(__file__), ROOT)
    base_args = ["--cpu-trees", "0", "--no-eps", "--no-extras", "--no-side"]
    made_by = f"python3 bench.py --take-profiles {','.join(stems)}"

    def prof(tag, prof_args, bench_args, timeout_s):
        d = os.path.join(raw, tag)
        cmd = ["rocprofv3", *prof_args, "-f", "csv", "-d", d, "-o", "run", "--", py, me,
               *bench_args]
        rc = _run_pass(cmd, os.path.join(raw, tag + ".log"), timeout_s)
        if rc != 0:
            raise SystemExit(f"profile pass {tag} failed with exit code {rc}")
        return d, cmd

    calib = None
    if any(PROFILE_SPECS[s]["counters"] for s in stems):
        fd, fcmd = prof("copy_fetch", ["--pmc", "FETCH_SIZE"], ["--calibrate-copy", "1024"], 120)
        wd, wcmd = prof("copy_write", ["--pmc", "WRITE_SIZE"], ["--calibrate-copy", "1024"], 120)
        fr = [r for r in _csv_rows(fd, "counter_collection.csv") if "copy" in r["Kernel_Name"].lower()
              or "Copy" in r["Kernel_Name"]]
        wr = [r for r in _csv_rows(wd, "counter_collection.csv") if "copy" in r["Kernel_Name"].lower()
              or "Copy" in r["Kernel_Name"]]
        big_f = max(float(r["Counter_Value"]) for r in fr)
        big_w = max(float(r["Counter_Value"]) for r in wr)
        kib = 1024 * 1024  # 1 GiB read and 1 GiB written, in KiB
        calib = {"fetch_factor": kib / big_f, "write_factor": kib / big_w,
                 "fetch_kib": big_f, "write_kib": big_w,
                 "commands": [" ".join(fcmd), " ".join(wcmd)]}
    for stem in stems:
        spec = PROFILE_SPECS[stem]
        h = kernel_hash(spec["sources"])
        files = hashed_files(spec["sources"])
        to = spec["timeout"]
        # kernel trace
        td, tcmd = prof(stem + "_trace", ["--kernel-trace", "--stats"],
                        [*spec["args"], *base_args, "--steps", "3", "--warmup", "1"], to)
        child = _child_json(os.path.join(raw, stem + "_trace.log"))
        stats = _csv_rows(td, "kernel_stats.csv")
        lines = [f"# rocprofv3 kernel trace: {spec['title']}",
                 f"# made by: {made_by}",
                 f"# command: {' '.join(tcmd)}",
                 f"# kernel sources hashed: {' '.join(files)}",
                 f"kernel_source_sha256_16: {h}"]
        if child and "launches" in child:
            for lab, v in child["launches"].items():
                lines.append(f"bench_kernel_ms_hip_events.{lab}: {v['kernel_ms']:.4f}")
        def col(r, *keys):
            for k in keys:
                for kk in r:
                    if kk.lower() == k.lower():
                        return r[kk]
            return None
        tot = sum(float(col(r, "TotalDurationNs") or 0) for r in stats)
        inv_ns = 0.0
        lines.append("# kernel | calls | avg_ms | min_ms | max_ms | share_%")
        for r in sorted(stats, key=lambda r: -float(col(r, "TotalDurationNs") or 0)):
            name = _short(col(r, "Name", "KernelName", "Kernel_Name") or "?")
            tns = float(col(r, "TotalDurationNs") or 0)
            if name.startswith("gemm") or name.startswith("gj_"):
                inv_ns += tns
            if len(lines) < 5 + 16 + 8:
                lines.append(f"{name} | {col(r, 'Calls')} | {float(col(r, 'AverageNs') or 0) / 1e6:.4f} | "
                             f"{float(col(r, 'MinNs') or 0) / 1e6:.4f} | "
                             f"{float(col(r, 'MaxNs') or 0) / 1e6:.4f} | "
                             f"{100 * tns / tot if tot else 0:.2f}")
        if stem == "group_closeness_ba20k" and child and "inverse_calls" in child:
            lines.append(f"inverse_kernels_ms_per_call: {inv_ns / 1e6 / child['inverse_calls']:.4f}")
        with open(os.path.join(out_dir, f"{stem}_kernel_trace.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
        print(f"wrote {stem}_kernel_trace.txt", flush=True)
        if not spec["counters"]:
            continue
        one = [*spec["args"], *base_args, "--steps", "1", "--warmup", "0"]
        passes = {"fetch": ["FETCH_SIZE"], "write": ["WRITE_SIZE"],
                  "tcc": ["TCC_HIT_sum", "TCC_MISS_sum"],
                  "sq": ["SQ_INSTS_VALU", "SQ_INSTS_VMEM", "SQ_INSTS_LDS", "SQ_WAVES",
                         "SQ_BUSY_CYCLES"]}
        got, cmds, child1 = {}, [], None
        for tag, ctrs in passes.items():
            d, cmd = prof(f"{stem}_{tag}", ["--pmc", *ctrs], one, to)
            cmds.append(" ".join(cmd))
            got[tag] = _dispatch_counters(_csv_rows(d, "counter_collection.csv"), spec["kernels"])
            child1 = child1 or _child_json(os.path.join(raw, f"{stem}_{tag}.log"))
        last = (child1 or {}).get("profile_last_dispatches")
        labels = spec["labels"]
        out = [f"# rocprofv3 counters: {spec['title']}",
               f"# made by: {made_by}",
               "# passes (one counter set each, one step, no warm-up):"]
        out += [f"#   {c}" for c in cmds]
        out += ["# calibration: a plain 1 GiB device copy, same two counters:"]
        out += [f"#   {c}" for c in calib["commands"]]
        out += [f"#   copy FETCH_SIZE {calib['fetch_kib']:.0f} KiB for 1048576 KiB read -> "
                f"fetch factor {calib['fetch_factor']:.3f}",
                f"#   copy WRITE_SIZE {calib['write_kib']:.0f} KiB for 1048576 KiB written -> "
                f"write factor {calib['write_factor']:.3f}",
                "# hbm bytes = (FETCH_SIZE x fetch factor + WRITE_SIZE x write factor) x 1024",
                f"# kernel sources hashed: {' '.join(files)}",
                f"kernel_source_sha256_16: {h}",
                f"kernels: {' + '.join(spec['kernels'])}",
                f"fetch_factor: {calib['fetch_factor']:.4f}",
                f"write_factor: {calib['write_factor']:.4f}"]
        # per-kernel totals over every dispatch of the pass
        names = sorted({v[0] for v in got["fetch"].values()})
        for nm in names:
            tf = sum(v[1].get("FETCH_SIZE", 0) for v in got["fetch"].values() if v[0] == nm)
            tw = sum(v[1].get("WRITE_SIZE", 0) for v in got["write"].values() if v[0] == nm)
            nd = sum(1 for v in got["fetch"].values() if v[0] == nm)
            sq = {c: sum(v[1].get(c, 0) for v in got["sq"].values() if v[0] == nm)
                  for c in passes["sq"]}
            out.append(f"kernel {nm}: dispatches {nd} fetch_kib {tf:.0f} write_kib {tw:.0f} "
                       + " ".join(f"{c.lower()} {sq[c]:.0f}" for c in passes["sq"]))
        if labels:
            seq = {t: [got[t][i] for i in sorted(got[t])] for t in ("fetch", "write", "tcc", "sq")}
            if last:
                # only the run's own launches (the earlier dispatches: tuning runs)
                for t in seq:
                    seq[t] = seq[t][-int(last):]
            nl = len(labels)
            for t in seq:
                if len(seq[t]) % nl:
                    raise SystemExit(f"{stem}: {len(seq[t])} {t} dispatches do not split into "
                                     f"{nl} launches")
            launches = (child1 or {}).get("launches", {})
            out.append(f"labels: {' '.join(labels)}")
            for li, lab in enumerate(labels):
                def part(t):
                    k = len(seq[t]) // nl
                    return seq[t][li * k:(li + 1) * k]
                fk = sum(v[1].get("FETCH_SIZE", 0) for v in part("fetch"))
                wk = sum(v[1].get("WRITE_SIZE", 0) for v in part("write"))
                hit = sum(v[1].get("TCC_HIT_sum", 0) for v in part("tcc"))
                miss = sum(v[1].get("TCC_MISS_sum", 0) for v in part("tcc"))
                byt = (fk * calib["fetch_factor"] + wk * calib["write_factor"]) * 1024
                out.append(f"dispatches.{lab}: {' + '.join(v[0] for v in part('fetch'))}")
                out.append(f"fetch_kib_per_launch.{lab}: {fk:.0f}")
                out.append(f"write_kib_per_launch.{lab}: {wk:.0f}")
                out.append(f"hbm_bytes_per_launch.{lab}: {byt:.0f}")
                out.append(f"tcc_hit.{lab}: {hit:.0f}")
                out.append(f"tcc_miss.{lab}: {miss:.0f}")
                if hit + miss:
                    out.append(f"tcc_hit_rate.{lab}: {hit / (hit + miss):.3f}")
                tl = ((child or {}).get("launches") or {}).get(lab) or launches.get(lab)
                if tl:
                    alg = tl["algorithmic_bytes"]
                    out.append(f"algorithmic_bytes_per_launch.{lab}: {alg:.0f}")
                    out.append(f"traffic_over_algorithmic.{lab}: {byt / alg:.2f}")
                    out.append(f"kernel_ms_hip_events.{lab}: {tl['kernel_ms']:.4f}")
                    out.append(f"hbm_gbs_at_that_time.{lab}: {byt / tl['kernel_ms'] / 1e6:.0f}")
        with open(os.path.join(out_dir, f"{stem}_traffic.txt"), "w") as f:
            f.write("\n".join(out) + "\n")
        print(f"wrote {stem}_traffic.txt", flush=True)


def _launches_of(res) -> dict:
    """label -> {kernel_ms, algorithmic_bytes} of a workload's sampling launches."""
    out = {}
    if "per_alpha" in res:
        for a, r in res["per_alpha"].items():
            out[f"alpha{a}"] = {"kernel_ms": r["roofline"]["kernel_ms"],
                                "algorithmic_bytes": r["roofline"]["algorithmic_bytes_per_launch"]}
    elif "batched" in res:
        rf = res["batched"]["roofline"]
        out["run"] = {"kernel_ms": rf["kernel_ms"], "algorithmic_bytes": rf["algorithmic_bytes_per_launch"]}
    elif "samplers" in res and len(res["samplers"]) == 1:
        rf = next(iter(res["samplers"].values()))["roofline"]
        out["step"] = {"kernel_ms": rf["kernel_ms"], "algorithmic_bytes": rf["algorithmic_bytes_per_launch"]}
    elif "roofline" in res and "kernel_ms" in res["roofline"]:
        rf = res["roofline"]
        out["step"] = {"kernel_ms": rf["kernel_ms"], "algorithmic_bytes": rf["algorithmic_bytes_per_launch"]}
    return out


# --------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-trees", type=int, default=640,
                    help="trees the CPU oracle samples for the baseline (0 = skip)")
    ap.add_argument("--no-eps", action="store_true",
                    help="skip the time-to-eps=0.1 legs and the random-access probe")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: no grid, batch and R-MAT 2^22 extras")
    ap.add_argument("--no-side", action="store_true",
                    help="skip side comparisons (the batch's per-job launches)")
    ap.add_argument("--extra-steps", type=int, default=3, help="timed steps of each extra")
    ap.add_argument("--sampler", default="auto",
                    choices=["auto", "lane", "coop", "lds", "hyb", "tile"])
    ap.add_argument("--config", default="ba200k",
                    choices=["ba200k", "ba200k_w", "er1000", "grid1000", "rmat_batch", "rmat22",
                             "solve", "rank", "group"],
                    help="workload; the default is the headline configuration")
    ap.add_argument("--lds-repop", type=int, default=None, choices=[0, 1, 2, 3],
                    help="LDS sampler: pop re-formed 2-cycles within their round "
                         "(0 never, 1 weighted graphs, 2 always, 3 always and tuned in batches)")
    ap.add_argument("--coop-repop", type=int, default=None, choices=[0, 1, 2],
                    help="global-counter sampler: the same option (coop_repop)")
    ap.add_argument("--phase-timing", action="store_true",
                    help="report per-phase times of the workgroup sampler (adds clock reads)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    ap.add_argument("--take-profiles", default=None, metavar="STEMS",
                    help="comma-separated workloads (or 'all') to run under rocprofv3; "
                         "summaries go to --profile-out")
    ap.add_argument("--profile-out", default=os.path.join(ROOT, "profile_runs"),
                    help="directory for the summaries and the raw rocprofv3 output")
    args = ap.parse_args()
    if args.take_profiles:
        stems = list(PROFILE_SPECS) if args.take_profiles == "all" else args.take_profiles.split(",")
        for s in stems:
            if s not in PROFILE_SPECS:
                raise SystemExit(f"unknown workload {s}; known: {', '.join(PROFILE_SPECS)}")
        os.makedirs(args.profile_out, exist_ok=True)
        take_profiles(stems, args.profile_out)
        return
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

    import inputs

    if args.config != "ba200k":
        import torch
        import paper_2101_06192_amd as fc
        dev = torch.device("cuda:0")
        _options(args, fc, dev)
        res = other_config(args, fc, inputs, dev)
        res = {"metric": "trees/s", "n_gpus": 1, "data": "synthetic", "dtype": "u32",
               "higher_is_better": True, "steps": args.steps, "warmup": args.warmup, **res}
        res["launches"] = _launches_of(res)
        print(json.dumps(res), flush=True)
        return

    g = inputs.barabasi_albert(WORKLOAD["n"], WORKLOAD["m_per_vertex"], WORKLOAD["seed"])
    # the CPU leg first: its worker processes are forked before the GPU is used
    cpu = cpu_baseline(g, args.cpu_trees) if args.cpu_trees > 0 else None
    import torch
    import paper_2101_06192_amd as fc
    dev = torch.device("cuda:0")
    _options(args, fc, dev)
    dg = fc.to_device(g, dev)
    trees = WORKLOAD["trees"]
    alpha = WORKLOAD["alpha"]
    torch.cuda.synchronize()

    stats = []

    def step():
        out = fc.farness(dg, alpha=alpha, seed=WORKLOAD["seed"], tau=trees, device=dev,
                         as_torch=True, sampler=args.sampler)
        stats.append(out["stats"])
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = trees / (elapsed / args.steps)

    st = stats[-1]
    walk_steps = st["walk_steps"]
    ms_kernel = sum(s["ms_sample"] for s in stats) / len(stats)
    kernels = {}
    for s in stats:
        for k, v in _kernels_ms(s).items():
            kernels[k] = kernels.get(k, 0.0) + v / len(stats)
    alg_bytes = wilson_bytes(walk_steps, g.n * trees, st["roots"])
    stem = "wilson_lds_ba200k" if st["sampler"] == "wilson_lds" else None
    traffic = traffic_of(stem) if stem else None

    eps_leg = None
    ceiling = None
    if not args.no_eps:
        torch.cuda.synchronize()
        te = time.perf_counter()
        o = fc.diag_estimate(dg, alpha=alpha, eps=0.1, delta=0.1, seed=0, device=dev,
                             as_torch=True, sampler=args.sampler)
        torch.cuda.synchronize()
        eps_leg = {"tau": o["tau"], "ms": 1000.0 * (time.perf_counter() - te)}
        # the random-access rate the sampler runs against: independent random
        # 4-byte loads and atomic adds over a 4 GiB footprint (far beyond caches)
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
        "sampler": st["sampler"],
        "walk_steps_per_s": walk_steps / (ms_per_step / 1000.0),
        "walk_steps_per_tree": walk_steps / trees,
        "trees_in_flight": st["trees_in_flight"],
        "time_to_eps0.1_diag": eps_leg,
        "roofline": roofline_hbm(alg_bytes, ms_kernel, traffic, kernel=" + ".join(kernels),
                                 kernels_ms=kernels, random_access_ceiling=ceiling),
        "cpu_baseline": cpu,
    }
    if traffic and ceiling:
        # the measured line traffic against the line rate of independent random
        # loads over 4 GiB (each fetches a whole 128-byte line): how close the
        # kernel runs to what the memory system gives random gathers
        line_rate = ceiling["random_loads_per_s"] * 128.0
        line["roofline"]["random_line_ceiling_gbs"] = line_rate / 1e9
        line["roofline"]["random_line_ceiling_frac"] = traffic / (ms_kernel / 1000.0) / line_rate
    if args.phase_timing:
        line["phase_ms_per_workgroup"] = _phases(st)
    line["launches"] = {"step": {"kernel_ms": ms_kernel, "algorithmic_bytes": alg_bytes}}
    if not args.no_extras:
        es = max(1, args.extra_steps)
        extras = {}
        t0 = time.perf_counter()
        extras["grid1000"] = leg_grid(fc, inputs, dev, es, 1)
        extras["rmat_batch"] = leg_batch(fc, inputs, dev, es, 1, side=not args.no_side)
        extras["rmat22"] = leg_rmat22(fc, inputs, dev, max(1, es - 1), 1, samplers=("hyb",),
                                      eps=not args.no_eps)
        extras["ba200k_w"] = leg_weighted(fc, inputs, dev, es, 1, eps=not args.no_eps)
        extras["er1000"] = leg_er1000(fc, inputs, dev, es, 1, samplers=("auto",))
        extras["solve"] = leg_solve(fc, inputs, dev, es, 1)
        extras["wall_s"] = time.perf_counter() - t0
        if ceiling:
            _add_line_ceiling(extras, ceiling["random_loads_per_s"] * 128.0)
        line["extras"] = extras
    print(json.dumps(line), flush=True)


def _add_line_ceiling(obj, line_rate):
    """Every roofline inside obj that carries counter traffic gets the same
    comparison as the headline: traffic per second against the line rate of
    independent random loads."""
    if isinstance(obj, dict):
        rf = obj.get("roofline")
        if isinstance(rf, dict) and rf.get("traffic") and rf.get("kernel_ms"):
            rf["random_line_ceiling_frac"] = rf["traffic"] / (rf["kernel_ms"] / 1000.0) / line_rate
        for v in obj.values():
            _add_line_ceiling(v, line_rate)


def _options(args, fc, dev):
    if args.lds_repop is not None:
        fc.set_option("lds_repop", args.lds_repop, dev)
    if args.coop_repop is not None:
        fc.set_option("coop_repop", args.coop_repop, dev)
    if args.phase_timing:
        fc.set_option("phase_timing", 1, dev)


def other_config(args, fc, inputs, dev) -> dict:
    """The non-headline workloads, alone."""
    c, st, wu = args.config, args.steps, args.warmup
    if c == "er1000":
        smp = ("lane", "coop", "lds") if args.sampler == "auto" else (args.sampler,)
        return leg_er1000(fc, inputs, dev, st, wu, smp, phase=args.phase_timing)
    if c == "rmat22":
        smp = ("coop", "hyb") if args.sampler == "auto" else (args.sampler,)
        return leg_rmat22(fc, inputs, dev, st, wu, smp, eps=not args.no_eps,
                          phase=args.phase_timing)
    if c == "ba200k_w":
        return leg_weighted(fc, inputs, dev, st, wu, args.sampler, eps=not args.no_eps,
                            phase=args.phase_timing)
    if c == "grid1000":
        return leg_grid(fc, inputs, dev, st, wu, args.sampler, phase=args.phase_timing)
    if c == "rmat_batch":
        return leg_batch(fc, inputs, dev, st, wu, side=not args.no_side)
    if c == "solve":
        return leg_solve(fc, inputs, dev, st, wu)
    if c == "rank":
        return leg_rank(fc, inputs, dev, st, wu)
    if c == "group":
        res = leg_group(fc, inputs, dev, st, wu, side=not args.no_side)
        if args.no_side:  # every call (k = 1 and k = 50) inverts one 20000 x 20000 matrix
            res["inverse_calls"] = 2 * (st + wu)
        return res
    raise SystemExit(f"unknown config {c}")


if __name__ == "__main__":
    main()
