"""Benchmark: exact Gaussian elimination over F_p on one MI355X.

Headline workload (the largest single-system configuration): one dense
n = 16384 system with 64 right-hand sides over a seeded 31-bit prime field,
entries uniform in [0, p) (seed 3).  A step is one full linac_solve on inputs
already resident in HBM: pack [A | B], eliminate, extract X / rank / pivots /
consistency.  The reported path is the library's AUTO choice (the blocked
int8-MFMA path at this size); the plain path (one fused step kernel per pivot
column, scalar mulmod) is timed once on the same input and reported beside
it.  The metric counts 2 n^3 / 3 operations per square system (right-hand
sides excluded).

Beside the headline the same JSON line carries the other workloads under
"other_configs": c1 (n = 256, latency in microseconds per solve and per pivot
step), c2 (n = 8192, 16 right-hand sides, AUTO and plain), c4 (4096 uneven
systems in one persistent launch replayed from a hipGraph, systems/s, with the
same systems solved one by one on the plain path) and c5 (64 instances of a
12000 x 10000 shared-sparsity-pattern matrix, full RREF).  "cpu_baseline" is
the C oracle timed on this host on a bounded sample of the headline
distribution, plus one single-threaded n = 2048 run.

    python bench.py [--config c3|c1|c2|c4|c5] [--path auto|plain|int8|fp64]
                    [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]

Per-kernel rooflines come from one extra instrumented solve in which the
library records a HIP event pair around every hot-kernel launch on the stream
that kernel runs on (outside the timed steps, so event recording does not
slow them):
  step          plain path, HBM-bound: 8 algorithmic bytes per element update
                (int32 read + write), peak 8000 GB/s;
  leaf/trail    blocked path, int8 MFMA: 32 int8 operations per mod-p
  products      multiply-add (16 limb products, 2 ops each), peak 5000 TOP/s
                (the leaves' pivot selections and operand builds are listed
                by time only);
  select        vector ALU (FP64): the leaf's pivot selection eliminates its
                first chunk of 32 candidate rows fraction-free, one lazy
                multiply-subtract pair (13 FP64 instructions) per element
                update; peak 256 CU x 64 lanes x 2.4 GHz / 13 = 3.02e12
                updates/s.  One workgroup runs the chain of 32 dependent
                pivots, so this kernel is bound by that chain's latency, far
                below the chip's ALU peak;
  batched       a system is reduced in passes of 16 pivot columns; each pass
                streams the rows that are still candidates (plus its own
                pivot rows, written once) from the first 16-aligned column
                after the pass: read and write, 8 bytes per element, counted
                for a full-rank system.  That pass traffic against 8000 GB/s
                is one roof; the other is the FP64 matrix cores, where one
                element update (one pivot applied to one entry) is 2 FMAs of
                an exact split product, 4 flops against 78.6 TFLOP/s.  The
                bound reported is the nearer of the two, the other beside it.
  leaf chain    the sum of the leaves' selection and product launches per
                solve and per leaf (with the leaf pipeline a launch runs one
                leaf's product beside the next leaf's first selection, and its
                time appears in both the leaf-product and selection records).
The headline "roofline" is the kernel with the largest total time.
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
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
I8_PEAK_TOPS = 5000.0
FP64_PEAK_TFLOPS = 78.6
BATCHED_PB = 16  # pivot columns per pass of the batched kernel
SELECT_UPDATES_PEAK = 256 * 64 * 2.4e9 / 13.0  # lazy FP64 updates/s
LEAF = 32
PROFILES = os.path.join(ROOT, "profiles")


def batched_pass_model(m: int, n: int, k: int):
    """(bytes, updates) of the batched kernel's row updates on a full-rank
    m x n system with k right-hand sides: the pass at pivot columns j0..
    rewrites the rows still without a pivot and writes its own pivot rows,
    from the first 16-aligned column after the pass (the right-hand sides
    included); each rewritten element takes one update per pivot of the
    pass."""
    ncols, rank, nbytes, upd = n + k, 0, 0, 0
    for j0 in range(0, n, BATCHED_PB):
        if rank >= m:
            break
        npv = min(BATCHED_PB, n - j0, m - rank)
        width = ncols - (min(j0 + BATCHED_PB, n) & ~15)
        cand = m - rank - npv
        nbytes += 8 * cand * width + 4 * npv * width
        upd += cand * width * npv
        rank += npv
    return nbytes, upd


def gj_updates(m: int, n: int, ncols: int) -> int:
    """Element updates of Gauss-Jordan on an m x ncols matrix with n pivot
    columns: step j rewrites every row but the pivot row from column j on."""
    steps = min(m, n)
    return sum((m - 1) * (ncols - j) for j in range(steps))


def metric_ops(n: int) -> float:
    return 2.0 * n ** 3 / 3.0


def rect_metric_ops(m: int, n: int, r: int) -> float:
    """2(mnr - (m+n) r^2 / 2 + r^3 / 3): the square formula for rank-r m x n."""
    return 2.0 * (m * n * r - (m + n) * r * r / 2.0 + r ** 3 / 3.0)


def blocked_work(m: int, n: int, ncols: int, panel: int, forward: bool = False):
    """Algorithmic work of the two-level blocked path on a full-rank system:
    mod-p multiply-adds of the leaf products (K = leaf width, N = panel width +
    leaf width: the leaf's own columns, the panel columns after it and the
    transform block up to it) and of the trailing products (K = panel width, N
    = trailing columns), over every row (Gauss-Jordan) or, for a solve
    (forward elimination), over the rows that are not pivots of an earlier
    panel: m - j0 of them at panel j0."""
    leaf_macs = 0
    trail_macs = 0
    for j0 in range(0, n, panel):
        wj = min(panel, n - j0)
        rows = m - min(j0, m) if forward else m
        for l0 in range(0, wj, LEAF):
            wl = min(LEAF, wj - l0)
            leaf_macs += rows * (wj + wl) * wl
        trail_macs += rows * (ncols - j0 - wj) * wj
    return leaf_macs, trail_macs


def select_updates(n: int, panel: int) -> int:
    """Element updates of the leaves' first-chunk eliminations on a full-rank
    system: a leaf of wl columns takes wl pivots in a chunk of 32 rows, and
    each pivot rewrites the 31 other rows over the wl - 1 leaf columns after it
    and the transform columns before it (wl - 1 in all)."""
    total = 0
    for j0 in range(0, n, panel):
        wj = min(panel, n - j0)
        for l0 in range(0, wj, LEAF):
            wl = min(LEAF, wj - l0)
            total += wl * 31 * (wl - 1)
    return total


def kernel_source_hash(names) -> str:
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2605_25863_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, src_hash: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when absent or taken on a different kernel source."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != src_hash:
        return None
    return d.get("bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_seconds(n: int, k: int, threads: int = 0) -> float:
    """Wall time of the C oracle's Gauss-Jordan on one seeded dense n x n
    system of the c3 distribution with k right-hand sides (generation
    excluded)."""
    import oracle
    import workloads
    A, B, p = workloads.config("c3", n=n)
    M = np.concatenate([A.astype(np.uint64), B.astype(np.uint64)[:, :k]], axis=1)
    t0 = time.perf_counter()
    oracle.gauss_jordan(M, n, p, impl="c", threads=threads)
    return time.perf_counter() - t0


def cpu_baseline(target_s: float = 15.0, single_thread: bool = True):
    """The C oracle (OpenMP over the rows of a step) on a bounded sample of the
    headline workload: dense systems of the c3 distribution (seed 3, its
    seeded 31-bit prime, 64 right-hand sides), calibrated at n = 1024 and then
    run once at the size that takes about target_s seconds.  Beside it, one
    single-threaded run at n = 2048 without right-hand sides, the size and
    shape of the paper's single-thread CPU comparator (Sec. 4.1, Table 1)."""
    import oracle
    threads = oracle.max_threads()
    t1 = _oracle_seconds(1024, 64)
    rate = gj_updates(1024, 1024, 1024 + 64) / t1
    n = 1024
    for cand in range(1536, 8193, 512):
        if gj_updates(cand, cand, cand + 64) / rate <= target_s:
            n = cand
    t = _oracle_seconds(n, 64) if n != 1024 else t1
    rec = {"value": round(metric_ops(n) / t / 1e9, 3), "unit": "GOP/s", "cores": threads,
           "kind": "oracle",
           "sample": f"C oracle Gauss-Jordan (uint64, %, OpenMP over the rows of a step, "
                     f"{threads} threads) on one dense n={n} system of the headline "
                     f"distribution (seed 3, its 31-bit prime, 64 right-hand sides), "
                     f"{t:.2f} s; the headline system itself (n=16384) would take about "
                     f"{gj_updates(16384, 16384, 16448) / (gj_updates(n, n, n + 64) / t) / 60:.0f} "
                     f"min at this rate",
           "seconds": round(t, 3), "n": n, "cpu_model": _cpu_model(),
           "affinity_cpus": len(os.sched_getaffinity(0)),
           "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    if single_thread:
        ts = _oracle_seconds(2048, 0, threads=1)
        # the paper's single-thread CPU fit (Sec. 4.1, Table 1): a3 x^3 + a2 x^2 + ...
        fit = 1.76e-9 * 2048 ** 3 + 1.13e-6 * 2048 ** 2 + 1.92e-15 * 2048 + 7.61e-12
        rec["single_thread_n2048"] = {
            "seconds": round(ts, 3), "gop_per_s": round(metric_ops(2048) / ts / 1e9, 4),
            "threads": 1, "shape": "2048 x 2048, no right-hand side (RREF)",
            "paper_single_thread_fit_s": round(fit, 2)}
    if threads > 1:
        # restore the full thread count for later callers in this process
        _oracle_seconds(64, 0, threads=threads)
    return rec


PATHS = {"auto": 0, "plain": 1, "int8": 2, "fp64": 3}
KERNEL_SOURCES = ["plain.hip", "blocked.hip", "leaf.hip", "leafprod.h", "field.h"]


def _resolved_plan(lx, m, n, path_name, panel):
    """(path name, panel width) the library takes for this shape and request."""
    pth, pw = lx.plan(m, n, PATHS[path_name], panel)
    return {v: k for k, v in PATHS.items() if k != "auto"}[pth], pw


def _rooflines(kinds, m, n, ncols, path_name, panel, src_hash, workload):
    out = {}
    if path_name == "plain":
        upd = gj_updates(m, n, ncols)
        if "step" in kinds:
            nl, ms = kinds["step"]
            out["step"] = {"bound": "hbm", "kernel": "plain_step_kernel", "launches": nl,
                           "avg_launch_us": ms * 1e3 / nl,
                           "algorithmic_bytes_per_launch": 8.0 * upd / nl,
                           "achieved": 8.0 * upd / (ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s"}
    else:
        # a solve with right-hand sides runs forward elimination on the int8 path
        # from the tuned size on
        fwd = path_name == "int8" and ncols > n and min(m, n) >= _tuned("forward_min", 12288)
        leaf_macs, trail_macs = blocked_work(m, n, ncols, panel, forward=fwd)
        per_mac_ops, peak, unit = (32.0, I8_PEAK_TOPS, "TOP/s") if path_name == "int8" else \
            (2.0, FP64_PEAK_TFLOPS, "TFLOP/s")
        int8 = path_name == "int8"
        # With the leaf pipeline a fused launch ("leaf_fused") runs a leaf's product on
        # every row but the next leaf's first chunk beside that leaf's first
        # selection, so its time is counted in both of those records (each then
        # bounds its kernel's own time from above); "leaf_chain" is the total.
        def merged(*names):
            got = [kinds[k] for k in names if k in kinds]
            return (sum(c for c, _ in got), sum(t for _, t in got)) if got else None
        for kind, macs, kname, parts in (("leaf_product", leaf_macs,
                                          "leaf_product_i8_kernel (leaf transform)" if int8
                                          else "gemm_f64_kernel (leaf transform)",
                                          ("leaf_product", "leaf_fused")),
                                         ("trail_product", trail_macs,
                                          ("gemm_i8_kernel" if int8 else "gemm_f64_kernel")
                                          + " (trailing update)", ("trail_product",))):
            got = merged(*parts)
            if got:
                nl, ms = got
                out[kind] = {"bound": "mfma", "kernel": kname,
                             "launches": nl, "avg_launch_us": ms * 1e3 / nl,
                             "algorithmic_ops_per_launch": per_mac_ops * macs / nl,
                             "achieved": per_mac_ops * macs / (ms / 1e3) / 1e12, "peak": peak,
                             "unit": unit, "time_of": list(parts), "total_ms": ms}
        got = merged("select", "leaf_fused")
        if got:
            nl, ms = got
            upd = select_updates(n, panel)
            out["select"] = {"bound": "alu", "kernel": "leaf_select_kernel (first chunk, then "
                                                       "the tree or Y launch)",
                             "limiter": "latency of the dependent pivot chain in one workgroup",
                             "launches": nl, "avg_launch_us": ms * 1e3 / nl,
                             "algorithmic_updates_per_launch": upd / nl,
                             "achieved": upd / (ms / 1e3) / 1e9,
                             "peak": SELECT_UPDATES_PEAK / 1e9, "unit": "Gupdates/s",
                             "time_of": ["select", "leaf_fused"], "total_ms": ms}
        chain = merged("select", "leaf_product", "leaf_fused")
        if chain:
            leaves = sum(-(-min(panel, n - j0) // LEAF) for j0 in range(0, n, panel))
            out["leaf_chain"] = {"bound": "latency", "kernel": "leaf selections and products",
                                 "launches": chain[0], "avg_launch_us": chain[1] * 1e3 / chain[0],
                                 "leaves": leaves, "us_per_leaf": round(chain[1] * 1e3 / leaves, 2),
                                 "achieved": per_mac_ops * leaf_macs / (chain[1] / 1e3) / 1e12,
                                 "peak": peak, "unit": unit,
                                 "time_of": ["select", "leaf_product", "leaf_fused"],
                                 "total_ms": chain[1]}
    for name, r in out.items():
        r["frac"] = float(f"{r['achieved'] / r['peak']:.3g}")
        r["achieved"] = float(f"{r['achieved']:.4g}")
        r["peak"] = float(f"{r['peak']:.4g}")
        r["avg_launch_us"] = round(r["avg_launch_us"], 3)
        r["total_ms"] = round(r["total_ms"] if "total_ms" in r else kinds[name][1], 3)
        r["traffic"] = measured_traffic(r["kernel"].split()[0], workload, src_hash)
    return out


def _free_cuda():
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def bench_dense(config: str, steps: int, warmup: int, path_name_req: str = "auto",
                panel_req: int = 0, n_override=None, plain_reps: int = 1, plain_warmup: int = 0,
                instrument: bool = True):
    """One dense system of workload c1..c3: linac_solve on the AUTO (or
    requested) path, timed over `steps` calls after `warmup`; the plain path on
    the same input beside it (`plain_reps` calls, 0 to skip)."""
    import torch
    import paper_2605_25863_amd as lx
    import workloads

    A, B, p = workloads.config(config, n=n_override)
    m, n = A.shape
    k = B.shape[1]
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A.astype(np.int32)).to(dev)
    Bt = torch.from_numpy(B.astype(np.int32)).to(dev)
    del A, B
    out = (torch.empty((n, k), dtype=torch.int32, device=dev),
           torch.zeros(1, dtype=torch.int32, device=dev),
           torch.empty(min(m, n), dtype=torch.int32, device=dev),
           torch.empty(k, dtype=torch.uint8, device=dev))
    stream = torch.cuda.current_stream()
    path_name, panel = _resolved_plan(lx, m, n, path_name_req, panel_req)
    path = PATHS[path_name]
    ws = torch.empty(lx.solve_workspace_bytes(m, n, k, path, panel_req), dtype=torch.uint8,
                     device=dev)

    def timed_solves(path, ws, steps, warmup):
        for _ in range(warmup):
            lx.solve(At, Bt, p, path=path, out=out, workspace=ws, stream=stream,
                     panel_width=panel_req)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lx.solve(At, Bt, p, path=path, out=out, workspace=ws, stream=stream,
                     panel_width=panel_req)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_step = timed_solves(path, ws, steps, warmup)
    rank = int(out[1].item())
    assert rank == min(m, n), f"unexpected rank {rank}"
    value = metric_ops(n) / t_step / 1e9
    rec = {"value": round(value, 3), "unit": "GOP/s", "ms_per_step": round(t_step * 1e3, 3),
           "steps": steps, "warmup": warmup,
           "dtype": "u32" if path_name == "plain" else ("i8-mfma/u32" if path_name == "int8"
                                                         else "f64-mfma/u32"),
           "config": {"workload": f"{config}: one dense n={n} system, {k} right-hand sides, "
                                  f"p={p}, {path_name} path", "n": n, "k": k, "p": p,
                      "path": path_name, "panel": panel,
                      "seed": workloads.CONFIGS[config]["seed"]}}
    if instrument:
        # one extra solve with an event pair around every hot-kernel launch
        cap = n + 4 * (n // 32 + 8) + 64
        lt = lx.LaunchTimes(cap)
        lx.solve(At, Bt, p, path=path, out=out, workspace=ws, stream=stream,
                 panel_width=panel_req, per_launch=lt)
        kinds = lt.by_kind()
        src_hash = kernel_source_hash(KERNEL_SOURCES)
        roofs = _rooflines(kinds, m, n, n + k, path_name, panel, src_hash, config)
        # the dominant kernel (the leaf chain is a sum of kernels, not one)
        single = [name for name in roofs if name != "leaf_chain"]
        dominant = max(single, key=lambda name: roofs[name]["total_ms"]) if single else None
        rec["roofline"] = roofs.get(dominant)
        rec["rooflines"] = roofs
        rec["kernel_ms_by_kind"] = {kk: round(v[1], 3) for kk, v in kinds.items()}
    if path_name != "plain" and plain_reps > 0:
        del ws
        _free_cuda()
        wsp = torch.empty(lx.solve_workspace_bytes(m, n, k, lx.PATH_PLAIN), dtype=torch.uint8,
                          device=dev)
        tp = timed_solves(lx.PATH_PLAIN, wsp, plain_reps, plain_warmup)
        assert int(out[1].item()) == min(m, n)
        rec["plain"] = {"value": round(metric_ops(n) / tp / 1e9, 3), "unit": "GOP/s",
                        "ms_per_step": round(tp * 1e3, 3), "reps": plain_reps,
                        "speedup_of_reported_path": round(tp / t_step, 2)}
        del wsp
    del At, Bt, out
    _free_cuda()
    return rec


def bench_c1_latency(reps: int = 50):
    """c1 (n = 256, one right-hand side, p = 2^31 - 1): latency of one solve on
    the AUTO path, in microseconds, and per pivot step."""
    import torch
    import paper_2605_25863_amd as lx
    import workloads

    A, B, p = workloads.config("c1")
    n, k = A.shape[1], B.shape[1]
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A.astype(np.int32)).to(dev)
    Bt = torch.from_numpy(B.astype(np.int32)).to(dev)
    out = (torch.empty((n, k), dtype=torch.int32, device=dev),
           torch.zeros(1, dtype=torch.int32, device=dev),
           torch.empty(n, dtype=torch.int32, device=dev),
           torch.empty(k, dtype=torch.uint8, device=dev))
    path_name, _ = _resolved_plan(lx, n, n, "auto", 0)
    ws = torch.empty(lx.solve_workspace_bytes(n, n, k), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    timer = lx.HipTimer()
    times = []
    for i in range(reps + 5):
        timer.record_begin(ctypes_stream(stream))
        lx.solve(At, Bt, p, out=out, workspace=ws, stream=stream)
        timer.record_end(ctypes_stream(stream))
        t = timer.elapsed_ms()
        if i >= 5:
            times.append(t)
    us = float(np.median(times)) * 1e3
    return {"us_per_solve": round(us, 2), "us_per_step": round(us / n, 3),
            "gop_per_s": round(metric_ops(n) / (us * 1e-6) / 1e9, 3), "path": path_name,
            "reps": reps, "timing": "HIP events on the solve's stream, median",
            "workload": "c1: one dense n=256 system, 1 right-hand side, p=2^31-1, seed 1"}


def ctypes_stream(stream):
    import ctypes
    return ctypes.c_void_p(stream.cuda_stream)


def bench_batched(steps: int = 10, warmup: int = 2, plain_compare: bool = True):
    """The 4096-system workload: systems/s of the batched persistent launch
    (graph replay) next to the same systems solved one by one on the plain
    path."""
    import torch
    import paper_2605_25863_amd as lx
    import workloads

    systems = workloads.batched_systems()
    prep = lx.prepare_batched(systems)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        lx.solve_batched(systems, prepared=prep, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lx.solve_batched(systems, prepared=prep, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / steps
    sps = len(systems) / (ms_per_step / 1e3)
    ops = sum(metric_ops(s["n"]) for s in systems)
    model = [batched_pass_model(s["n"], s["n"], s["k"]) for s in systems]
    pass_bytes = sum(b for b, _ in model)
    upd = sum(u for _, u in model)
    lt = lx.LaunchTimes(4)
    lx.solve_batched(systems, prepared=prep, stream=stream, per_launch=lt)
    kinds = lt.by_kind()
    nl, kms = kinds["batched"]
    secs = kms / 1e3
    hbm = {"bound": "hbm", "achieved": round(pass_bytes / secs / 1e9, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(pass_bytes / secs / 1e9 / HBM_PEAK_GBS, 4),
           "algorithmic_bytes_per_launch": pass_bytes / nl}
    mfma = {"bound": "mfma", "achieved": round(4 * upd / secs / 1e12, 2),
            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(4 * upd / secs / 1e12 / FP64_PEAK_TFLOPS, 4),
            "algorithmic_flops_per_launch": 4 * upd / nl, "dtype": "fp64"}
    near, other = (hbm, mfma) if hbm["frac"] >= mfma["frac"] else (mfma, hbm)
    roof = dict(near)
    roof.update({"kernel": "batched_kernel", "launches": nl,
                 "avg_launch_us": round(kms * 1e3 / nl, 3),
                 "traffic": measured_traffic("batched_kernel", "c4",
                                             kernel_source_hash(["batched.hip", "field.h"])),
                 other["bound"]: {kk: vv for kk, vv in other.items() if kk != "bound"}})
    rec = {"metric": "systems/s batched (4096 uneven systems, one persistent launch)",
           "value": round(sps, 1), "unit": "systems/s", "steps": steps, "warmup": warmup,
           "ms_per_step": round(ms_per_step, 3), "dtype": "u32",
           "config": {"workload": "c4: 4096 systems, n~U{32..512}, k~U{1..8}, a seeded 31-bit "
                                  "prime each, 205 rank deficient"},
           "gop_per_s": round(ops / (ms_per_step / 1e3) / 1e9, 2),
           "roofline": roof}
    if plain_compare:
        # the same systems, one linac_solve each on the plain path
        wss = []
        for it in prep["items"]:
            mm, nn = it["A"].shape
            kk = it["B"].shape[1]
            wss.append(torch.empty(lx.solve_workspace_bytes(mm, nn, kk, lx.PATH_PLAIN),
                                   dtype=torch.uint8, device="cuda:0"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it, ws in zip(prep["items"], wss):
            lx.solve(it["A"], it["B"], it["p"], path=lx.PATH_PLAIN, workspace=ws, stream=stream,
                     out=(it["X"], it["rank"], it["pivots"], it["cons"][: it["X"].shape[1]]))
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        rec["plain_systems_per_s"] = round(len(systems) / tp, 1)
        rec["speedup_vs_plain"] = round(sps / (len(systems) / tp), 2)
        del wss
    del prep
    _free_cuda()
    return rec


def bench_sparse_pattern(count: int = 64, steps: int = 2, warmup: int = 1,
                         path_name: str = "int8", panel: int = 0):
    """c5: `count` instances of a 12000 x 10000 sparse-pattern matrix (rank
    about 9500), full RREF with pivot columns, p = 2^31 - 1, all resident in
    HBM.  A step is one linac_rref_batched call over every instance (the
    working copies are restored from pristine device copies outside the timed
    region)."""
    import torch
    import paper_2605_25863_amd as lx
    import workloads

    dev = torch.device("cuda:0")
    mats = [A for _, A in workloads.sparse_pattern_instances_torch(dev, count=count)]
    m, n = mats[0].shape
    p = workloads.MERSENNE31
    path = PATHS[path_name]
    work = [torch.empty_like(A) for A in mats]
    ws = torch.empty(lx.rref_batched_workspace_bytes([(m, n)] * count, path, panel),
                     dtype=torch.uint8, device=dev)
    outs = [(torch.zeros(1, dtype=torch.int32, device=dev),
             torch.empty(min(m, n), dtype=torch.int32, device=dev)) for _ in range(count)]
    stream = torch.cuda.current_stream()
    ranks = []

    def one_pass(collect=False):
        for A, Wk in zip(mats, work):
            Wk.copy_(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lx.rref_batched(work, p, inplace=True, path=path, panel_width=panel, stream=stream,
                        workspace=ws, outs=outs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if collect:
            ranks.extend(int(r.item()) for r, _ in outs)
        return dt

    for _ in range(warmup):
        one_pass()
    ts = [one_pass(collect=(i == 0)) for i in range(steps)]
    t = float(np.median(ts))
    ops = sum(rect_metric_ops(m, n, rr) for rr in ranks)
    rec = {"metric": "mod-p elim GOP/s (2n^3/3 convention, rank-r rectangular)",
           "value": round(ops / t / 1e9, 3), "unit": "GOP/s", "steps": steps, "warmup": warmup,
           "ms_per_step": round(t * 1e3, 3), "dtype": "i8-mfma/u32",
           "data": "synthetic (seeded shared sparsity pattern, stand-in for sample-point systems)",
           "config": {"workload": f"c5: {count} instances of {m}x{n}, 200 nnz per independent "
                                  f"row, 2500 dependent rows, p=2^31-1, full RREF, "
                                  f"{path_name} path, one linac_rref_batched call",
                      "instances": count, "lanes": _rref_lanes(),
                      "ranks": sorted(set(ranks))},
           "ms_per_instance": round(t * 1e3 / count, 3)}
    del mats, work, ws
    _free_cuda()
    return rec


def bench_load_matrix(reps: int = 20):
    """System construction (Sec. 3.3): the 20000 x 20000 monomial matrix of the
    construction workload (48 basis variables, degrees 1..12 padded to 12), one
    linac_load_matrix launch timed with HIP events on its stream.  Roofs: the
    output write (4 bytes per entry) against HBM, and the FP64 chain (d - 1
    modular products per entry, 6 FP64 instructions each) against 256 CU x 64
    lanes x 2.4 GHz."""
    import torch
    import paper_2605_25863_amd as lx
    import workloads
    cfg = workloads.LM_CONFIG
    bases, L, p = workloads.monomial_system(**cfg)
    dev = torch.device("cuda:0")
    Bt = torch.from_numpy(bases.astype(np.int32)).to(dev)
    Lt = torch.from_numpy(L).to(dev)
    A = torch.empty((cfg["nrows"], cfg["ncols"]), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        lx.load_matrix(Bt, Lt, p, out=A, stream=stream)
    timer = lx.HipTimer()
    sptr = ctypes_stream(stream)
    timer.record_begin(sptr)
    for _ in range(reps):
        lx.load_matrix(Bt, Lt, p, out=A, stream=stream)
    timer.record_end(sptr)
    t = timer.elapsed_ms() / reps / 1e3
    entries = cfg["nrows"] * cfg["ncols"]
    d = cfg["d"]
    out_bytes = 4.0 * entries + 4.0 * cfg["nrows"] * cfg["nbasis"] + 4.0 * cfg["ncols"] * d
    mulmods = entries * (d - 1)
    alu_peak = 256 * 64 * 2.4e9 / 6.0  # modular products per second
    rec = {"metric": "entries/s (A[r,c] = prod_t bases[r, lindices[c,t]] mod p)",
           "value": round(entries / t, 1), "unit": "entries/s", "ms_per_launch": round(t * 1e3, 4),
           "reps": reps, "dtype": "f64 chain/u32",
           "config": {"workload": f"system construction: {cfg['nrows']} sampling points x "
                                  f"{cfg['ncols']} monomials, {cfg['nbasis']} basis variables, "
                                  f"degree {d}, p=2^31-1, seed {cfg['seed']}"},
           "roofline": {"bound": "alu", "kernel": "load_matrix_kernel<16, true>",
                        "achieved": round(mulmods / t / 1e9, 2),
                        "peak": round(alu_peak / 1e9, 1), "unit": "G modmul/s",
                        "frac": round(mulmods / t / alu_peak, 4),
                        "hbm": {"achieved": round(out_bytes / t / 1e9, 1), "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(out_bytes / t / 1e9 / HBM_PEAK_GBS, 4)},
                        "traffic": None}}
    del Bt, Lt, A
    _free_cuda()
    return rec


def bench_colstep(n: int = 2048, k: int = 4, reps: int = 2):
    """The column-step paths: a dense n x n solve over the 62-bit prime
    2^62 - 57 (uint64 residues) and the LUP factorisation of a dense n x n
    matrix over 2^31 - 1, each timed end to end with HIP events."""
    import torch
    import paper_2605_25863_amd as lx
    import workloads
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(21)
    p62 = 4611686018427387847
    A = torch.from_numpy(rng.integers(0, p62, size=(n, n), dtype=np.int64)).to(dev)
    B = torch.from_numpy(rng.integers(0, p62, size=(n, k), dtype=np.int64)).to(dev)
    stream = torch.cuda.current_stream()
    sptr = ctypes_stream(stream)
    out = {}
    lx.solve_u64(A, B, p62, stream=stream)
    timer = lx.HipTimer()
    timer.record_begin(sptr)
    for _ in range(reps):
        X, r, piv, cons = lx.solve_u64(A, B, p62, stream=stream)
    timer.record_end(sptr)
    t = timer.elapsed_ms() / reps / 1e3
    assert int(r.item()) == n
    out["u64_solve"] = {"value": round(metric_ops(n) / t / 1e9, 3), "unit": "GOP/s",
                        "ms_per_solve": round(t * 1e3, 2), "reps": reps,
                        "config": {"workload": f"one dense n={n} system, {k} right-hand sides, "
                                               f"p=2^62-57 (uint64 residues), seed 21"}}
    A32 = torch.from_numpy(workloads.uniform(rng, (n, n), workloads.MERSENNE31).astype(np.int32)).to(dev)
    lx.lup(A32, workloads.MERSENNE31, stream=stream)
    timer.record_begin(sptr)
    for _ in range(reps):
        LU, perm, r, piv = lx.lup(A32, workloads.MERSENNE31, stream=stream)
    timer.record_end(sptr)
    t = timer.elapsed_ms() / reps / 1e3
    assert int(r.item()) == n
    out["lup"] = {"value": round(metric_ops(n) / t / 1e9, 3), "unit": "GOP/s",
                  "ms_per_factorisation": round(t * 1e3, 2), "reps": reps,
                  "config": {"workload": f"LUP of one dense n={n} matrix, p=2^31-1, seed 21"}}
    del A, B, A32
    _free_cuda()
    return out


def _tuned(key: str, default: int) -> int:
    import paper_2605_25863_amd as lx
    try:
        return int(json.load(open(lx.TUNING_FILE)).get(key, default))
    except OSError:
        return default


def _rref_lanes() -> int:
    import paper_2605_25863_amd as lx
    try:
        return int(json.load(open(lx.TUNING_FILE)).get("rref_lanes", 4))
    except OSError:
        return 4


def copy_calibration(mib: int = 1024, reps: int = 3):
    """A plain device copy of a known size, for scaling the FETCH_SIZE /
    WRITE_SIZE hardware counters into bytes (run it under the same rocprofv3
    --pmc command as the kernel being measured)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "reps": reps}), flush=True)


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="workload of the headline line (default c3, the largest single "
                         "system); c1, c2, c4 and c5 are also reported beside it unless "
                         "--no-extras")
    ap.add_argument("--n", type=int, default=None, help="resize the dense workload")
    ap.add_argument("--path", default="auto", choices=list(PATHS))
    ap.add_argument("--panel", type=int, default=0, help="blocked panel width (0 = tuned)")
    ap.add_argument("--instances", type=int, default=64, help="c5 instances")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-compare", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    plain_reps = 0 if args.no_plain_compare else 1
    common = {"n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "data": "synthetic (seeded uniform residues)"}
    if args.config == "c4":
        rec = bench_batched(args.steps, args.warmup, not args.no_plain_compare)
    elif args.config == "c5":
        rec = bench_sparse_pattern(args.instances, args.steps, args.warmup,
                                   "plain" if args.path == "plain" else
                                   ("fp64" if args.path == "fp64" else "int8"), args.panel)
    else:
        _progress(f"{args.config} headline")
        rec = bench_dense(args.config, args.steps, args.warmup, args.path, args.panel, args.n,
                          plain_reps=plain_reps)
        rec["metric"] = "mod-p elim GOP/s (2n^3/3 mulmod-add)"
    out = {"metric": rec.pop("metric"), "value": rec.pop("value"), "unit": rec.pop("unit"),
           "n_gpus": 1, "steps": rec.pop("steps"), "warmup": rec.pop("warmup"),
           "ms_per_step": rec.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": rec.pop("dtype"),
           "data": rec.pop("data", common["data"]), "config": rec.pop("config")}
    out.update(rec)
    if args.config == "c3" and not args.no_extras and args.n is None:
        extras = {}
        _progress("c1 latency")
        extras["c1"] = bench_c1_latency()
        _progress("c2")
        c2 = bench_dense("c2", 5, 1, plain_reps=plain_reps, instrument=False)
        extras["c2"] = c2
        _progress("c4 batch")
        extras["c4"] = bench_batched(10, 2, not args.no_plain_compare)
        _progress("c5 sparse-pattern instances")
        extras["c5"] = bench_sparse_pattern(args.instances, 2, 1)
        _progress("system construction")
        extras["load_matrix"] = bench_load_matrix()
        _progress("64-bit solve and LUP")
        extras.update(bench_colstep())
        out["other_configs"] = extras
    if not args.no_cpu_baseline and args.config in ("c1", "c2", "c3"):
        _progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
