"""Benchmark: exact Gaussian elimination over F_p on one MI355X.

Default workload (the one the metric is quoted on): one dense n = 8192 system
with 16 right-hand sides over a seeded 31-bit prime field, entries uniform in
[0, p), solved by the plain Gauss-Jordan path (one fused step kernel per
pivot column).  A step is one full linac_solve: pack [A | B], 8192
elimination launches, extraction of X / rank / pivots / consistency.  Inputs
are resident in HBM before the timed region.

Prints one JSON line.  The metric counts 2 n^3 / 3 operations per square
system (the LINPACK convention, right-hand sides excluded).

    python bench.py [--steps K] [--warmup W] [--config c2] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def gj_updates(m: int, n: int, ncols: int) -> int:
    """Element updates of Gauss-Jordan on an m x ncols matrix with n pivot
    columns: step j rewrites every row but the pivot row from column j on."""
    steps = min(m, n)
    return sum((m - 1) * (ncols - j) for j in range(steps))


def metric_ops(n: int) -> float:
    return 2.0 * n ** 3 / 3.0


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


def cpu_baseline(target_s: float = 15.0):
    """The C oracle (OpenMP over rows) on a bounded sample of the same workload:
    calibrate at n = 1024, then one run sized for about target_s seconds."""
    import oracle
    import workloads
    threads = oracle.max_threads()

    def run(n):
        A, B, p = workloads.config("c2", n=n)
        M = np.concatenate([A.astype(np.uint64), B.astype(np.uint64)], axis=1)
        t0 = time.perf_counter()
        oracle.gauss_jordan(M, n, p, impl="c")
        return time.perf_counter() - t0

    t1 = run(1024)
    rate = gj_updates(1024, 1024, 1040) / t1
    n = 1024
    for cand in (1536, 2048, 2560, 3072, 3584, 4096):
        if gj_updates(cand, cand, cand + 16) / rate <= target_s:
            n = cand
    t = run(n) if n != 1024 else t1
    return {"value": metric_ops(n) / t / 1e9, "unit": "GOP/s", "cores": threads, "kind": "oracle",
            "sample": f"C oracle Gauss-Jordan (uint64, %, OpenMP over rows) on the same seeded "
                      f"distribution at n={n} with 16 right-hand sides; {t:.2f} s",
            "seconds": round(t, 3), "n": n}


def bench_dense(args):
    import torch
    import paper_2605_25863_amd as lx
    import workloads

    cfg = {"c1": 256, "c2": 8192, "c3": 16384}[args.config]
    n_override = args.n
    A, B, p = workloads.config(args.config, n=n_override)
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
    path = {"plain": lx.PATH_PLAIN, "int8": lx.PATH_BLOCKED_INT8, "auto": lx.PATH_AUTO}[args.path]
    ws = torch.empty(lx.solve_workspace_bytes(m, n, k, path, args.panel), dtype=torch.uint8,
                     device=dev)
    stream = torch.cuda.current_stream()
    timer = lx.HipTimer()
    launches = ctypes.c_int64(0)

    def step(timed):
        lx.solve(At, Bt, p, path=path, out=out, workspace=ws, stream=stream,
                 events=timer if timed else None, launches=launches if timed else None,
                 panel_width=args.panel)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
        kernel_ms.append(timer.elapsed_ms())  # waits for this step's last step kernel
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = metric_ops(n) / (ms_per_step / 1e3) / 1e9

    rank = int(out[1].item())
    assert rank == min(m, n), f"unexpected rank {rank}"

    nl = int(launches.value)
    upd = gj_updates(m, n, n + k)
    alg_bytes_per_launch = 8.0 * upd / max(nl, 1)
    avg_launch_s = (float(np.median(kernel_ms)) / 1e3) / max(nl, 1)
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9
    src_hash = kernel_source_hash(["plain.hip", "field.h"])
    traffic = measured_traffic("plain_step_kernel", args.config, src_hash)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "plain_step_kernel",
                "launches_per_step": nl, "avg_launch_us": round(avg_launch_s * 1e6, 3),
                "algorithmic_bytes_per_launch": round(alg_bytes_per_launch),
                "source_hash": src_hash}
    rec = {
        "metric": "mod-p elim GOP/s (2n^3/3 mulmod-add)",
        "value": round(value, 3),
        "unit": "GOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded uniform residues)",
        "config": {"workload": f"{args.config}: one dense n={n} system, {k} right-hand sides, "
                               f"p={p}, {args.path} Gauss-Jordan",
                   "n": n, "k": k, "p": p, "path": args.path, "seed": {"c1": 1, "c2": 2,
                                                                      "c3": 3}[args.config]},
        "roofline": roofline,
        "kernel_ms_per_step": round(float(np.median(kernel_ms)), 3),
    }
    return rec


def bench_batched(args):
    """The 4096-system workload: systems/s of the batched persistent launch
    (graph replay) next to the same systems solved one by one on the plain
    path."""
    import torch
    import paper_2605_25863_amd as lx
    import workloads

    systems = workloads.batched_systems()
    prep = lx.prepare_batched(systems)
    stream = torch.cuda.current_stream()
    timer = lx.HipTimer()
    for _ in range(args.warmup):
        lx.solve_batched(systems, prepared=prep, stream=stream)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lx.solve_batched(systems, prepared=prep, stream=stream, events=timer)
        kernel_ms.append(timer.elapsed_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    sps = len(systems) / (ms_per_step / 1e3)
    ops = sum(metric_ops(s["n"]) for s in systems)
    upd = sum(gj_updates(s["n"], s["n"], s["n"] + s["k"]) for s in systems)
    rec = {"metric": "systems/s batched (4096 uneven systems, one persistent launch)",
           "value": round(sps, 1), "unit": "systems/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic (seeded uniform residues)",
           "config": {"workload": "c4: 4096 systems, n~U{32..512}, k~U{1..8}, a seeded 31-bit "
                                  "prime each, 205 rank deficient"},
           "gop_per_s": round(ops / (ms_per_step / 1e3) / 1e9, 2),
           "kernel_ms_per_step": round(float(np.median(kernel_ms)), 3),
           "updates_per_s": round(upd / (float(np.median(kernel_ms)) / 1e3) / 1e12, 4)}
    if not args.no_plain_compare:
        # the same systems, one linac_solve each on the plain path
        outs, wss = [], []
        for it in prep["items"]:
            m, n = it["A"].shape
            k = it["B"].shape[1]
            wss.append(torch.empty(lx.solve_workspace_bytes(m, n, k, lx.PATH_PLAIN),
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
    return rec


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--n", type=int, default=None, help="resize the dense workload")
    ap.add_argument("--path", default="plain", choices=["plain", "int8", "auto"])
    ap.add_argument("--panel", type=int, default=0, help="blocked panel width (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-compare", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.config == "c4":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    rec = bench_dense(args)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline()
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
