"""Autotuner: measure the result-neutral choices of the library on this GPU and
write them as the JSON tuning table read by linac_load_tuning.

    python -m paper_2605_25863_amd.tune [--quick] [--out PATH]

It times, on seeded dense systems (entries uniform in [0, p), a seeded 31-bit
prime, 16 right-hand sides):
  * the plain path against the blocked int8 path at growing n, to find the
    crossover "blocked_min";
  * the blocked path at each candidate panel width, per size bucket ("panel"),
    up to n = 16384, where a solve eliminates forward under the default
    forward_min (the plain path is not timed once the crossover is found);
  * the look-ahead switch of the blocked path at the largest size ("lookahead");
  * forward elimination with back-substitution against Gauss-Jordan for blocked
    solves at n = 8192 and 16384 ("forward_min": the smallest size where
    forward elimination wins);
  * the workgroup shape of the int8 leaf product, 2, 3, 6 or 9 blocks of 16
    columns per workgroup, summed over n = 8192 and 16384 ("leaf_blocks");
  * the leaf pipeline (each leaf's product split so that the next leaf's first
    selection runs beside it) on and off, summed likewise ("leaf_pipeline");
  * the batched launch at 1, 2, 3, 4, 6 and 8 resident workgroups per compute
    unit on a batch of uneven systems ("batched_per_cu");
  * the batched RREF (linac_rref_batched) at 1, 2, 3, 4, 6 and 8 stream lanes
    on a batch of sparse-pattern matrices ("rref_lanes").
Every candidate configuration computes the same unique RREF, so the table only
changes speed.  The written file (default: tuning_gfx950.json next to this
module) is loaded by the Python binding at import.
"""

from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning_gfx950.json")
PANELS = (64, 96, 128, 192, 256, 320, 384, 512)


def _time_solve(lx, torch, At, Bt, p, path, panel, reps):
    m, n = At.shape
    k = Bt.shape[1]
    ws = torch.empty(lx.solve_workspace_bytes(m, n, k, path, panel), dtype=torch.uint8,
                     device="cuda")
    out = (torch.empty((n, k), dtype=torch.int32, device="cuda"),
           torch.zeros(1, dtype=torch.int32, device="cuda"),
           torch.empty(min(m, n), dtype=torch.int32, device="cuda"),
           torch.empty(k, dtype=torch.uint8, device="cuda"))
    lx.solve(At, Bt, p, path=path, panel_width=panel, out=out, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        lx.solve(At, Bt, p, path=path, panel_width=panel, out=out, workspace=ws)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def tune(quick: bool = False):
    import torch
    import paper_2605_25863_amd as lx
    import workloads

    systems_cache = {}

    def dense(seed, n):
        # the same seeded system serves every sweep at its size (seconds to draw at n = 16384)
        if (seed, n) not in systems_cache:
            systems_cache[(seed, n)] = workloads.dense_system(seed=seed, n=n, k=16)
        return systems_cache[(seed, n)]

    lx.load_tuning(None)  # measure from the built-in defaults
    sizes = (256, 512, 1024, 2048, 4096) if quick else (256, 512, 1024, 2048, 4096, 8192, 16384)
    reps = 2 if quick else 3
    report = {"crossover": {}, "panels": {}}
    blocked_min = None
    rules = []
    for n in sizes:
        A, B, p = dense(1000 + n, n)
        At = torch.from_numpy(A.astype(np.int32)).cuda()
        Bt = torch.from_numpy(B.astype(np.int32)).cuda()
        # past the crossover the plain path only costs time (seconds at n = 16384)
        t_plain = (None if blocked_min is not None and n > 8192 else
                   _time_solve(lx, torch, At, Bt, p, lx.PATH_PLAIN, 0, reps))
        per_panel = {}
        for w in PANELS:
            if w > n:
                continue
            per_panel[w] = _time_solve(lx, torch, At, Bt, p, lx.PATH_BLOCKED_INT8, w, reps)
        best_w = min(per_panel, key=per_panel.get)
        report["crossover"][n] = {"plain_s": t_plain, "blocked_s": per_panel[best_w]}
        report["panels"][n] = per_panel
        if blocked_min is None and t_plain is not None and per_panel[best_w] < t_plain:
            blocked_min = n
        rules.append({"n_max": n, "panel": best_w})
        plain_txt = "not timed" if t_plain is None else f"{t_plain * 1e3:.2f} ms"
        print(f"n={n}: plain {plain_txt}, best panel {best_w}: "
              f"{per_panel[best_w] * 1e3:.2f} ms", flush=True)
        del At, Bt
    # the largest measured size covers everything above it
    rules[-1]["n_max"] = 1 << 30
    # look-ahead (trailing remainder on a side stream) at the largest size
    n = sizes[-1]
    A, B, p = dense(1000 + n, n)
    At = torch.from_numpy(A.astype(np.int32)).cuda()
    Bt = torch.from_numpy(B.astype(np.int32)).cuda()
    per_la = {}
    for la in (0, 1):
        lx.load_tuning(json.dumps({"lookahead": la}))
        per_la[la] = _time_solve(lx, torch, At, Bt, p, lx.PATH_BLOCKED_INT8, rules[-1]["panel"],
                                 reps)
        print(f"n={n} lookahead={la}: {per_la[la] * 1e3:.2f} ms", flush=True)
    lookahead = min(per_la, key=per_la.get)
    # forward elimination + back-substitution against Gauss-Jordan (solves only)
    fwd_sizes = (4096, 8192) if quick else (8192, 16384)
    per_fwd = {}
    forward_min = 1 << 30
    for n in fwd_sizes:
        A, B, p = dense(2000 + n, n)
        At = torch.from_numpy(A.astype(np.int32)).cuda()
        Bt = torch.from_numpy(B.astype(np.int32)).cuda()
        panel = next(r["panel"] for r in rules if n <= r["n_max"])
        res = {}
        for fm in (0, 1 << 30):
            lx.load_tuning(json.dumps({"lookahead": lookahead, "forward_min": fm}))
            res["forward" if fm == 0 else "gauss_jordan"] = _time_solve(
                lx, torch, At, Bt, p, lx.PATH_BLOCKED_INT8, panel, reps)
        per_fwd[n] = res
        print(f"n={n}: forward {res['forward'] * 1e3:.2f} ms, Gauss-Jordan "
              f"{res['gauss_jordan'] * 1e3:.2f} ms", flush=True)
        if res["forward"] < res["gauss_jordan"] and forward_min == 1 << 30:
            forward_min = n
        del At, Bt
    # leaf-product workgroup shape, one value for all sizes: the smallest total
    per_leaf = {}
    for lb in (2, 3, 6, 9):
        lx.load_tuning(json.dumps({"lookahead": lookahead, "forward_min": forward_min,
                                   "leaf_blocks": lb}))
        per_leaf[lb] = {}
        for n in fwd_sizes:
            A, B, p = dense(2000 + n, n)
            At = torch.from_numpy(A.astype(np.int32)).cuda()
            Bt = torch.from_numpy(B.astype(np.int32)).cuda()
            panel = next(r["panel"] for r in rules if n <= r["n_max"])
            per_leaf[lb][n] = _time_solve(lx, torch, At, Bt, p, lx.PATH_BLOCKED_INT8, panel, reps)
            del At, Bt
        print(f"leaf_blocks={lb}: " + ", ".join(f"n={n} {t * 1e3:.2f} ms"
                                                 for n, t in per_leaf[lb].items()), flush=True)
    leaf_blocks = min(per_leaf, key=lambda lb: sum(per_leaf[lb].values()))
    # leaf pipeline (the next leaf's first selection beside the product) on or off
    per_pipe = {}
    for lp in (0, 1):
        lx.load_tuning(json.dumps({"lookahead": lookahead, "forward_min": forward_min,
                                   "leaf_blocks": leaf_blocks, "leaf_pipeline": lp}))
        per_pipe[lp] = {}
        for n in fwd_sizes:
            A, B, p = dense(2000 + n, n)
            At = torch.from_numpy(A.astype(np.int32)).cuda()
            Bt = torch.from_numpy(B.astype(np.int32)).cuda()
            panel = next(r["panel"] for r in rules if n <= r["n_max"])
            per_pipe[lp][n] = _time_solve(lx, torch, At, Bt, p, lx.PATH_BLOCKED_INT8, panel, reps)
            del At, Bt
        print(f"leaf_pipeline={lp}: " + ", ".join(f"n={n} {t * 1e3:.2f} ms"
                                                   for n, t in per_pipe[lp].items()), flush=True)
    leaf_pipeline = min(per_pipe, key=lambda lp: sum(per_pipe[lp].values()))
    # batched: resident workgroups per CU
    systems = workloads.batched_systems(seed=4, count=512 if quick else 4096)
    prep = lx.prepare_batched(systems)
    per_cu = {}
    for c in (1, 2, 3, 4, 6, 8):
        lx.load_tuning(json.dumps({"batched_per_cu": c}))
        lx.solve_batched(systems, prepared=prep)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            lx.solve_batched(systems, prepared=prep)
        torch.cuda.synchronize()
        per_cu[c] = (time.perf_counter() - t0) / reps
        print(f"batched per_cu={c}: {per_cu[c] * 1e3:.2f} ms", flush=True)
    best_cu = min(per_cu, key=per_cu.get)
    # batched RREF: stream lanes, on sparse-pattern matrices (the tuned panels)
    count = 8 if quick else 16
    mats = [A for _, A in workloads.sparse_pattern_instances_torch(torch.device("cuda"), count=count)]
    pm = workloads.MERSENNE31
    work = [torch.empty_like(A) for A in mats]
    base = {"blocked_min": blocked_min or sizes[-1] * 2, "panel": rules, "lookahead": lookahead,
            "forward_min": forward_min, "leaf_blocks": leaf_blocks, "leaf_pipeline": leaf_pipeline}
    per_lanes = {}
    for lanes in (1, 2, 3, 4, 6, 8):
        lx.load_tuning(json.dumps(dict(base, rref_lanes=lanes)))
        ws = torch.empty(lx.rref_batched_workspace_bytes([tuple(A.shape)] * count), dtype=torch.uint8,
                         device="cuda")
        ts = []
        for rep in range(reps + 1):
            for A, Wk in zip(mats, work):
                Wk.copy_(A)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lx.rref_batched(work, pm, inplace=True, workspace=ws)
            torch.cuda.synchronize()
            if rep:  # the first pass warms up
                ts.append(time.perf_counter() - t0)
        per_lanes[lanes] = float(np.median(ts))
        del ws
        print(f"rref_batched lanes={lanes}: {per_lanes[lanes] * 1e3:.2f} ms "
              f"({count} matrices)", flush=True)
    best_lanes = min(per_lanes, key=per_lanes.get)
    del mats, work
    systems_cache.clear()
    table = {"arch": "gfx950", "blocked_min": blocked_min or sizes[-1] * 2,
             "panel": rules, "batched_per_cu": best_cu, "lookahead": lookahead,
             "rref_lanes": best_lanes, "forward_min": forward_min, "leaf_blocks": leaf_blocks,
             "leaf_pipeline": leaf_pipeline,
             "measured": {"crossover_s": report["crossover"], "panel_s": report["panels"],
                          "lookahead_s": per_la, "forward_s": per_fwd, "leaf_blocks_s": per_leaf,
                          "leaf_pipeline_s": per_pipe,
                          "batched_s": per_cu,
                          "rref_lanes_s": per_lanes,
                          "batched_workload": f"{len(systems)} uneven systems of the c4 "
                                              f"distribution (seed 4), mean of {reps} launches",
                          "rref_lanes_workload": f"{count} sparse-pattern matrices of "
                                                 f"12000 x 10000 (seed 5), median of {reps}"}}
    lx.restore_tuning()
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()
    table = tune(args.quick)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({k: table[k] for k in ("blocked_min", "panel", "batched_per_cu",
                                             "lookahead", "rref_lanes", "forward_min",
                                             "leaf_blocks", "leaf_pipeline")}))


if __name__ == "__main__":
    main()
