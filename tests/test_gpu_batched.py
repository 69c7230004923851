"""GPU parity of the batched persistent path (one launch, hipGraph replay)
against the CPU oracle, bit for bit, per system."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
import paper_2605_25863_amd as lx

pytestmark = pytest.mark.gpu


def _check_all(systems, got, ref=None, tag=""):
    ref = ref if ref is not None else oracle.solve_many(systems)
    for i, (g, r) in enumerate(zip(got, ref)):
        for name, a, b in zip(("X", "rank", "pivots", "consistent"), g, r):
            assert np.array_equal(np.asarray(a), np.asarray(b)), f"{tag} system {i}: {name}"


def test_small_batch(gpu):
    systems = workloads.batched_systems(seed=21, count=96, n_lo=1, n_hi=90, deficient_frac=0.2)
    print("small batch", flush=True)
    _check_all(systems, lx.solve_batched(systems), tag="small")


def test_mixed_shapes_batch(gpu):
    cases = workloads.small_cases(seed=8, count=80, max_dim=72, max_k=8)
    rng = np.random.default_rng(1)
    extra = []
    for m, n, k in [(0, 4, 2), (4, 0, 2), (1, 1, 1), (3, 3, 0), (200, 150, 5), (150, 200, 3)]:
        p = workloads.draw_prime31(rng)
        extra.append(dict(A=workloads.uniform(rng, (m, n), p), B=workloads.uniform(rng, (m, k), p),
                          p=p))
    systems = cases + extra
    print("mixed batch", flush=True)
    _check_all(systems, lx.solve_batched(systems), tag="mixed")


def test_graph_replays(gpu):
    """Replay the captured graph several times with eager work in between; every
    replay must reproduce the oracle."""
    import torch
    systems = workloads.batched_systems(seed=33, count=64, n_lo=16, n_hi=120, deficient_frac=0.1)
    ref = oracle.solve_many(systems)
    prep = lx.prepare_batched(systems)
    for rep in range(4):
        for it in prep["items"]:
            it["X"].fill_(12345)
            it["rank"].fill_(-7)
        torch.cuda.synchronize()
        lx.solve_batched(systems, prepared=prep)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        got = []
        for it in prep["items"]:
            r = int(it["rank"].item())
            got.append((it["X"].cpu().numpy().astype(np.uint32), r,
                        it["pivots"].cpu().numpy()[:r].astype(np.int64),
                        it["cons"].cpu().numpy()[: it["X"].shape[1]].astype(np.uint8)))
        _check_all(systems, got, ref, tag=f"replay {rep}")
        del junk


def test_c4_full_batch(gpu):
    """The 4096-system workload: a seeded subset against the oracle, every system
    through certificates (rank, A X = B on consistent columns)."""
    systems = workloads.batched_systems()
    print("c4 batch", flush=True)
    got = lx.solve_batched(systems)
    idx = np.random.default_rng(4).choice(len(systems), size=256, replace=False)
    sub = [systems[i] for i in idx]
    _check_all(sub, [got[i] for i in idx], tag="c4 subset")
    for s, (X, r, piv, cons) in zip(systems, got):
        n = s["n"]
        assert r == (n - 1 if s["deficient"] else n)
        assert cons.all()  # dependent rows were built on [A | B]
        assert np.array_equal(oracle.matmul_mod(s["A"], X, s["p"]), s["B"].astype(np.uint64))
