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


def _lowrank(rng, m, n, r, p):
    """(U V) mod p with small factors (entries below 2^15, so int64 sums are exact)."""
    U = rng.integers(0, 1 << 15, size=(m, r), dtype=np.int64)
    V = rng.integers(0, 1 << 15, size=(r, n), dtype=np.int64)
    return ((U @ V) % p).astype(np.uint32)


def test_passes_at_the_limits(gpu):
    """The batched kernel reduces a system in passes of 16 pivot columns: systems
    at the size limits of one workgroup (1024 rows, n + k = 2048), passes that
    hold free columns, passes cut short when the rank reaches m, rank-deficient
    and inconsistent systems, p = 2 and 3, and an all-zero system."""
    rng = np.random.default_rng(77)
    systems = []

    def add(A, B, p):
        systems.append(dict(A=np.ascontiguousarray(A, dtype=np.uint32),
                            B=np.ascontiguousarray(B, dtype=np.uint32), p=int(p)))

    p31 = workloads.draw_prime31(rng)
    add(workloads.uniform(rng, (1024, 1000), p31), workloads.uniform(rng, (1024, 8), p31), p31)
    add(workloads.uniform(rng, (300, 2040), p31), workloads.uniform(rng, (300, 8), p31), p31)
    add(workloads.uniform(rng, (1024, 64), p31), workloads.uniform(rng, (1024, 3), p31), p31)
    add(workloads.uniform(rng, (500, 400), 2), workloads.uniform(rng, (500, 4), 2), 2)
    add(_lowrank(rng, 400, 400, 37, 3), workloads.uniform(rng, (400, 3), 3), 3)
    A = workloads.uniform(rng, (512, 480), p31)
    A[:, ::7] = 0  # free columns inside most passes
    add(A, workloads.uniform(rng, (512, 5), p31), p31)
    A = workloads.uniform(rng, (512, 480), p31)
    A[:, 9::11] = A[:, 3::11][:, : A[:, 9::11].shape[1]]  # repeated columns: free later on
    add(A, workloads.uniform(rng, (512, 5), p31), p31)
    A = _lowrank(rng, 600, 500, 45, p31)
    B = np.concatenate([_lowrank(rng, 600, 3, 45, p31), workloads.uniform(rng, (600, 3), p31)], axis=1)
    add(A, B, p31)  # rank 45 (w.h.p.); random right-hand sides are inconsistent
    add(np.zeros((64, 64), dtype=np.uint32), workloads.uniform(rng, (64, 2), p31), p31)
    add(workloads.uniform(rng, (7, 1500), p31), workloads.uniform(rng, (7, 1), p31), p31)
    print("limits batch", [(s["A"].shape, s["B"].shape[1], s["p"]) for s in systems], flush=True)
    _check_all(systems, lx.solve_batched(systems), tag="limits")


def test_pivot_search_fallbacks(gpu):
    """The pivot search keeps the first 16 candidate rows reduced in registers
    and falls back to scanning the other candidates (each replaying the pass's
    pivots) when every window row is zero at a column; rows zero in all of a
    pass's columns are left out of the search.  Systems built to take each of
    these routes: a block of top rows zero at some columns, duplicated top rows
    (zero after the first is taken), a sparse system over F_3, rows zero in a
    whole pass, and fewer candidates than the window."""
    rng = np.random.default_rng(91)
    p31 = workloads.draw_prime31(rng)
    systems = []

    def add(A, B, p):
        systems.append(dict(A=np.ascontiguousarray(A, dtype=np.uint32),
                            B=np.ascontiguousarray(B, dtype=np.uint32), p=int(p)))

    A = workloads.uniform(rng, (300, 200), p31)
    A[:40, [5, 21, 40, 77]] = 0  # the window is zero there; the pivot lies past it
    add(A, workloads.uniform(rng, (300, 4), p31), p31)
    A = workloads.uniform(rng, (200, 150), p31)
    A[1:20] = A[0]  # duplicated top rows: zero once the first is a pivot
    add(A, workloads.uniform(rng, (200, 3), p31), p31)
    A = workloads.uniform(rng, (120, 100), 3) * (rng.random((120, 100)) < 0.15)
    add(A, workloads.uniform(rng, (120, 2), 3), 3)
    A = workloads.uniform(rng, (100, 90), p31)
    A[16:, :32] = 0  # after the first pass, no candidate is non-zero in columns 16..31
    add(A, workloads.uniform(rng, (100, 5), p31), p31)
    add(workloads.uniform(rng, (10, 40), p31), workloads.uniform(rng, (10, 2), p31), p31)
    A = workloads.uniform(rng, (64, 64), 7)
    A[:, 20:36] = 0  # a whole pass of free columns
    add(A, workloads.uniform(rng, (64, 1), 7), 7)
    print("fallback batch", [(s["A"].shape, s["B"].shape[1], s["p"]) for s in systems], flush=True)
    _check_all(systems, lx.solve_batched(systems), tag="fallbacks")


def test_validate_rejects_out_of_range_entry(gpu):
    """opts.validate checks every system of a batch against its own prime: one
    entry equal to p in one system's B makes the whole call return
    LINAC_E_RANGE before the batch runs; the same batch without it solves."""
    systems = workloads.batched_systems(seed=44, count=12, n_lo=8, n_hi=40)
    ref = oracle.solve_many(systems)
    _check_all(systems, lx.solve_batched(systems, validate=True), ref, tag="validate ok")
    bad = [dict(s) for s in systems]
    bad[7] = dict(bad[7])
    bad[7]["B"] = bad[7]["B"].copy()
    bad[7]["B"][3, 0] = bad[7]["p"]
    with pytest.raises(lx.LinacError) as e:
        lx.solve_batched(bad, validate=True)
    assert e.value.status == 4
