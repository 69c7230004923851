"""GPU parity of the blocked path (panel Gauss-Jordan + exact int8-MFMA trailing
product) against the CPU oracle, bit for bit.

Panel widths are chosen so that panels are ragged (n not a multiple of the
width), free columns fall inside panels, and the last panel is partial.  At the
full sizes (n = 8192 and 16384) the results are checked by certificates on
every row: rank = n, pivots 0..n-1, A X = B (exactly at n = 8192, by
Freivalds' check at n = 16384), and at n = 16384 also the RREF of [A | B],
whose left block must be the identity and whose right block must solve the
system.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from tests import certs
import paper_2605_25863_amd as lx

pytestmark = pytest.mark.gpu

INT8 = lx.PATH_BLOCKED_INT8


def _solve(A, B, p, panel, path=INT8):
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A).astype(np.int32)).cuda()
    Bt = torch.from_numpy(np.ascontiguousarray(B).astype(np.int32)).cuda()
    m, n = A.shape
    k = B.shape[1]
    X = torch.empty((n, k), dtype=torch.int32, device="cuda")
    rank = torch.zeros(1, dtype=torch.int32, device="cuda")
    piv = torch.empty(min(m, n), dtype=torch.int32, device="cuda")
    cons = torch.empty(k, dtype=torch.uint8, device="cuda")
    lx.solve(At, Bt, p, path=path, out=(X, rank, piv, cons), panel_width=panel)
    torch.cuda.synchronize()
    r = int(rank.item())
    return (X.cpu().numpy().astype(np.uint32), r, piv.cpu().numpy()[:r].astype(np.int64),
            cons.cpu().numpy().astype(np.uint8))


def _cmp(A, B, p, panel, tag):
    got = _solve(A, B, p, panel)
    ref = oracle.solve(A, B, p)
    for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
        assert np.array_equal(np.asarray(g), np.asarray(r)), f"{tag}: {name} differs"


def _cmp_rref(A, p, panel, tag):
    import torch
    R, rank, piv = lx.rref(A, p, path=INT8, panel_width=panel)
    torch.cuda.synchronize()
    Rr, rr, pr = oracle.rref(A, p)
    r = int(rank.item())
    assert r == rr, f"{tag}: rank"
    assert np.array_equal(R.cpu().numpy().astype(np.uint32), Rr), f"{tag}: RREF differs"
    assert np.array_equal(piv.cpu().numpy()[:r], pr), f"{tag}: pivots"


@pytest.mark.parametrize("m,n,k,p,panel", [
    (300, 300, 5, None, 64),
    (300, 300, 3, workloads.MERSENNE31, 32),
    (257, 333, 17, None, 96),
    (500, 420, 0, 65521, 256),
    (129, 700, 9, None, 128),
    (600, 600, 8, None, 512),
    (700, 650, 6, None, 192),
    (800, 760, 4, None, 320),
    (900, 880, 5, None, 384),
    (1000, 1000, 3, workloads.MERSENNE31, 384),
    (64, 64, 1, 2, 32),
    (100, 100, 2, 3, 64),
])
def test_dense_panels(gpu, m, n, k, p, panel):
    rng = np.random.default_rng(m * 31 + n + panel)
    if p is None:
        p = workloads.draw_prime31(rng)
    A = workloads.uniform(rng, (m, n), p)
    B = workloads.uniform(rng, (m, k), p)
    tag = f"blocked m={m} n={n} k={k} p={p} panel={panel}"
    print(tag, flush=True)
    _cmp(A, B, p, panel, tag)
    _cmp_rref(A, p, panel, tag)


def test_structured(gpu):
    rng = np.random.default_rng(77)
    p = workloads.draw_prime31(rng)
    # free columns inside panels, a zero block, duplicated columns
    Z = workloads.uniform(rng, (330, 400), p)
    Z[:, 30:45] = 0
    Z[:, 100:140] = Z[:, 0:40]
    Z[:, 255:260] = 0
    B = workloads.uniform(rng, (330, 4), p)
    B[:, 1] = oracle.matmul_mod(Z, workloads.uniform(rng, (400, 1), p), p)[:, 0]
    for panel in (32, 64, 256):
        tag = f"freecols panel={panel}"
        print(tag, flush=True)
        _cmp(Z, B, p, panel, tag)
        _cmp_rref(Z, p, panel, tag)
    # low rank
    L = workloads.uniform(rng, (350, 150), p).astype(np.uint64)
    U = workloads.uniform(rng, (150, 380), p).astype(np.uint64)
    A = oracle.matmul_mod(L, U, p).astype(np.uint32)
    B2 = workloads.uniform(rng, (350, 3), p)
    B2[:, 0] = oracle.matmul_mod(A, workloads.uniform(rng, (380, 1), p), p)[:, 0]
    for panel in (64, 128):
        _cmp(A, B2, p, panel, f"lowrank panel={panel}")
    # sparse rows (many zero multipliers), rank deficient
    S = workloads.uniform(rng, (400, 380), p)
    S[rng.random(S.shape) < 0.95] = 0
    _cmp(S, B2[:1].repeat(400, axis=0)[:, :2], p, 64, "sparse")
    _cmp_rref(S, p, 64, "sparse")


def test_small_cases_blocked(gpu):
    for i, c in enumerate(workloads.small_cases(seed=99, count=48, max_dim=70, max_k=6)):
        tag = f"small {i} {c['kind']} {c['A'].shape} p={c['p']}"
        _cmp(c["A"], c["B"], c["p"], 32, tag)


def test_c2_slice_against_oracle(gpu):
    """n = 1536 of the c2 distribution (16 right-hand sides, panel 256 and the
    tuned panel), bit for bit against the oracle."""
    A, B, p = workloads.config("c2", n=1536)
    ref = oracle.solve(A, B, p)
    for panel in (256, 0):
        got = _solve(A, B, p, panel, path=INT8)
        for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
            assert np.array_equal(np.asarray(g), np.asarray(r)), f"c2 slice panel={panel}: {name}"


@pytest.mark.parametrize("panel", [192, 320, 384])
def test_structured_wide_panels(gpu, panel):
    """Free columns inside 192-, 320- and 384-wide panels, a zero block, duplicated
    columns, inconsistent right-hand sides; solve and RREF against the oracle."""
    rng = np.random.default_rng(panel)
    p = workloads.draw_prime31(rng)
    Z = workloads.uniform(rng, (820, 900), p)
    Z[:, 30:45] = 0
    Z[:, 200:260] = Z[:, 0:60]
    Z[:, 383:390] = 0
    Z[700:] = Z[:120]
    B = workloads.uniform(rng, (820, 4), p)
    B[:, 1] = oracle.matmul_mod(Z, workloads.uniform(rng, (900, 1), p), p)[:, 0]
    tag = f"wide panel={panel}"
    print(tag, flush=True)
    _cmp(Z, B, p, panel, tag)
    _cmp_rref(Z, p, panel, tag)


def test_lookahead_off(gpu):
    """The blocked int8 path with the look-ahead switched off in the tuning
    table (the table can select it), against the oracle; the shipped table is
    restored afterwards."""
    rng = np.random.default_rng(5150)
    p = workloads.draw_prime31(rng)
    A = workloads.uniform(rng, (1100, 1000), p)
    A[:, 100:110] = 0
    B = workloads.uniform(rng, (1100, 3), p)
    lx.load_tuning('{"lookahead": 0}')
    try:
        for panel in (128, 256):
            tag = f"lookahead off panel={panel}"
            print(tag, flush=True)
            _cmp(A, B, p, panel, tag)
            _cmp_rref(A, p, panel, tag)
    finally:
        lx.restore_tuning()


def test_auto_plan_sizes_against_oracle(gpu):
    """The AUTO path at sizes where the shipped table picks each of its panel
    widths (and the plain/blocked crossover), against the oracle."""
    import json
    table = json.load(open(lx.TUNING_FILE))
    sizes = {int(table.get("blocked_min", 1024)), int(table.get("blocked_min", 1024)) - 1}
    prev = 0
    for rule in table.get("panel", []):
        lo = max(prev + 1, int(table.get("blocked_min", 1024)))
        hi = int(rule["n_max"])
        if lo <= hi:
            sizes.add(min(hi, lo + 37))
        prev = hi
    for n in sorted(s for s in sizes if s <= 2600):
        A, B, p = workloads.config("c2", n=n)
        A, B = A[:, :n], B[:, :3]
        path, panel = lx.plan(n, n)
        tag = f"auto n={n} plan=({path},{panel})"
        print(tag, flush=True)
        got = _solve(A, B, p, 0, path=lx.PATH_AUTO)
        ref = oracle.solve(A, B, p)
        for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
            assert np.array_equal(np.asarray(g), np.asarray(r)), f"{tag}: {name}"


def test_c1_blocked(gpu):
    A, B, p = workloads.config("c1")
    _cmp(A, B, p, 64, "c1 blocked")


def test_c2_full_size_blocked(gpu):
    A, B, p = workloads.config("c2")
    print("c2 blocked full size", flush=True)
    X, r, piv, cons = _solve(A, B, p, 256)
    assert r == 8192 and np.array_equal(piv, np.arange(8192)) and cons.all()
    assert np.array_equal(oracle.matmul_mod(A, X, p), B.astype(np.uint64))


def test_c3_full_size_blocked(gpu):
    """n = 16384, 64 right-hand sides: rank, pivots and A X = B on every row
    (Freivalds), for the solve and for the RREF of [A | B]."""
    import torch
    A, B, p = workloads.config("c3")
    n = A.shape[1]
    print("c3 blocked full size: solve", flush=True)
    X, r, piv, cons = _solve(A, B, p, 0)
    assert r == n and np.array_equal(piv, np.arange(n)) and cons.all()
    assert certs.freivalds_solution(A, X, B, p), "c3 solve: A X != B"
    print("c3 blocked full size: rref of [A | B]", flush=True)
    M = torch.from_numpy(np.concatenate([A, B], axis=1).astype(np.int32)).cuda()
    R, rank, pv = lx.rref(M, p, inplace=True, path=INT8)
    torch.cuda.synchronize()
    assert int(rank.item()) == n
    assert np.array_equal(pv.cpu().numpy()[:n], np.arange(n))
    R = R.cpu().numpy().view(np.uint32)
    del M
    left = R[:, :n]
    assert np.count_nonzero(left) == n and np.all(np.diagonal(left) == 1), "left block is not I"
    del left
    XR = np.ascontiguousarray(R[:, n:])
    assert np.array_equal(XR, X), "RREF right block differs from the solve's X"
    assert certs.freivalds_solution(A, XR, B, p), "c3 rref: right block does not solve A X = B"


FP64 = lx.PATH_BLOCKED_FP64


@pytest.mark.parametrize("m,n,k,bits,panel", [
    (300, 300, 5, 20, 64),
    (257, 333, 7, 16, 96),
    (500, 420, 0, 21, 256),
    (129, 700, 3, 13, 128),
    (700, 650, 9, 20, 512),
])
def test_fp64_variant(gpu, m, n, k, bits, panel):
    """The FP64-MFMA trailing product for p < 2^21, bit-exact."""
    rng = np.random.default_rng(m + n + bits)
    p = workloads.draw_prime_bits(rng, bits)
    assert p < (1 << 21)
    A = workloads.uniform(rng, (m, n), p)
    B = workloads.uniform(rng, (m, k), p)
    if m > 10:
        A[7] = A[3]
        A[:, 5] = 0
    tag = f"fp64 m={m} n={n} k={k} p={p} panel={panel}"
    print(tag, flush=True)
    got = _solve(A, B, p, panel, path=FP64)
    ref = oracle.solve(A, B, p)
    for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
        assert np.array_equal(np.asarray(g), np.asarray(r)), f"{tag}: {name}"
    import torch
    R, rank, piv = lx.rref(A, p, path=FP64, panel_width=panel)
    torch.cuda.synchronize()
    Rr, rr, pr = oracle.rref(A, p)
    assert int(rank.item()) == rr
    assert np.array_equal(R.cpu().numpy().astype(np.uint32), Rr)


def test_fp64_large_and_rejects_big_primes(gpu):
    rng = np.random.default_rng(12)
    p = workloads.draw_prime_bits(rng, 20)
    n = 4096
    A = workloads.uniform(rng, (n, n), p)
    B = workloads.uniform(rng, (n, 8), p)
    X, r, piv, cons = _solve(A, B, p, 256, path=FP64)
    assert r == n and cons.all()
    assert np.array_equal(oracle.matmul_mod(A, X, p), B.astype(np.uint64))
    with pytest.raises(lx.LinacError) as e:
        lx.solve(A[:8, :8], B[:8], workloads.MERSENNE31, path=FP64)
    assert e.value.status == 2


@pytest.mark.parametrize("m,n,panel,kind", [
    (3000, 200, 64, "late"),       # each leaf's only pivot candidates sit in the last rows
    (2500, 300, 256, "zero_leaves"),  # whole leaves of zero columns (no pivot at all)
    (4200, 160, 128, "tall_lowrank"),  # rank 100 spread over 4200 rows: deep merge trees
    (700, 900, 96, "scattered"),   # pivots of every leaf spread over many chunks
])
def test_selection_trees(gpu, m, n, panel, kind):
    """Leaves whose basis is not inside the first chunk of candidate rows, so the
    selection merges bases up the tree (and reaches the root)."""
    rng = np.random.default_rng(m + n + panel)
    p = workloads.draw_prime31(rng)
    if kind == "late":
        A = np.zeros((m, n), dtype=np.uint32)
        A[m - n:, :] = workloads.uniform(rng, (n, n), p)
        A[:m - n, ::7] = workloads.uniform(rng, (m - n, len(range(0, n, 7))), p)
    elif kind == "zero_leaves":
        A = workloads.uniform(rng, (m, n), p)
        A[:, 32:96] = 0
        A[:, 200:232] = 0
    elif kind == "tall_lowrank":
        L = workloads.uniform(rng, (m, 100), p).astype(np.uint64)
        L[rng.random(m) < 0.97] = 0
        U = workloads.uniform(rng, (100, n), p).astype(np.uint64)
        A = oracle.matmul_mod(L, U, p).astype(np.uint32)
    else:
        A = workloads.uniform(rng, (m, n), p)
        A[rng.random((m, n)) < 0.995] = 0
    B = workloads.uniform(rng, (m, 3), p)
    B[:, 0] = oracle.matmul_mod(A, workloads.uniform(rng, (n, 1), p), p)[:, 0]
    tag = f"trees {kind} m={m} n={n} panel={panel} p={p}"
    print(tag, flush=True)
    _cmp(A, B, p, panel, tag)
    _cmp_rref(A, p, panel, tag)
    q = workloads.draw_prime_bits(rng, 20)
    Aq, Bq = A % q, B % q
    ref = oracle.solve(Aq, Bq, q)
    got = _solve(Aq, Bq, q, panel, path=FP64)
    for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
        assert np.array_equal(np.asarray(g), np.asarray(r)), f"{tag} fp64: {name}"


def test_forward_elimination_small_systems(gpu):
    """Solves with forward elimination and back-substitution (forced from
    every size through the tuning table) on ragged panels, rectangular, rank
    deficient and free-column systems, against the oracle.  The same results
    as Gauss-Jordan, which the rest of this file checks."""
    import json
    table = json.load(open(lx.TUNING_FILE))
    table["forward_min"] = 1
    lx.load_tuning(json.dumps(table))
    try:
        rng = np.random.default_rng(321)
        for m, n, k, panel in [(300, 300, 5, 64), (257, 333, 17, 96), (700, 650, 6, 192),
                               (900, 880, 5, 384), (600, 600, 8, 512), (129, 700, 9, 128),
                               (800, 300, 3, 64), (64, 64, 1, 32)]:
            A, B, p = workloads.dense_system(seed=m * 7 + n, n=n, k=k, m=m)
            if m > 10:
                A[m // 3] = A[1]          # rank deficient, consistent or not
                A[:, n // 2] = 0          # a free column inside a panel
                A[:, min(n - 1, 2 * panel + 5)] = A[:, 3]
            tag = f"forward m={m} n={n} k={k} panel={panel}"
            print(tag, flush=True)
            got = lx.solve(A, B, p, path=lx.PATH_BLOCKED_INT8, panel_width=panel)
            ref = oracle.solve(A, B, p)
            for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
                assert np.array_equal(np.asarray(g), np.asarray(r)), f"{tag}: {name}"
        for i, c in enumerate(workloads.small_cases(seed=4321, count=40, max_dim=90, max_k=6)):
            got = lx.solve(c["A"], c["B"], c["p"], path=lx.PATH_BLOCKED_INT8, panel_width=32)
            ref = oracle.solve(c["A"], c["B"], c["p"])
            for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
                assert np.array_equal(np.asarray(g), np.asarray(r)), f"small case {i}: {name}"
    finally:
        lx.restore_tuning()


@pytest.mark.parametrize("leaf_blocks", [3, 6, 9])
def test_leaf_product_shapes(gpu, leaf_blocks):
    """Every workgroup shape of the int8 leaf product the tuning table can pick
    (16-column blocks per workgroup), on ragged panels, a selection tree and
    free columns, against the oracle."""
    import json
    table = json.load(open(lx.TUNING_FILE))
    table["leaf_blocks"] = leaf_blocks
    lx.load_tuning(json.dumps(table))
    try:
        for m, n, k, panel in [(300, 300, 5, 64), (700, 650, 6, 192), (900, 880, 5, 384),
                               (257, 333, 17, 96)]:
            A, B, p = workloads.dense_system(seed=m + 11 * n, n=n, k=k, m=m)
            A[m // 2] = A[5]
            A[:, n // 3] = 0
            A[40:80] = 0  # zero rows inside the first candidate chunks: the selection tree
            tag = f"leaf_blocks={leaf_blocks} m={m} n={n} panel={panel}"
            print(tag, flush=True)
            got = lx.solve(A, B, p, path=lx.PATH_BLOCKED_INT8, panel_width=panel)
            ref = oracle.solve(A, B, p)
            for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
                assert np.array_equal(np.asarray(g), np.asarray(r)), f"{tag}: {name}"
            R, rank, piv = lx.rref(A, p, path=lx.PATH_BLOCKED_INT8, panel_width=panel)
            Rr, rr, pr = oracle.rref(A, p)
            import torch
            torch.cuda.synchronize()
            assert int(rank.item()) == rr and np.array_equal(R.cpu().numpy().astype(np.uint32), Rr)
    finally:
        lx.restore_tuning()


@pytest.mark.parametrize("pipeline,forward", [(1, 0), (1, 1), (0, 0), (0, 1)])
def test_leaf_pipeline(gpu, pipeline, forward):
    """The leaf products split in two (the next leaf's first chunk, then the
    other rows on a second stream while the next selection runs), and unsplit,
    for RREFs and for solves by Gauss-Jordan and by forward elimination,
    against the oracle.  The cases reach the chunk's corner cases: leaves with
    fewer pivots than columns (free and repeated columns), first chunks short
    of full rank (zero and repeated rows: the selection tree decides), lists
    shorter than a chunk near the end, and few rows."""
    import json
    import torch
    table = json.load(open(lx.TUNING_FILE))
    table["leaf_pipeline"] = pipeline
    table["forward_min"] = 1 if forward else 1 << 30
    lx.load_tuning(json.dumps(table))
    try:
        rng = np.random.default_rng(777 + 10 * pipeline + forward)
        cases = []
        for m, n, k, panel in [(300, 300, 5, 64), (700, 650, 6, 192), (257, 333, 17, 96),
                               (40, 300, 3, 128), (520, 200, 4, 64)]:
            A, B, p = workloads.dense_system(seed=m + 13 * n, n=n, k=k, m=m)
            if m > 100:
                A[m // 2] = A[5]
                A[:, n // 3] = 0
                A[:, n // 4] = A[:, 2]
                A[40:80] = 0
            cases.append((f"dense m={m} n={n}", A, B, p, panel))
        p3 = 3
        A3 = (rng.random((400, 380)) < 0.05).astype(np.uint32) * rng.integers(1, 3, (400, 380),
                                                                             dtype=np.uint32)
        B3 = rng.integers(0, p3, (400, 2), dtype=np.uint32)
        cases.append(("sparse F_3", A3, B3, p3, 64))
        for tag0, A, B, p, panel in cases:
            tag = f"pipeline={pipeline} forward={forward} {tag0} panel={panel}"
            print(tag, flush=True)
            got = lx.solve(A, B, p, path=lx.PATH_BLOCKED_INT8, panel_width=panel)
            ref = oracle.solve(A, B, p)
            for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
                assert np.array_equal(np.asarray(g), np.asarray(r)), f"{tag}: {name}"
            R, rank, piv = lx.rref(A, p, path=lx.PATH_BLOCKED_INT8, panel_width=panel)
            Rr, rr, pr = oracle.rref(A, p)
            torch.cuda.synchronize()
            assert int(rank.item()) == rr, f"{tag}: rref rank"
            assert np.array_equal(R.cpu().numpy().astype(np.uint32), Rr), f"{tag}: rref"
    finally:
        lx.restore_tuning()
