"""GPU parity of the plain Gauss-Jordan path against the CPU oracle.

Every comparison is bit-exact: the RREF, the rank, the pivot columns, the
consistency flags and the particular solution are uniquely defined (Sec. 5.1,
Sec. 5.2), so any correct elimination order must reproduce them exactly.  At
the full n = 8192 size the oracle would take minutes, so there the outputs are
checked through properties that determine them: A X = B exactly with rank n
(a unique solution) and pivots 0..n-1.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
import paper_2605_25863_amd as lx

pytestmark = pytest.mark.gpu

PLAIN = lx.PATH_PLAIN


def _cmp_solve(A, B, p, tag=""):
    got = lx.solve(A, B, p, path=PLAIN)
    ref = oracle.solve(A, B, p)
    names = ("X", "rank", "pivots", "consistent")
    for name, g, r in zip(names, got, ref):
        assert np.array_equal(np.asarray(g), np.asarray(r)), f"{tag}: {name} differs"


def _cmp_rref(A, p, tag=""):
    import torch
    R, rank, piv = lx.rref(A, p, path=PLAIN)
    torch.cuda.synchronize()
    Rr, rr, pr = oracle.rref(A, p)
    r = int(rank.item())
    assert r == rr, f"{tag}: rank {r} != {rr}"
    assert np.array_equal(R.cpu().numpy().astype(np.uint32), Rr), f"{tag}: RREF differs"
    pv = piv.cpu().numpy()
    assert np.array_equal(pv[:r], pr), f"{tag}: pivots differ"
    assert np.all(pv[r:] == -1), f"{tag}: pivot padding"


def test_small_random_cases(gpu):
    cases = workloads.small_cases(seed=2024, count=96, max_dim=70, max_k=8)
    for i, c in enumerate(cases):
        tag = f"case {i} kind={c['kind']} p={c['p']} shape={c['A'].shape} k={c['B'].shape[1]}"
        print(tag, flush=True)
        _cmp_solve(c["A"], c["B"], c["p"], tag)
        _cmp_rref(c["A"], c["p"], tag)


@pytest.mark.parametrize("m,n,k,p", [
    (300, 300, 5, None),               # several row tiles, two column chunks, ragged tails
    (257, 300, 3, workloads.MERSENNE31),
    (700, 450, 0, None),               # tall, no right-hand side
    (129, 700, 9, 65521),              # wide: pivots run out of rows before columns
    (1000, 1000, 16, None),
])
def test_medium_dense(gpu, m, n, k, p):
    rng = np.random.default_rng(m * 7 + n)
    if p is None:
        p = workloads.draw_prime31(rng)
    A = workloads.uniform(rng, (m, n), p)
    B = workloads.uniform(rng, (m, k), p)
    tag = f"dense m={m} n={n} k={k} p={p}"
    print(tag, flush=True)
    _cmp_solve(A, B, p, tag)
    _cmp_rref(A, p, tag)


def test_rank_deficient_and_structured(gpu):
    rng = np.random.default_rng(5)
    p = workloads.draw_prime31(rng)
    n = 320
    L = workloads.uniform(rng, (n, 200), p).astype(np.uint64)
    U = workloads.uniform(rng, (200, n), p).astype(np.uint64)
    A = oracle.matmul_mod(L, U, p).astype(np.uint32)      # rank 200
    B = workloads.uniform(rng, (n, 4), p)
    B[:, 0] = oracle.matmul_mod(A, workloads.uniform(rng, (n, 1), p), p)[:, 0]  # consistent
    print("lowrank 320 rank 200", flush=True)
    _cmp_solve(A, B, p, "lowrank")
    _cmp_rref(A, p, "lowrank")
    # sparse: most multipliers are zero, exercising the skip of untouched rows
    S = workloads.uniform(rng, (400, 380), p)
    S[rng.random(S.shape) < 0.97] = 0
    print("sparse 400x380", flush=True)
    _cmp_solve(S, B[:1].repeat(400, axis=0)[:, :2], p, "sparse")
    _cmp_rref(S, p, "sparse")
    # whole zero columns at tile boundaries and a block of free columns
    Z = workloads.uniform(rng, (260, 330), p)
    Z[:, 60:70] = 0
    Z[:, 255:258] = 0
    Z[:, 100:140] = Z[:, 0:40]
    print("free columns", flush=True)
    _cmp_solve(Z, B[:260, :3], p, "freecols")
    _cmp_rref(Z, p, "freecols")


def test_edge_shapes(gpu):
    p = 7
    rng = np.random.default_rng(9)
    for m, n, k in [(0, 5, 2), (5, 0, 2), (0, 0, 0), (1, 1, 1), (1, 9, 0), (9, 1, 3), (3, 3, 0),
                    (64, 64, 1), (65, 63, 2)]:
        A = rng.integers(0, p, size=(m, n)).astype(np.uint32)
        B = rng.integers(0, p, size=(m, k)).astype(np.uint32)
        tag = f"edge m={m} n={n} k={k}"
        print(tag, flush=True)
        _cmp_solve(A, B, p, tag)
        if m and n:
            _cmp_rref(A, p, tag)
    for p in (2, 3):
        A = rng.integers(0, p, size=(90, 90)).astype(np.uint32)
        B = rng.integers(0, p, size=(90, 3)).astype(np.uint32)
        _cmp_solve(A, B, p, f"p={p}")
        _cmp_rref(A, p, f"p={p}")


def test_c1_workload(gpu):
    A, B, p = workloads.config("c1")
    print("c1", flush=True)
    _cmp_solve(A, B, p, "c1")
    _cmp_rref(A, p, "c1")


def test_inputs_untouched_and_deterministic(gpu):
    import torch
    A, B, p = workloads.config("c2", n=600)
    At = torch.from_numpy(A.astype(np.int32)).cuda()
    Bt = torch.from_numpy(B.astype(np.int32)).cuda()
    A0, B0 = At.clone(), Bt.clone()
    out1 = [t.clone() for t in lx.solve(At, Bt, p, path=PLAIN)]
    out2 = [t.clone() for t in lx.solve(At, Bt, p, path=PLAIN)]
    torch.cuda.synchronize()
    assert torch.equal(At, A0) and torch.equal(Bt, B0)
    for a, b in zip(out1, out2):
        assert torch.equal(a, b)


def test_validate_flag(gpu):
    A = np.array([[1, 2], [3, 9]], dtype=np.uint32)
    B = np.zeros((2, 1), dtype=np.uint32)
    with pytest.raises(lx.LinacError) as e:
        lx.solve(A, B, 7, path=PLAIN, validate=True)
    assert e.value.status == 4


def test_c2_full_size_certificate(gpu):
    """n = 8192, 16 right-hand sides, seeded 31-bit prime (the benchmark input)."""
    import torch
    A, B, p = workloads.config("c2")
    print("c2 full size", flush=True)
    X, rank, piv, cons = lx.solve(A, B, p, path=PLAIN)
    assert rank == 8192 and np.array_equal(piv, np.arange(8192)) and cons.all()
    assert np.array_equal(oracle.matmul_mod(A, X, p), B.astype(np.uint64))
