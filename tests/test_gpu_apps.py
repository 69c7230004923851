"""GPU parity of the calls around the elimination: the system construction
(linac_load_matrix, Sec. 3.3) and the null-space basis and column basis of a
rank factorisation (linac_nullspace, linac_column_basis, Sec. 5.1), all
through the C ABI, against the oracle bit for bit.

Construction cases cover every kernel instance (degree buckets 1-8, 9-16,
17-32 and the generic degree above 32; bases rows staged in LDS and, for more
than 8191 basis variables, read from global memory), tiles with ragged tails
in both directions, index lists with out-of-range entries (a factor 0), d = 0
and empty shapes.  At the full construction workload (20000 x 20000, 48 basis
variables, degree up to 12) sampled rows are compared with the oracle.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
import paper_2605_25863_amd as lx
from tests import certs

pytestmark = pytest.mark.gpu

P31 = 2147483629  # a 31-bit prime below 2^31 - 1


@pytest.mark.parametrize("nrows,ncols,nbasis,d,p", [
    (70, 600, 9, 3, workloads.MERSENNE31),   # 3 row tiles (ragged), 3 column tiles (ragged)
    (33, 257, 48, 8, P31),                   # degree bucket 8 at its top
    (65, 300, 20, 9, 65521),                 # bucket 16 at its bottom
    (40, 513, 100, 16, 2),
    (31, 129, 7, 17, 3),                     # bucket 32
    (37, 200, 64, 32, workloads.MERSENNE31),
    (35, 140, 10, 33, P31),                  # generic degree
    (12, 70, 5, 47, 7),
    (6, 300, 9000, 5, P31),                  # 9000 basis variables: read from global memory
    (1, 1, 1, 1, 5),
    (130, 1, 3, 4, 65521),
])
def test_load_matrix_matches_oracle(gpu, nrows, ncols, nbasis, d, p):
    rng = np.random.default_rng(nrows * 1000 + ncols + d)
    bases = workloads.uniform(rng, (nrows, nbasis), p)
    L = rng.integers(0, nbasis, size=(ncols, d)).astype(np.int32)
    print(f"load_matrix {nrows}x{ncols} nbasis={nbasis} d={d} p={p}", flush=True)
    got = lx.load_matrix(bases, L, p)
    assert np.array_equal(got, oracle.load_matrix(bases, L, p))


def test_load_matrix_edge_cases(gpu):
    p = 65521
    rng = np.random.default_rng(3)
    bases = workloads.uniform(rng, (20, 6), p)
    # out-of-range and negative indices are factors 0
    L = rng.integers(-3, 9, size=(50, 4)).astype(np.int32)
    assert np.array_equal(lx.load_matrix(bases, L, p), oracle.load_matrix(bases, L, p))
    # d = 0: every entry is the empty product 1
    assert np.array_equal(lx.load_matrix(bases, np.zeros((9, 0), np.int32), p),
                          np.ones((20, 9), np.uint32))
    # no basis variables: every index is out of range
    Z = lx.load_matrix(np.zeros((4, 0), np.uint32), np.zeros((3, 2), np.int32), p)
    assert Z.shape == (4, 3) and not Z.any()
    assert lx.load_matrix(bases, np.zeros((0, 3), np.int32), p).shape == (20, 0)
    assert lx.load_matrix(np.zeros((0, 6), np.uint32), L, p).shape == (0, 50)


def test_load_matrix_vandermonde_and_solve(gpu):
    """A Vandermonde system built on the device from the padded monomials
    x^c, solved on the device: the interpolation recovers the coefficients."""
    p = workloads.MERSENNE31
    n = 300
    x = workloads.vandermonde_nodes(seed=17, count=n, p=p)
    bases = np.stack([np.ones(n, np.uint64), x.astype(np.uint64)], axis=1).astype(np.uint32)
    L = np.zeros((n, n), dtype=np.int32)
    for c in range(n):
        L[c, :c] = 1
    A = lx.load_matrix(bases, L, p)
    assert np.array_equal(A, oracle.load_matrix(bases, L, p))
    coef = workloads.uniform(np.random.default_rng(4), (n, 1), p)
    b = oracle.matmul_mod(A, coef, p).astype(np.uint32)
    X, rank, piv, cons = lx.solve(A, b, p)
    assert rank == n and cons[0] == 1
    assert np.array_equal(X, coef)


def test_load_matrix_full_size_sampled_rows(gpu):
    import torch
    cfg = workloads.LM_CONFIG
    bases, L, p = workloads.monomial_system(**cfg)
    dev = torch.device("cuda", 0)
    Bt = torch.from_numpy(bases.astype(np.int32)).to(dev)
    Lt = torch.from_numpy(L).to(dev)
    A = lx.load_matrix(Bt, Lt, p)
    torch.cuda.synchronize()
    rows = np.random.default_rng(9).choice(cfg["nrows"], size=24, replace=False)
    rows = np.concatenate([rows, [0, 31, 32, cfg["nrows"] - 1]])
    got = A[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.uint32)
    assert np.array_equal(got, oracle.load_matrix(bases[rows], L, p))


def _rank_factor_case(A, p, tag):
    import torch
    dev = torch.device("cuda", 0)
    At = torch.from_numpy(A.astype(np.int32)).to(dev)
    R, rank, piv = lx.rref(At, p)
    K, free = lx.canonical_kernel(R, rank, piv, p, with_free=True)
    C = lx.column_basis(At, rank, piv)
    torch.cuda.synchronize()
    m, n = A.shape
    Rr, r, pr = oracle.rref(A, p)
    assert int(rank.item()) == r, tag
    Kr = oracle.canonical_kernel(Rr, pr, n, p).astype(np.uint32)
    Kg = K.cpu().numpy().astype(np.uint32)
    assert np.array_equal(Kg[:, : n - r], Kr), f"{tag}: kernel basis differs"
    assert not Kg[:, n - r:].any(), f"{tag}: columns past n - r are not zero"
    fr = free.cpu().numpy()[:n]
    want_free = [c for c in range(n) if c not in set(pr.tolist())]
    assert fr[: n - r].tolist() == want_free and np.all(fr[n - r:] == -1), tag
    Cg = C.cpu().numpy().astype(np.uint32)
    assert np.array_equal(Cg[:, :r], oracle.rank_factor_columns(A, pr).astype(np.uint32)), tag
    assert not Cg[:, r:].any(), tag


@pytest.mark.parametrize("m,n,r,p", [
    (40, 60, 25, workloads.MERSENNE31),
    (300, 280, 280, P31),   # full column rank: empty kernel
    (50, 600, 50, 65521),   # wide, several column blocks of K
    (90, 90, 0, 7),         # zero matrix: K = -I
    (1, 1, 1, 2),
    (120, 70, 33, 3),
])
def test_nullspace_and_column_basis_match_oracle(gpu, m, n, r, p):
    rng = np.random.default_rng(m + 7 * n + r)
    if r:
        L = workloads.uniform(rng, (m, r), p)
        U = workloads.uniform(rng, (r, n), p)
        A = oracle.matmul_mod(L, U, p).astype(np.uint32)
    else:
        A = np.zeros((m, n), np.uint32)
    print(f"rank factorisation {m}x{n} r={r} p={p}", flush=True)
    _rank_factor_case(A, p, f"{m}x{n} r={r}")


def test_rank_factorization_small_cases(gpu):
    for i, c in enumerate(workloads.small_cases(seed=77, count=40, max_dim=40, max_k=1)):
        _rank_factor_case(c["A"], c["p"], f"case {i} kind={c['kind']} p={c['p']}")
    C, R, K, r = lx.rank_factorization(np.eye(5, dtype=np.uint32), 11)
    assert r == 5 and K.shape == (5, 0) and np.array_equal(C, np.eye(5, dtype=np.uint32))


def test_nullspace_truncated_and_empty(gpu):
    import torch
    p = 101
    A = np.zeros((3, 6), np.uint32)
    A[0, 1] = 5
    A[1, 4] = 7
    dev = torch.device("cuda", 0)
    R, rank, piv = lx.rref(torch.from_numpy(A.astype(np.int32)).to(dev), p)
    K2 = lx.canonical_kernel(R, rank, piv, p, kcols=2)  # basis has 4 columns: keep 2
    Kfull = oracle.canonical_kernel(oracle.rref(A, p)[0], [1, 4], 6, p).astype(np.uint32)
    assert np.array_equal(K2.cpu().numpy().astype(np.uint32), Kfull[:, :2])
    # n = 0 and m = 0
    R0, rank0, piv0 = lx.rref(torch.zeros((0, 4), dtype=torch.int32, device=dev), p)
    K0 = lx.canonical_kernel(R0, rank0, piv0, p)
    assert np.array_equal(K0.cpu().numpy().astype(np.uint32), (p - 1) * np.eye(4, dtype=np.uint32))


def test_sparse_pattern_instance_kernel_certificate(gpu):
    """A K = 0 on every row of a full-size sparse-pattern instance
    (12000 x 10000, rank 9500), by Freivalds' check with two random vectors,
    and A = C R through the device column basis."""
    import torch
    _, A = next(iter(workloads.sparse_pattern_instances(count=64, instances=[7])))
    p = workloads.MERSENNE31
    dev = torch.device("cuda", 0)
    At = torch.from_numpy(A.astype(np.int32)).to(dev)
    R, rank, piv = lx.rref(At.clone(), p)
    K = lx.canonical_kernel(R, rank, piv, p)
    C = lx.column_basis(At, rank, piv)
    torch.cuda.synchronize()
    r = int(rank.item())
    n = A.shape[1]
    Kh = K.cpu().numpy()[:, : n - r].astype(np.uint64)
    for s in (1, 2):
        v = np.random.default_rng(s).integers(0, p, size=(n - r, 1), dtype=np.uint64)
        assert not oracle.matmul_mod(A, oracle.matmul_mod(Kh, v, p), p).any(), "A K != 0"
    Ch = C.cpu().numpy()[:, :r]
    Rh = R.cpu().numpy()[:r]
    pv = piv.cpu().numpy()[:r]
    assert np.array_equal(Ch, A[:, pv]), "C is not A[:, J]"
    assert certs.freivalds_rank_factorisation(A, Rh, r, pv, p)
