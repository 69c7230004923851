"""Pins of the CPU oracle to mathematics (runs without a GPU).

The oracle is trusted by the GPU parity tests only because these checks tie
it to facts that do not depend on its own code: brute-force enumeration over
tiny fields, the closed-form Vandermonde determinant, uniqueness of the
reduced row-echelon form (invariance under row permutation, row scaling and
the choice of pivot), the rank factorisation and null space of Sec. 5.1, and
agreement of three independent implementations.  The mutation tests plant
plausible mistakes in a copy of the oracle and require the pins to catch
each of them.
"""

from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
import workloads
from tests import pins

IMPLS = ("c", "numpy", "python")


def _rref(impl):
    return lambda A, p: oracle.rref(A, p, impl=impl)


def _solve(impl):
    return lambda A, B, p: oracle.solve(A, B, p, impl=impl)


# --- brute force over tiny fields ------------------------------------------

@pytest.mark.parametrize("impl", IMPLS)
def test_rref_exhaustive_gf2_3x3(impl):
    """Every 3x3 matrix over GF(2): shape predicate, row space, rank."""
    for bits in range(1 << 9):
        A = np.array([(bits >> s) & 1 for s in range(9)], dtype=np.uint64).reshape(3, 3)
        pins.check_rref_bruteforce(_rref(impl), A, 2)


@pytest.mark.parametrize("impl", IMPLS)
@pytest.mark.parametrize("p", [3, 5, 7])
def test_rref_bruteforce_small_fields(impl, p):
    rng = np.random.default_rng(100 + p)
    for _ in range(40):
        m = int(rng.integers(1, 4 if p == 7 else 5))
        n = int(rng.integers(1, 6))
        A = rng.integers(0, p, size=(m, n)).astype(np.uint64)
        if rng.random() < 0.3 and m > 1:
            A[-1] = (A[0] * int(rng.integers(0, p))) % p  # force a dependency
        pins.check_rref_bruteforce(_rref(impl), A, p)


@pytest.mark.parametrize("impl", IMPLS)
@pytest.mark.parametrize("p", [2, 3, 5])
def test_solve_bruteforce(impl, p):
    """Count all x in F_p^n: consistency, p^(n-r) solutions, particular solution."""
    rng = np.random.default_rng(200 + p)
    for _ in range(30):
        m = int(rng.integers(1, 5))
        n = int(rng.integers(1, 5 if p < 5 else 4))
        k = int(rng.integers(1, 4))
        A = rng.integers(0, p, size=(m, n)).astype(np.uint64)
        if rng.random() < 0.4:
            A[:, -1] = 0
        if rng.random() < 0.4 and m > 1:
            A[-1] = A[0]
        B = rng.integers(0, p, size=(m, k)).astype(np.uint64)
        pins.check_solve_bruteforce(_solve(impl), A, B, p)


# --- closed forms ----------------------------------------------------------

@pytest.mark.parametrize("impl", IMPLS)
@pytest.mark.parametrize("p,size", [(7, 5), (65521, 12), (workloads.MERSENNE31, 24),
                                    (1000003, 16)])
def test_vandermonde_determinant(impl, p, size):
    """det V = prod_{i<j} (x_j - x_i) mod p; 0 with a repeated node."""
    if impl == "python" and size > 16:
        size = 16
    x = workloads.vandermonde_nodes(seed=size, count=size, p=p)
    V = pins.vandermonde(x, size, p)
    assert oracle.det(V, p, impl=impl) == pins.vandermonde_det(x, p)
    # a repeated node makes two equal rows
    x2 = x.copy()
    x2[-1] = x2[0]
    V2 = pins.vandermonde(x2, size, p)
    assert oracle.det(V2, p, impl=impl) == 0
    R, r, piv = oracle.rref(V2, p, impl=impl)
    assert r == size - 1


@pytest.mark.parametrize("p", [65521, workloads.MERSENNE31])
def test_vandermonde_rank_and_interpolation(p):
    """rank V (m x n) = min(#distinct nodes, n); V c = b recovers c."""
    rng = np.random.default_rng(7)
    for m, n, distinct in [(20, 12, 20), (12, 20, 12), (30, 30, 17)]:
        x = workloads.vandermonde_nodes(seed=m * n, count=distinct, p=p)
        nodes = np.concatenate([x, rng.choice(x, size=m - distinct)]) if m > distinct else x
        V = pins.vandermonde(nodes, n, p)
        for impl in IMPLS:
            _, r, _ = oracle.rref(V, p, impl=impl)
            assert r == min(distinct, n)
    # interpolation: square distinct -> unique coefficients
    n = 24
    x = workloads.vandermonde_nodes(seed=1, count=n, p=p)
    V = pins.vandermonde(x, n, p)
    c = rng.integers(0, p, size=(n, 3)).astype(np.uint64)
    b = pins._mm(V, c, p).astype(np.uint64)
    for impl in IMPLS:
        X, r, piv, cons = oracle.solve(V, b, p, impl=impl)
        assert r == n and list(piv) == list(range(n)) and cons.all()
        assert np.array_equal(X.astype(np.uint64), c)


# --- uniqueness of the RREF -------------------------------------------------

@pytest.mark.parametrize("impl", ("numpy", "python"))
@pytest.mark.parametrize("rule", ("last", "random"))
def test_pivot_rule_invariance(impl, rule):
    """Any non-zero pivot gives the same RREF (Sec. 3.2, Pivoting)."""
    for case in workloads.small_cases(seed=31, count=24, max_dim=12, max_k=0):
        A, p = case["A"], case["p"]
        ref = oracle.rref(A, p, impl="c")
        got = oracle.rref(A, p, impl=impl, pivot_rule=rule, seed=5)
        assert np.array_equal(ref[0], got[0]) and ref[1] == got[1]
        assert np.array_equal(ref[2], got[2])


def test_row_permutation_scaling_idempotence():
    rng = np.random.default_rng(11)
    for case in workloads.small_cases(seed=41, count=32, max_dim=20, max_k=0):
        A, p = case["A"].astype(np.uint64), case["p"]
        R, r, piv = oracle.rref(A, p)
        perm = rng.permutation(A.shape[0])
        assert np.array_equal(oracle.rref(A[perm], p)[0], R)
        scale = rng.integers(1, p, size=(A.shape[0], 1)).astype(np.uint64)
        As = (A * scale) % p if p < (1 << 32) else A
        assert np.array_equal(oracle.rref(As, p)[0], R)
        R2, r2, piv2 = oracle.rref(R, p)
        assert np.array_equal(R2, R) and r2 == r and np.array_equal(piv2, piv)
        pins.is_rref(R, r, piv, p)


def test_rank_of_transpose():
    for case in workloads.small_cases(seed=51, count=32, max_dim=24, max_k=0):
        A, p = case["A"], case["p"]
        assert oracle.rref(A, p)[1] == oracle.rref(np.ascontiguousarray(A.T), p)[1]


def test_rank_factorisation_and_kernel():
    """A = C R and A K = 0 (Sec. 5.1) on low-rank products."""
    rng = np.random.default_rng(61)
    for p in (5, 65521, workloads.MERSENNE31):
        for m, n, r in [(10, 14, 6), (16, 9, 9), (12, 12, 0), (20, 20, 13)]:
            L = rng.integers(0, p, size=(m, r)).astype(np.uint64)
            U = rng.integers(0, p, size=(r, n)).astype(np.uint64)
            A = pins._mm(L, U, p).astype(np.uint64) if r else np.zeros((m, n), np.uint64)
            pins.check_rank_factorisation(_rref("c"), A, p)
            if p > 1000:  # product of random factors has full rank r w.h.p.
                assert oracle.rref(A, p)[1] == r


def test_identity_and_zero():
    p = 65521
    for m, n in [(5, 5), (3, 7), (7, 3)]:
        I = np.eye(m, n, dtype=np.uint64)
        R, r, piv = oracle.rref(I, p)
        assert np.array_equal(R, I) and r == min(m, n) and list(piv) == list(range(min(m, n)))
        Z = np.zeros((m, n), dtype=np.uint64)
        R, r, piv = oracle.rref(Z, p)
        assert r == 0 and not R.any() and len(piv) == 0


def test_empty_shapes():
    p = 7
    for m, n, k in [(0, 3, 2), (3, 0, 2), (0, 0, 0), (4, 4, 0)]:
        A = np.zeros((m, n), dtype=np.uint64)
        B = np.ones((m, k), dtype=np.uint64)
        X, r, piv, cons = oracle.solve(A, B, p)
        assert r == 0 and X.shape == (n, k)
        # a zero A is consistent only with a zero b; with no equations every b fits
        assert all(c == (1 if m == 0 else 0) for c in cons)


# --- arithmetic -----------------------------------------------------------

def test_inverse_exhaustive_and_fermat():
    p = 65521
    a = np.arange(1, p, dtype=np.uint64)
    inv = np.array([oracle.inv(int(v), p) for v in a], dtype=np.uint64)
    assert np.all(a * inv % p == 1)
    rng = np.random.default_rng(3)
    for q in (workloads.MERSENNE31, 2147483629, 1073741827, 2, 3):
        vals = [1, 2, q - 1, (q + 1) // 2] + [int(v) for v in rng.integers(1, q, size=200)]
        for v in vals:
            v %= q
            if v == 0:
                continue
            iv = oracle.inv(v, q)
            assert v * iv % q == 1
            assert iv == oracle.powmod(v, q - 2, q)


def test_miller_rabin_of_the_input_generator():
    """The prime draw of the seeded inputs: MR(2,7,61) equals trial division."""
    limit = 1 << 16
    sieve = np.ones(limit, dtype=bool)
    sieve[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = False
    for v in range(limit):
        assert workloads.is_prime_u32(v) == bool(sieve[v])
    for v in (2047, 3277, 4033, 4681, 8321, 561, 1105, 1729, 2465, 3215031751):
        assert not workloads.is_prime_u32(v)
    assert workloads.is_prime_u32(workloads.MERSENNE31)
    rng = np.random.default_rng(2)
    p = workloads.draw_prime31(rng)
    assert (1 << 30) <= p < (1 << 31) and workloads.is_prime_u32(p)


# --- agreement of the three implementations --------------------------------

def test_three_way_agreement_small_cases():
    for case in workloads.small_cases(seed=71, count=48, max_dim=14, max_k=4):
        A, B, p = case["A"], case["B"], case["p"]
        outs = [oracle.solve(A, B, p, impl=i) for i in IMPLS]
        for o in outs[1:]:
            assert np.array_equal(o[0], outs[0][0])
            assert o[1] == outs[0][1]
            assert np.array_equal(o[2], outs[0][2])
            assert np.array_equal(o[3], outs[0][3])
        X, r, piv, cons = outs[0]
        A64, B64, X64 = (np.asarray(v, dtype=np.int64) for v in (A, B, X))
        for t in range(B.shape[1]):
            if cons[t]:
                assert np.array_equal(pins._mm(A64, X64[:, t:t + 1], p)[:, 0], B64[:, t])


def test_c_and_numpy_agree_medium():
    for seed, n, k in [(1, 96, 3), (2, 130, 5)]:
        A, B, p = workloads.dense_system(seed, n, k)
        A[5] = A[3]  # rank deficient, B consistent on no column in general
        c = oracle.solve(A, B, p, impl="c")
        nump = oracle.solve(A, B, p, impl="numpy")
        for a, b in zip(c, nump):
            assert np.array_equal(np.asarray(a), np.asarray(b))


def test_batch_entry_matches_single():
    systems = workloads.batched_systems(seed=9, count=24, n_lo=8, n_hi=40, deficient_frac=0.25)
    many = oracle.solve_many(systems, threads=4)
    for s, got in zip(systems, many):
        ref = oracle.solve(s["A"], s["B"], s["p"])
        for a, b in zip(ref, got):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        if s["deficient"]:
            assert got[1] == s["n"] - 1 and got[3].all()


def test_certificate_c1():
    """The n=256 workload: full rank and A X = B exactly."""
    A, B, p = workloads.config("c1")
    X, r, piv, cons = oracle.solve(A, B, p)
    assert r == 256 and list(piv) == list(range(256)) and cons.all()
    assert np.array_equal(oracle.matmul_mod(A, X, p), B.astype(np.uint64))
    assert np.array_equal(oracle.matmul_mod(A, X, p), pins._mm(A, X, p).astype(np.uint64))
