"""GPU parity of the column-step paths through the C ABI: Gauss-Jordan for
64-bit primes (linac_rref_u64 / linac_solve_u64, Sec. 3.2 "Number types") and
the LUP factorisation with the fixed pivot rule (linac_lup / linac_lup_u64,
the paper's future work of Sec. 6), against the oracle bit for bit.

Shapes span several 32-row tiles and column chunks with ragged tails (the
64-bit update kernel takes 128 columns per chunk, the 32-bit one 256), are
rectangular both ways, rank deficient, with free columns and all-zero
columns, and include empty dimensions.  Primes: 2, 3, 65521, 2^31 - 1, a
33-bit prime, 2^62 - 57 and 2^63 - 25.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
import paper_2605_25863_amd as lx

pytestmark = pytest.mark.gpu

P33 = 4294967311
P62 = 4611686018427387847
P63 = 9223372036854775783


def _matrix(rng, m, n, p, kind):
    A = np.array(rng.integers(0, 2 ** 63 - 1, size=(m, n), dtype=np.int64), dtype=np.uint64)
    A %= np.uint64(p)
    if kind == "deficient" and m > 2:
        A[m - 1] = A[0]
        A[m // 2] = 0
    if kind == "freecols" and n > 3:
        A[:, 1] = 0
        A[:, n // 2] = A[:, 0]
    if kind == "lowrank" and m > 4 and n > 4:
        r = min(m, n) // 3
        L = A[:, :r] % np.uint64(min(p, 1 << 20))
        U = A[:r, :] % np.uint64(min(p, 1 << 20))
        A = np.array((L.astype(object).dot(U.astype(object))) % p, dtype=np.uint64)
    return A


CASES = [(70, 300, "dense"), (300, 70, "dense"), (129, 129, "deficient"), (64, 257, "freecols"),
         (90, 90, "lowrank"), (1, 1, "dense"), (33, 0, "dense"), (0, 17, "dense")]


@pytest.mark.parametrize("p", [2, 65521, workloads.MERSENNE31, P33, P62, P63])
def test_rref_and_solve_u64_match_oracle(gpu, p):
    rng = np.random.default_rng(p % 100003)
    for m, n, kind in CASES:
        A = _matrix(rng, m, n, p, kind)
        tag = f"u64 p={p} {m}x{n} {kind}"
        print(tag, flush=True)
        R, r, piv = lx.rref_u64(A, p)
        Rr, rr, pr = oracle.rref(A, p, impl="c_wide")
        assert r == rr and np.array_equal(piv, pr), tag
        assert np.array_equal(R, Rr.astype(np.uint64)), tag
        k = 3
        B = _matrix(rng, m, k, p, "dense")
        if m > 3:
            B[:, 1] = 0  # consistent whatever the rank
        X, r2, piv2, cons = lx.solve_u64(A, B, p)
        Xo, ro, po, co = oracle.solve(A, B, p, impl="c_wide")
        assert r2 == ro and np.array_equal(piv2, po) and np.array_equal(cons, co), tag
        assert np.array_equal(X, Xo.astype(np.uint64)), tag


def test_u64_larger_dense(gpu):
    rng = np.random.default_rng(8)
    A = _matrix(rng, 600, 600, P62, "dense")
    B = _matrix(rng, 600, 4, P62, "dense")
    X, r, piv, cons = lx.solve_u64(A, B, P62)
    Xo, ro, po, co = oracle.solve(A, B, P62, impl="c_wide")
    assert r == ro == 600 and np.array_equal(X, Xo.astype(np.uint64)) and np.all(cons == 1)


@pytest.mark.parametrize("p", [3, 65521, workloads.MERSENNE31, P33, P62, P63])
def test_lup_matches_oracle(gpu, p):
    rng = np.random.default_rng(7 + p % 10007)
    for m, n, kind in CASES:
        A = _matrix(rng, m, n, p, kind)
        if p < 2 ** 31:
            A = A.astype(np.uint32)
        tag = f"lup p={p} {m}x{n} {kind}"
        print(tag, flush=True)
        LU, perm, r, piv = lx.lup(A, p)
        LUo, permo, ro, pivo = oracle.lup(A, p)
        assert r == ro and np.array_equal(piv, pivo), tag
        assert np.array_equal(perm, permo), tag
        assert np.array_equal(LU.astype(np.uint64), LUo), tag


def test_lup_factorisation_certificate(gpu):
    """P A = L U on a 500 x 480 rank-deficient matrix (Freivalds' check with two
    random vectors, all products mod p exact)."""
    p = workloads.MERSENNE31
    rng = np.random.default_rng(12)
    A = workloads.uniform(rng, (500, 480), p)
    A[400:] = A[:100]
    LU, perm, r, piv = lx.lup(A, p)
    assert r == 400
    Pm, L, U = oracle.lup_factors(LU, perm, r, piv, p)
    for s in (1, 2):
        v = np.random.default_rng(s).integers(0, p, size=(480, 1), dtype=np.uint64)
        lhs = oracle.matmul_mod(A[perm], v, p)
        rhs = oracle.matmul_mod(L, oracle.matmul_mod(U, v, p), p)
        assert np.array_equal(lhs, rhs)


def test_validate_range_u64(gpu):
    A = np.array([[1, 2], [3, P62]], dtype=np.uint64)
    with pytest.raises(lx.LinacError) as err:
        lx.rref_u64(A, P62, validate=True)
    assert err.value.status == 4
    with pytest.raises(lx.LinacError) as err:
        lx.lup(A, P62, validate=True)
    assert err.value.status == 4
