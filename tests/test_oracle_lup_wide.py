"""Pins of the oracle's LUP factorisation and of its Gauss-Jordan for primes
up to 2^63 (runs without a GPU).

LUP (the paper's future work, Sec. 6; forward elimination with the first
non-zero pivot in the original row order):
* P A = L U exactly (Python-int products), L unit lower triangular, U in row
  echelon form with its leading entries at the pivot columns J and zero rows
  from the rank on;
* J equals the pivot columns of the RREF (pinned elsewhere), since both are
  the columns that raise the rank of the leading columns;
* the pivot rule, restated without elimination: perm[s] is the smallest row q
  outside perm[:s] whose first J[s] + 1 entries are not in the span of those
  of the rows perm[:s] (a rank test through the RREF oracle).  A row's
  reduced entry at J[s] is the remainder of its prefix after removing the
  span of the echelon pivot rows, so it is non-zero exactly then;
* the C (128-bit products) and Python-int statements agree, and planted
  mistakes in a copy fail the checks.

Gauss-Jordan for 31- to 63-bit primes (Sec. 3.2 "Number types"): the wide C
oracle equals the Python-int statement; on rank-r products L U the result has
rank r, is in RREF and A = A[:, J] R, which fixes R; Vandermonde systems
interpolate exactly.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from tests import certs, pins

P62 = 4611686018427387847   # 2^62 - 57, prime
P63 = 9223372036854775783   # 2^63 - 25, prime
PRIMES = [2, 3, 7, 65521, 2147483647, 4294967311, P62, P63]


def _rand(rng, shape, p):
    return np.array([[int(rng.integers(0, 2 ** 62)) % p for _ in range(shape[1])]
                     for _ in range(shape[0])], dtype=np.uint64).reshape(shape)


def _low_rank(rng, m, n, r, p):
    if r == 0:
        return np.zeros((m, n), dtype=np.uint64)
    return pins._mm(_rand(rng, (m, r), p), _rand(rng, (r, n), p), p).astype(np.uint64)


def _check_lup(A, p, out):
    LU, perm, r, J = out
    A = np.asarray(A, dtype=np.uint64)
    m, n = A.shape
    assert sorted(int(q) for q in perm) == list(range(m)), "perm is not a permutation"
    Pm, L, U = oracle.lup_factors(LU, perm, r, J, p)
    assert np.array_equal(pins._mm(Pm, A, p), pins._mm(L, U, p)), "P A != L U"
    assert np.all(np.triu(L.astype(object), 1) == 0) and np.all(np.diagonal(L) == 1)
    for i in range(m):
        if i < r:
            c = int(J[i])
            assert U[i, c] != 0 and not np.any(U[i, :c]), "U row is not echelon"
        else:
            assert not np.any(U[i]), "U row past the rank is not zero"
    _, rr, Jr = oracle.rref(A, p, impl="python")
    assert r == rr and list(J) == list(Jr), "pivots differ from the RREF's"
    # the pivot rule, by ranks of prefixes
    for s in range(r):
        cols = int(J[s]) + 1
        prev = [int(q) for q in perm[:s]]
        for q in range(m):
            if q in prev:
                continue
            sub = A[prev + [q], :cols]
            grows = oracle.rref(sub, p, impl="python")[1] == s + 1
            if q < perm[s]:
                assert not grows, f"row {q} should have been the pivot of step {s}"
            elif q == perm[s]:
                assert grows, f"pivot row {q} of step {s} does not raise the rank"
                break


@pytest.mark.parametrize("p", PRIMES)
def test_lup_random_and_low_rank(p):
    rng = np.random.default_rng(900 + p % 997)
    for _ in range(12):
        m, n = int(rng.integers(1, 7)), int(rng.integers(1, 7))
        r = int(rng.integers(0, min(m, n) + 1))
        A = _low_rank(rng, m, n, r, p) if rng.random() < 0.6 else _rand(rng, (m, n), p)
        if rng.random() < 0.3:
            A[:, int(rng.integers(0, n))] = 0
        c = oracle.lup(A, p, impl="c")
        py = oracle.lup(A, p, impl="python")
        for a, b in zip(c, py):
            assert np.array_equal(np.asarray(a), np.asarray(b)), "C and Python LUP differ"
        _check_lup(A, p, c)


def test_lup_edge_shapes():
    p = 101
    for A in (np.zeros((3, 4), np.uint64), np.eye(4, dtype=np.uint64), np.zeros((0, 3), np.uint64),
              np.zeros((2, 0), np.uint64), np.array([[0, 5], [3, 0]], np.uint64)):
        out = oracle.lup(A, p)
        if A.size:
            _check_lup(A, p, out)
        assert out[2] == oracle.rref(A, p)[1]
    # a row swap is forced: the first row starts with zero
    LU, perm, r, J = oracle.lup(np.array([[0, 5], [3, 0]], np.uint64), p)
    assert list(perm) == [1, 0] and r == 2


def _lup_mutant(kind):
    def lup(A, p):
        W = [[int(x) for x in row] for row in np.asarray(A).tolist()]
        m, n = len(W), len(W[0]) if W else 0
        is_piv, prow, J = [False] * m, [], []
        for j in range(n):
            cand = [q for q in range(m) if not is_piv[q] and W[q][j] % p]
            if not cand:
                continue
            r0 = cand[-1] if kind == "last_candidate" else cand[0]
            inv = pow(W[r0][j], p - 2, p)
            if kind == "normalised_pivot":
                W[r0] = [x * inv % p for x in W[r0]]
            for q in range(m):
                if q == r0 or is_piv[q] or W[q][j] == 0:
                    continue
                g = W[q][j] * inv % p
                if kind == "unnormalised_multiplier":
                    g = W[q][j]
                W[q][j] = g
                for c in range(j + 1, n):
                    W[q][c] = (W[q][c] - g * W[r0][c]) % p
            is_piv[r0] = True
            prow.append(r0)
            J.append(j)
        perm = np.array(prow + [q for q in range(m) if not is_piv[q]], dtype=np.int64)
        Wa = np.array(W, dtype=np.uint64).reshape(m, n)
        return Wa[perm], perm, len(prow), np.array(J, dtype=np.int64)
    return lup


@pytest.mark.parametrize("kind", ["last_candidate", "normalised_pivot", "unnormalised_multiplier"])
def test_lup_mutants_are_caught(kind):
    rng = np.random.default_rng(4)
    caught = False
    for _ in range(20):
        p = 7
        A = _rand(rng, (4, 4), p)
        try:
            _check_lup(A, p, _lup_mutant(kind)(A, p))
        except AssertionError:
            caught = True
            break
    assert caught


@pytest.mark.parametrize("p", [2147483647, 4294967311, P62, P63])
def test_wide_gauss_jordan(p):
    rng = np.random.default_rng(31 + p % 1009)
    for m, n, r in [(9, 12, 5), (14, 8, 8), (6, 6, 0), (10, 10, 10)]:
        A = _low_rank(rng, m, n, r, p)
        R, rr, J = oracle.rref(A, p)  # dispatches to the wide C oracle above 2^32
        Rp, rp, Jp = oracle.rref(A, p, impl="python")
        assert rr == rp == r and list(J) == list(Jp) and np.array_equal(R, Rp)
        pins.is_rref(R, rr, J, p)
        C = A[:, J]
        assert np.array_equal(pins._mm(C, R[:rr], p), np.asarray(A, dtype=object) % p), "A != C R"


def test_wide_vandermonde_interpolation():
    p = P62
    n = 12
    nodes = [int(x) for x in np.random.default_rng(2).choice(10 ** 12, size=n, replace=False)]
    V = np.array([[pow(x, c, p) for c in range(n)] for x in nodes], dtype=np.uint64)
    coef = np.array([[int(v)] for v in np.random.default_rng(3).integers(0, 2 ** 62, size=n)],
                    dtype=np.uint64) % np.uint64(p)
    b = pins._mm(V, coef, p).astype(np.uint64)
    X, r, J, cons = oracle.solve(V, b, p)
    assert r == n and cons[0] == 1
    assert np.array_equal(X, coef)
