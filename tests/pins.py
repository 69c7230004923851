"""Checks that pin an RREF / solve implementation to mathematics, not to itself.

Each check takes the implementation under test as a callable, so the same
checks run on the oracle and on deliberately broken copies of it (the
mutation tests).  Every check raises AssertionError on failure.

Facts used (none of them re-derives the implementation's own formula):

* the reduced row-echelon form is unique and is characterised by its shape
  (leading ones, strictly increasing pivot columns, zero elsewhere in pivot
  columns, zero rows last) together with its row space (Sec. 3.2, Sec. 5.1);
* row operations preserve the solution set of A x = b; a system is
  consistent iff rank(A) = rank([A | b]) and then has p^(n-r) solutions over
  F_p (Sec. 5.2);
* det of a Vandermonde matrix is prod_{i<j} (x_j - x_i);
* A = C R with C = A[:, J] (rank factorisation) and A K = 0 for the
  canonical kernel K (Sec. 5.1).
"""

from __future__ import annotations

import itertools

import numpy as np


def is_rref(R, rank, pivots, p):
    R = np.asarray(R, dtype=np.int64)
    m, n = R.shape
    assert 0 <= rank <= min(m, n)
    assert len(pivots) == rank
    assert list(pivots) == sorted(set(int(c) for c in pivots)), "pivots not strictly increasing"
    assert np.all((R >= 0) & (R < p))
    for s in range(rank):
        c = int(pivots[s])
        assert R[s, c] == 1, "pivot entry is not 1"
        assert not np.any(R[s, :c]), "non-zero left of a pivot"
        col = R[:, c].copy()
        col[s] = 0
        assert not np.any(col), "pivot column not a unit vector"
    assert not np.any(R[rank:]), "rows below the rank are not zero"


def row_space(M, p):
    """All vectors of the row space of M over F_p (a set of tuples)."""
    M = np.asarray(M, dtype=np.int64)
    m, n = M.shape
    out = set()
    for coef in itertools.product(range(p), repeat=m):
        v = np.zeros(n, dtype=np.int64)
        for c, row in zip(coef, M):
            if c:
                v = (v + c * row) % p
        out.add(tuple(int(x) for x in v))
    return out


def check_rref_bruteforce(rref_fn, A, p):
    """RREF shape predicate + equal row space (enumerated) + rank = log_p |span|."""
    R, rank, piv = rref_fn(A, p)
    is_rref(R, rank, piv, p)
    span_a = row_space(A, p)
    span_r = row_space(np.asarray(R)[:rank] if rank else np.zeros((1, A.shape[1]), np.int64), p)
    assert span_a == span_r, "row space changed"
    assert len(span_a) == p ** rank, "rank disagrees with the size of the row space"


def check_solve_bruteforce(solve_fn, A, B, p):
    """Count every x in F_p^n; compare consistency, rank and the particular solution."""
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    m, n = A.shape
    X, rank, piv, cons = solve_fn(A, B, p)
    X = np.asarray(X, dtype=np.int64)
    free = [c for c in range(n) if c not in set(int(c) for c in piv)]
    assert len(free) == n - rank
    xs = np.array(list(itertools.product(range(p), repeat=n)), dtype=np.int64).reshape(-1, n)
    AX = (xs @ A.T) % p  # (#x, m)
    for t in range(B.shape[1]):
        count = int(np.sum(np.all(AX == B[:, t][None, :], axis=1)))
        if count:
            assert cons[t] == 1, "consistent system reported inconsistent"
            assert count == p ** (n - rank), "solution count is not p^(n-r)"
            assert np.array_equal((A @ X[:, t]) % p, B[:, t]), "X is not a solution"
            assert not np.any(X[free, t]), "free variables are not zero"
        else:
            assert cons[t] == 0, "inconsistent system reported consistent"
            assert not np.any(X[:, t]), "inconsistent column of X is not zero"


def vandermonde(nodes, ncols, p):
    nodes = [int(x) for x in nodes]
    return np.array([[pow(x, c, p) for c in range(ncols)] for x in nodes], dtype=np.uint64)


def vandermonde_det(nodes, p):
    d = 1
    nodes = [int(x) for x in nodes]
    for i in range(len(nodes)):
        for j in range(i + 1, len(nodes)):
            d = d * (nodes[j] - nodes[i]) % p
    return d


def check_rank_factorisation(rref_fn, A, p):
    """A = C R with C = A[:, J], and A K = 0 with K of width n - r."""
    A = np.asarray(A, dtype=np.int64)
    R, rank, piv = rref_fn(A, p)
    R = np.asarray(R, dtype=np.int64)[:rank]
    C = A[:, list(int(c) for c in piv)]
    assert np.array_equal(_mm(C, R, p), A % p), "A != C R"
    n = A.shape[1]
    free = [c for c in range(n) if c not in set(int(c) for c in piv)]
    K = np.zeros((n, len(free)), dtype=np.int64)
    for f, c in enumerate(free):
        K[c, f] = p - 1
        for s, pc in enumerate(piv):
            K[int(pc), f] = R[s, c]
    assert not np.any(_mm(A, K, p)), "A K != 0"


def _mm(A, B, p):
    """Exact (A @ B) mod p with Python ints (small sizes)."""
    A = np.asarray(A, dtype=object)
    B = np.asarray(B, dtype=object)
    if A.shape[1] == 0:
        return np.zeros((A.shape[0], B.shape[1]), dtype=np.int64)
    return (A.dot(B) % p).astype(np.int64)
