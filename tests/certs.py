"""Certificates for results too large for the oracle (full-size workloads).

Freivalds' check: for a claimed identity X = Y Z over F_p, a uniformly random
vector v gives X v = Y (Z v) always when the identity holds, and with
probability at most 1/p when some entry differs (each independent v).  The
products are matrix-vector products mod p (oracle.matmul_mod, exact), so a
check costs O(rows x columns) instead of a matrix product.
"""

from __future__ import annotations

import numpy as np

import oracle


def _vec(rng, n, p):
    return rng.integers(0, p, size=(n, 1), dtype=np.uint64)


def freivalds_rank_factorisation(A, R, r, piv, p, seeds=(1, 2)):
    """A = A[:, J] R[:r] on every row of A (Sec. 5.1): every row of A is the
    combination of R's rows given by its own entries at the pivot columns, so
    span(A) lies in span(R[:r])."""
    A = np.asarray(A)
    Rr = np.asarray(R)[:r]
    C = A[:, np.asarray(piv, dtype=np.int64)]
    for s in seeds:
        v = _vec(np.random.default_rng(s), A.shape[1], p)
        lhs = oracle.matmul_mod(A, v, p)
        rhs = oracle.matmul_mod(C, oracle.matmul_mod(Rr, v, p), p) if r else np.zeros_like(lhs)
        if not np.array_equal(lhs, rhs):
            return False
    return True


def freivalds_solution(A, X, B, p, seeds=(1, 2)):
    """A X = B on every row and every right-hand side, tested on random
    combinations of the right-hand sides."""
    A = np.asarray(A)
    X = np.asarray(X)
    B = np.asarray(B)
    for s in seeds:
        v = _vec(np.random.default_rng(s), X.shape[1], p)
        lhs = oracle.matmul_mod(A, oracle.matmul_mod(X, v, p), p)
        if not np.array_equal(lhs, oracle.matmul_mod(B, v, p)):
            return False
    return True


def is_rref_form(R, r, piv):
    """Leading ones at strictly increasing pivot columns, zero to their left,
    unit pivot columns, zero rows from r on (no arithmetic needed)."""
    R = np.asarray(R)
    piv = np.asarray(piv, dtype=np.int64)
    if len(piv) != r or np.any(np.diff(piv) <= 0) or np.any(R[r:]):
        return False
    for i, c in enumerate(piv):
        if R[i, c] != 1 or np.any(R[i, :c]):
            return False
    sub = R[:r][:, piv]
    return int(np.count_nonzero(sub)) == r and bool(np.all(np.diagonal(sub) == 1))
