"""Pins of the oracle's applications of the RREF (Sec. 5.1): the canonical
null-space basis and the removal of the bottom zero rows (runs without a GPU).

The canonical kernel K of A is fixed by two facts that do not use its own
construction: every column of K lies in ker(A) (checked with Python-int
products), and K restricted to the free (non-pivot) variables is -I.  A kernel
vector is determined by its free coordinates (the pivot variables follow from
them), so exactly one matrix has both properties; its width n - r is the
dimension of ker(A), which brute-force enumeration confirms on tiny fields.
Planted mistakes (a +I block, a transposed row/column index, a dropped row
copy) must fail these checks.
"""

from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
import workloads
from tests import pins


def _check_kernel(A, p, K, pivots):
    A = np.asarray(A, dtype=np.int64)
    m, n = A.shape
    K = np.asarray(K, dtype=np.int64)
    free = [c for c in range(n) if c not in set(int(c) for c in pivots)]
    assert K.shape == (n, len(free)), "kernel width is not n - r"
    assert np.all((K >= 0) & (K < p))
    if K.shape[1]:
        assert not np.any(pins._mm(A, K, p)), "a column of K is not in ker(A)"
        minus_i = (np.eye(len(free), dtype=np.int64) * (p - 1)) % p
        assert np.array_equal(K[free], minus_i), "free rows of K are not -I"


def _kernel_dim_bruteforce(A, p):
    A = np.asarray(A, dtype=np.int64)
    n = A.shape[1]
    xs = np.array(list(itertools.product(range(p), repeat=n)), dtype=np.int64).reshape(-1, n)
    return int(np.sum(~np.any((xs @ A.T) % p, axis=1)))


@pytest.mark.parametrize("p", [2, 3, 5])
def test_canonical_kernel_bruteforce(p):
    rng = np.random.default_rng(700 + p)
    for _ in range(40):
        m, n = int(rng.integers(1, 5)), int(rng.integers(1, 6))
        A = rng.integers(0, p, size=(m, n)).astype(np.uint64)
        if rng.random() < 0.4 and m > 1:
            A[-1] = (A[0] * int(rng.integers(0, p))) % p
        R, r, piv = oracle.rref(A, p)
        K = oracle.canonical_kernel(R, piv, n, p)
        _check_kernel(A, p, K, piv)
        assert _kernel_dim_bruteforce(A, p) == p ** K.shape[1], "dim ker(A) != n - r"


def test_canonical_kernel_structured():
    """Low-rank products over a 31-bit field and edge shapes."""
    rng = np.random.default_rng(71)
    p = workloads.MERSENNE31
    for m, n, r in [(10, 14, 6), (16, 9, 9), (12, 12, 0), (5, 30, 4), (1, 1, 1), (3, 1, 0)]:
        L = workloads.uniform(rng, (m, r), p).astype(np.uint64)
        U = workloads.uniform(rng, (r, n), p).astype(np.uint64)
        A = pins._mm(L, U, p).astype(np.uint64) if r else np.zeros((m, n), np.uint64)
        R, rr, piv = oracle.rref(A, p)
        assert rr == r
        _check_kernel(A, p, oracle.canonical_kernel(R, piv, n, p), piv)
    # identity: no kernel; zero matrix: K = -I
    I = np.eye(6, dtype=np.uint64)
    R, r, piv = oracle.rref(I, 7)
    assert oracle.canonical_kernel(R, piv, 6, 7).shape == (6, 0)
    Z = np.zeros((4, 5), dtype=np.uint64)
    R, r, piv = oracle.rref(Z, 7)
    assert np.array_equal(oracle.canonical_kernel(R, piv, 5, 7), 6 * np.eye(5, dtype=np.uint64))


def _kernel_mutant(kind):
    def K(R, pivots, n, p):
        R = np.asarray(R).astype(np.int64)
        piv = [int(c) for c in pivots]
        free = [c for c in range(n) if c not in set(piv)]
        out = np.zeros((n, len(free)), dtype=np.int64)
        for f, c in enumerate(free):
            out[c, f] = 1 if kind == "plus_identity" else p - 1
            for s, pc in enumerate(piv):
                if kind == "dropped_row" and s == 0:
                    continue
                if kind == "transposed":
                    out[pc, f] = R[min(c, R.shape[0] - 1), min(s, R.shape[1] - 1)] % p
                else:
                    out[pc, f] = R[s, c] % p
        return out.astype(np.uint64)
    return K


@pytest.mark.parametrize("kind", ["plus_identity", "dropped_row", "transposed"])
def test_kernel_mutants_are_caught(kind):
    rng = np.random.default_rng(9)
    caught = False
    for _ in range(30):
        p = 5
        A = rng.integers(0, p, size=(3, 5)).astype(np.uint64)
        R, r, piv = oracle.rref(A, p)
        try:
            _check_kernel(A, p, _kernel_mutant(kind)(R, piv, 5, p), piv)
        except AssertionError:
            caught = True
            break
    assert caught


def test_drop_bottom_zero_rows():
    """The number of kept rows of an RREF equals the rank found by brute force,
    the kept rows are the first rows, and interior zero rows of a matrix that is
    not an RREF are kept (only the bottom run is removed)."""
    rng = np.random.default_rng(13)
    for p in (2, 3):
        for _ in range(30):
            m, n = int(rng.integers(1, 5)), int(rng.integers(1, 5))
            A = rng.integers(0, p, size=(m, n)).astype(np.uint64)
            R, r, piv = oracle.rref(A, p)
            D = oracle.drop_bottom_zero_rows(R)
            span = pins.row_space(A, p)
            assert len(span) == p ** D.shape[0], "kept rows != rank"
            assert np.array_equal(D, R[: D.shape[0]])
    M = np.array([[1, 0], [0, 0], [0, 2], [0, 0], [0, 0]], dtype=np.uint64)
    assert np.array_equal(oracle.drop_bottom_zero_rows(M), M[:3])
    assert oracle.drop_bottom_zero_rows(np.zeros((3, 2), np.uint64)).shape == (0, 2)
    assert np.array_equal(oracle.drop_bottom_zero_rows(np.eye(3, dtype=np.uint64)),
                          np.eye(3, dtype=np.uint64))
    assert oracle.drop_bottom_zero_rows(np.zeros((0, 4), np.uint64)).shape == (0, 4)
