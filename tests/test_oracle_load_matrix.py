"""Pins of the oracle's system construction (Sec. 3.3): A[r, c] is the
product of the bases entries of row r that column c's index list names
(runs without a GPU).

The checks rest on facts that do not reuse the oracle's own loop:

* powers: with bases[r, v] = x_r^(e_v), the monomial of column c evaluates to
  x_r^(sum_t e_{lindices[c, t]}), which pow() gives directly;
* Vandermonde: bases[r] = [1, x_r] and column c listing c ones padded with
  the dummy variable (index 0, value 1; the padding convention of the
  paper's helper that pads shorter monomials) gives A[r, c] = x_r^c, whose
  determinant is the closed form prod_{i<j} (x_j - x_i);
* one index per column is a plain column gather of bases;
* splitting each index list in two gives the entrywise product of the two
  smaller matrices (the product is commutative and associative);
* the numpy (reduce after every factor) and Python-int (reduce once)
  statements agree, and a planted mistake in a copy fails these checks.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests import pins


def _powers_case(rng, p, nrows, nbasis, ncols, d):
    x = rng.integers(1, p, size=nrows)
    e = rng.integers(0, 50, size=nbasis)
    bases = np.array([[pow(int(xr), int(ev), p) for ev in e] for xr in x], dtype=np.uint64)
    L = rng.integers(0, nbasis, size=(ncols, d))
    want = np.array([[pow(int(xr), int(sum(e[L[c]])), p) for c in range(ncols)] for xr in x],
                    dtype=np.uint64)
    return bases, L, want


@pytest.mark.parametrize("p", [2, 7, 65521, 2147483647])
@pytest.mark.parametrize("impl", ["numpy", "python"])
def test_powers_closed_form(p, impl):
    rng = np.random.default_rng(31 + p % 1000)
    for nrows, nbasis, ncols, d in [(6, 5, 9, 3), (4, 1, 3, 7), (3, 8, 5, 1), (5, 4, 4, 12)]:
        bases, L, want = _powers_case(rng, p, nrows, nbasis, ncols, d)
        got = oracle.load_matrix(bases, L, p, impl=impl)
        assert np.array_equal(got.astype(np.uint64), want)


def test_vandermonde_with_dummy_padding():
    p = 2147483647
    rng = np.random.default_rng(5)
    n, d = 9, 8
    x = rng.choice(np.arange(2, 10 ** 6), size=n, replace=False)
    bases = np.array([[1, int(v)] for v in x], dtype=np.uint64)
    L = np.array([[1] * c + [0] * (d - c) for c in range(n)])  # degree c <= d
    A = oracle.load_matrix(bases, L, p)
    assert np.array_equal(A.astype(np.uint64), pins.vandermonde(x, n, p))
    assert oracle.det(A, p) == pins.vandermonde_det(x, p)
    # a repeated node gives a singular matrix
    bases[3] = bases[6]
    assert oracle.det(oracle.load_matrix(bases, L, p), p) == 0


def test_single_index_is_a_gather_and_empty_product_is_one():
    p = 1000003
    rng = np.random.default_rng(6)
    bases = rng.integers(0, p, size=(7, 11)).astype(np.uint64)
    L = rng.integers(0, 11, size=(13, 1))
    assert np.array_equal(oracle.load_matrix(bases, L, p), bases[:, L[:, 0]].astype(np.uint32))
    assert np.array_equal(oracle.load_matrix(bases, np.zeros((4, 0), np.int64), p),
                          np.ones((7, 4), np.uint32))
    assert oracle.load_matrix(bases, np.zeros((0, 3), np.int64), p).shape == (7, 0)
    assert oracle.load_matrix(np.zeros((0, 11), np.uint64), L, p).shape == (0, 13)


def test_split_index_lists_multiply_entrywise():
    p = 2147483647
    rng = np.random.default_rng(8)
    bases = rng.integers(0, p, size=(10, 20)).astype(np.uint64)
    L1 = rng.integers(0, 20, size=(15, 4))
    L2 = rng.integers(0, 20, size=(15, 5))
    A = oracle.load_matrix(bases, np.concatenate([L1, L2], axis=1), p).astype(object)
    B1 = oracle.load_matrix(bases, L1, p).astype(object)
    B2 = oracle.load_matrix(bases, L2, p).astype(object)
    assert np.array_equal(A, (B1 * B2) % p)
    # the order of the indices within a monomial does not matter
    perm = rng.permuted(np.concatenate([L1, L2], axis=1), axis=1)
    assert np.array_equal(oracle.load_matrix(bases, perm, p).astype(object), A)


def test_out_of_range_index_is_a_zero_factor():
    p = 101
    bases = np.arange(1, 13, dtype=np.uint64).reshape(3, 4)
    L = np.array([[0, 4], [-1, 1], [2, 3]])
    A = oracle.load_matrix(bases, L, p)
    assert not np.any(A[:, :2])
    assert np.array_equal(A[:, 2], (bases[:, 2] * bases[:, 3] % p).astype(np.uint32))
    assert np.array_equal(A, oracle.load_matrix(bases, L, p, impl="python"))


def _mutant(kind):
    def load(bases, lindices, p):
        B = np.asarray(bases, dtype=np.int64)
        L = np.asarray(lindices, dtype=np.int64)
        nrows, ncols, d = B.shape[0], L.shape[0], L.shape[1]
        A = np.ones((nrows, ncols), dtype=object)
        for r in range(nrows):
            for c in range(ncols):
                ts = range(d - 1) if kind == "dropped_factor" else range(d)
                for t in ts:
                    i = int(L[c, t])
                    if kind == "off_by_one":
                        i = min(i + 1, B.shape[1] - 1)
                    v = int(B[r, i])
                    A[r, c] = A[r, c] + v if kind == "sum_not_product" else A[r, c] * v
        return (A % p).astype(np.uint32)
    return load


@pytest.mark.parametrize("kind", ["dropped_factor", "off_by_one", "sum_not_product"])
def test_planted_mistakes_fail_the_closed_form(kind):
    rng = np.random.default_rng(17)
    p = 65521
    bases, L, want = _powers_case(rng, p, 4, 6, 7, 3)
    assert np.array_equal(oracle.load_matrix(bases, L, p).astype(np.uint64), want)
    assert not np.array_equal(_mutant(kind)(bases, L, p).astype(np.uint64), want)
