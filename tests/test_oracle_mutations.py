"""Planted mistakes in a copy of the oracle must fail the pins.

Each mutant is the Python-int Gauss-Jordan with one plausible slip (a
dropped term, a wrong sign, a wrong index, a transposed operand, a skipped
step).  The test passes only if at least one pin of tests/pins.py rejects the
mutant, which shows the pins would catch that class of bug in the oracle.
"""

from __future__ import annotations

import numpy as np
import pytest

import workloads
from tests import pins


def _gj(M, nsearch, p, bug):
    shape = np.asarray(M).shape
    M = [[int(x) for x in row] for row in np.asarray(M).tolist()]
    m, ncols = shape
    i = 0
    piv = []
    for j in range(nsearch):
        if i == m:
            break
        nz = [q for q in range(i, m) if M[q][j] % p != 0]
        if not nz:
            continue
        r = nz[0]
        if bug != "no_swap":
            M[i], M[r] = M[r], M[i]
        else:
            i_row = r
        head = M[i][j] if bug != "no_swap" else M[i_row][j]
        if bug == "no_swap":
            # normalise and use row r in place, leaving row order unsorted
            M[i_row] = [x * pow(head, p - 2, p) % p for x in M[i_row]]
            src = i_row
        else:
            e = p - 2 if bug != "bad_exponent" else p - 1
            M[i] = [x * pow(head, e, p) % p for x in M[i]] if bug != "no_normalise" else M[i]
            src = i
        for q in range(m):
            if q == src:
                continue
            if bug == "forward_only" and q < src:
                continue  # drops the rows above the pivot (REF, not RREF)
            f = M[q][j] if bug != "wrong_index" else M[q][min(j + 1, ncols - 1)]
            if f == 0:
                continue
            if bug == "wrong_sign":
                M[q] = [(a + f * b) % p for a, b in zip(M[q], M[src])]
            elif bug == "transposed":
                M[q] = [(a - f * M[src][c2] ) % p for c2, a in
                        zip([min(c, m - 1) for c in range(ncols)], M[q])]
            else:
                M[q] = [(a - f * b) % p for a, b in zip(M[q], M[src])]
        piv.append(j)
        i += 1
    return np.array(M, dtype=np.uint64).reshape(m, ncols), i, np.array(piv, dtype=np.int64)


def _mutant(bug):
    def rref(A, p):
        return _gj(A, np.asarray(A).shape[1], p, bug)

    def solve(A, B, p):
        A = np.asarray(A)
        B = np.asarray(B)
        n, k = A.shape[1], B.shape[1]
        R, r, piv = _gj(np.concatenate([A, B], axis=1), n, p, bug)
        cons = np.array([not np.any(R[r:, n + t]) for t in range(k)], dtype=np.uint8)
        X = np.zeros((n, k), dtype=np.uint64)
        for s, c in enumerate(piv):
            X[c] = R[s, n:]
        X[:, cons == 0] = 0
        return X, r, piv, cons

    return rref, solve


def _all_pins_pass(rref, solve) -> bool:
    try:
        rng = np.random.default_rng(5)
        for p in (3, 5):
            for _ in range(25):
                m, n = int(rng.integers(2, 4)), int(rng.integers(2, 4))
                A = rng.integers(0, p, size=(m, n)).astype(np.uint64)
                pins.check_rref_bruteforce(rref, A, p)
                B = rng.integers(0, p, size=(m, 2)).astype(np.uint64)
                pins.check_solve_bruteforce(solve, A, B, p)
        p = 65521
        x = workloads.vandermonde_nodes(seed=3, count=8, p=p)
        V = pins.vandermonde(x, 8, p)
        R, r, piv = rref(V, p)
        pins.is_rref(R, r, piv, p)
        pins.check_rank_factorisation(rref, V, p)
    except (AssertionError, IndexError, ValueError):
        return False
    return True


def test_reference_copy_passes():
    assert _all_pins_pass(*_mutant("none"))


@pytest.mark.parametrize("bug", ["no_swap", "bad_exponent", "no_normalise", "forward_only",
                                 "wrong_index", "wrong_sign", "transposed"])
def test_mutant_is_caught(bug):
    assert not _all_pins_pass(*_mutant(bug))
