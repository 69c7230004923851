"""The full-size certificates accept the oracle's results and reject planted
mistakes (runs without a GPU)."""

from __future__ import annotations

import numpy as np

import oracle
import workloads
from tests import certs


def _family(m=600, n=500):
    _, A = next(workloads.sparse_pattern_instances(seed=77, count=1, m=m, n=n, base_rows=450,
                                                   nnz=12))
    return A


def test_rank_factorisation_certificate():
    p = workloads.MERSENNE31
    A = _family()
    R, r, piv = oracle.rref(A, p)
    assert certs.is_rref_form(R, r, piv)
    assert certs.freivalds_rank_factorisation(A, R, r, piv, p)
    rng = np.random.default_rng(3)
    for _ in range(5):  # one wrong entry of R outside the pivot columns
        Rb = R.copy()
        i = int(rng.integers(0, r))
        free = [c for c in range(A.shape[1]) if c not in set(piv.tolist()) and c > piv[i]]
        c = free[int(rng.integers(0, len(free)))]
        Rb[i, c] = (int(Rb[i, c]) + 1 + int(rng.integers(0, p - 1))) % p
        assert certs.is_rref_form(Rb, r, piv)
        assert not certs.freivalds_rank_factorisation(A, Rb, r, piv, p)
    # a row of R past the rank made non-zero, or a pivot moved
    Rb = R.copy()
    Rb[r, -1] = 1
    assert not certs.is_rref_form(Rb, r, piv)
    Rb = R.copy()
    Rb[0, piv[0]] = 2
    assert not certs.is_rref_form(Rb, r, piv)


def test_solution_certificate():
    A, B, p = workloads.config("c2", n=300)
    X, r, piv, cons = oracle.solve(A, B, p)
    assert r == 300 and cons.all()
    assert certs.freivalds_solution(A, X, B, p)
    Xb = X.copy()
    Xb[17, 5] = (int(Xb[17, 5]) + 1) % p
    assert not certs.freivalds_solution(A, Xb, B, p)
