"""GPU parity on the shared-sparsity-pattern family (rectangular, rank deficient,
full RREF with pivot columns).

At reduced size the RREF, rank and pivots are compared with the oracle bit for
bit on both paths.  At the full 12000 x 10000 size (the oracle would take
minutes) the result is checked by properties that fix it: reduced row-echelon
form, the same rank and pivots on the plain and blocked paths, and every
sampled row of A equal to the combination of R's rows given by its entries at
the pivot columns (so span(A) lies in span(R), and equal ranks make the spans
equal; the RREF of a row space is unique).
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
import paper_2605_25863_amd as lx

pytestmark = pytest.mark.gpu

P = workloads.MERSENNE31


def _rref(A, path, panel=0):
    import torch
    R, rank, piv = lx.rref(A, P, path=path, panel_width=panel)
    torch.cuda.synchronize()
    r = int(rank.item())
    return R.cpu().numpy().astype(np.uint32), r, piv.cpu().numpy()[:r].astype(np.int64)


@pytest.mark.parametrize("path,panel", [(lx.PATH_BLOCKED_INT8, 64), (lx.PATH_BLOCKED_INT8, 256),
                                        (lx.PATH_PLAIN, 0)])
def test_sparse_pattern_reduced(gpu, path, panel):
    for idx, A in workloads.sparse_pattern_instances(seed=55, count=3, m=1200, n=1000,
                                                    base_rows=950, nnz=20):
        tag = f"pattern reduced idx={idx} path={path} panel={panel}"
        print(tag, flush=True)
        R, r, piv = _rref(A, path, panel)
        Rr, rr, pr = oracle.rref(A, P)
        assert r == rr, f"{tag}: rank {r} vs {rr}"
        assert np.array_equal(piv, pr), f"{tag}: pivots"
        assert np.array_equal(R, Rr), f"{tag}: RREF"


def _check_rref_form(R, r, piv):
    m, n = R.shape
    assert np.all(R[r:] == 0)
    assert np.all(np.diff(piv) > 0)
    for i, c in enumerate(piv):
        assert R[i, c] == 1
        assert np.all(R[i, :c] == 0)
    # pivot columns are unit vectors
    assert np.array_equal(R[:r][:, piv], np.eye(r, dtype=np.uint32))


def test_sparse_pattern_full_size(gpu):
    """One 12000 x 10000 instance of the family at full size."""
    _, A = next(workloads.sparse_pattern_instances(instances=[0]))
    print("pattern full size, blocked", flush=True)
    R, r, piv = _rref(A, lx.PATH_BLOCKED_INT8)
    print(f"rank {r}", flush=True)
    _check_rref_form(R, r, piv)
    print("pattern full size, plain", flush=True)
    Rp, rp, pivp = _rref(A, lx.PATH_PLAIN)
    assert r == rp and np.array_equal(piv, pivp)
    rows = np.random.default_rng(5).choice(A.shape[0], size=6, replace=False)
    Ar = A[rows].astype(np.uint64)
    comb = oracle.matmul_mod(Ar[:, piv], R[:r], P)
    assert np.array_equal(comb, Ar), "a sampled row of A is not in span(R)"
    # both paths agree on sampled rows of R
    for i in np.random.default_rng(6).choice(r, size=16, replace=False):
        assert np.array_equal(R[i], Rp[i])
