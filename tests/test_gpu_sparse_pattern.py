"""GPU parity on the shared-sparsity-pattern family (rectangular, rank deficient,
full RREF with pivot columns).

At reduced size the RREF, rank and pivots are compared with the oracle bit for
bit on both paths.  At the full 12000 x 10000 size (the oracle would take
minutes per instance) four seeded instances are checked by properties that fix
the result:
* R is in reduced row-echelon form with r non-zero rows;
* every row of A is the combination of R's rows given by its own entries at
  the pivot columns, A = A[:, J] R[:r] (Freivalds' check over all 12000
  rows, two random vectors), so span(A) lies in span(R[:r]);
* the plain path, an independent kernel, reports the same rank, so
  dim span(A) = r = dim span(R[:r]) and the two spans are equal; the RREF of
  a row space is unique, so R is the RREF of A.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from tests import certs
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


@pytest.mark.parametrize("idx", [0, 21, 42, 63])
def test_sparse_pattern_full_size(gpu, idx):
    """One 12000 x 10000 instance of the family at full size (see the module
    docstring for why these checks fix the RREF)."""
    _, A = next(workloads.sparse_pattern_instances(instances=[idx]))
    print(f"pattern full size idx={idx}, blocked", flush=True)
    R, r, piv = _rref(A, lx.PATH_BLOCKED_INT8)
    print(f"rank {r}", flush=True)
    assert 0 < r <= 9500
    assert certs.is_rref_form(R, r, piv), "not in reduced row-echelon form"
    assert certs.freivalds_rank_factorisation(A, R, r, piv, P), "A != A[:, J] R on some row"
    print(f"pattern full size idx={idx}, plain", flush=True)
    Rp, rp, pivp = _rref(A, lx.PATH_PLAIN)
    assert r == rp and np.array_equal(piv, pivp), "plain and blocked ranks or pivots differ"
    assert np.array_equal(R, Rp), "plain and blocked RREFs differ"
