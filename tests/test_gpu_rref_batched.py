"""GPU parity of linac_rref_batched (many RREFs in one call, reduced
concurrently on the library's stream lanes) against the oracle, through the
C ABI.

* a mixed batch (plain-path and blocked-path sizes, rectangular, rank
  deficient, one prime per matrix) against the oracle bit for bit, with 1, 2,
  3 and 8 lanes (the tuning key rref_lanes; results never depend on it);
* the shared-sparsity-pattern family at reduced size against the oracle;
* the full sparse-pattern workload, all 64 instances of 12000 x 10000 in one
  call: every instance has rank 9500 and is in reduced row-echelon form;
  instances 0, 21, 42 and 63 pass Freivalds' check A = A[:, J] R over all
  12000 rows and equal a single linac_rref call; instance 21 equals the C
  oracle's RREF bit for bit.
"""

from __future__ import annotations

import json

import numpy as np
import pytest

import oracle
import workloads
from tests import certs
import paper_2605_25863_amd as lx

pytestmark = pytest.mark.gpu

P = workloads.MERSENNE31


def _mixed_batch():
    rng = np.random.default_rng(404)
    mats, primes = [], []
    shapes = [(300, 300), (257, 420), (600, 380), (64, 64), (1, 5), (0, 4), (45, 0), (700, 700),
              (130, 900), (520, 520)]
    for i, (m, n) in enumerate(shapes):
        p = [P, 65521, 2, workloads.draw_prime31(rng)][i % 4]
        A = workloads.uniform(rng, (m, n), p)
        if m > 3 and n > 0:
            A[m // 2] = A[1]  # rank deficient
            A[:, n // 3] = 0  # a free column
        mats.append(A)
        primes.append(p)
    return mats, primes


def _check_against_oracle(mats, primes, tag):
    got = lx.rref_batched(mats, primes)
    for i, (A, p, (R, r, piv)) in enumerate(zip(mats, primes, got)):
        Rr, rr, pr = oracle.rref(A, p)
        assert r == rr, f"{tag} matrix {i}: rank {r} vs {rr}"
        assert np.array_equal(piv, pr), f"{tag} matrix {i}: pivots"
        assert np.array_equal(R, Rr), f"{tag} matrix {i}: RREF"


@pytest.mark.parametrize("lanes", [1, 2, 3, 8])
def test_mixed_batch_matches_oracle(gpu, lanes):
    mats, primes = _mixed_batch()
    table = json.load(open(lx.TUNING_FILE))
    table["rref_lanes"] = lanes
    lx.load_tuning(json.dumps(table))
    try:
        print(f"mixed batch, {lanes} lanes", flush=True)
        _check_against_oracle(mats, primes, f"lanes={lanes}")
    finally:
        lx.restore_tuning()


def test_sparse_pattern_reduced_batch(gpu):
    mats = [A for _, A in workloads.sparse_pattern_instances(seed=56, count=6, m=1200, n=1000,
                                                            base_rows=950, nnz=20)]
    _check_against_oracle(mats, [P] * len(mats), "pattern reduced")


def test_sparse_pattern_full_batch(gpu):
    import torch
    dev = torch.device("cuda", 0)
    count = 64
    mats = [A for _, A in workloads.sparse_pattern_instances_torch(dev, count=count)]
    keep = {i: mats[i].cpu().numpy().astype(np.uint32) for i in (0, 21, 42, 63)}
    print("full batch: 64 instances in one call", flush=True)
    outs = lx.rref_batched(mats, P, inplace=True)
    torch.cuda.synchronize()
    ranks = [int(r.item()) for _, r, _ in outs]
    assert ranks == [9500] * count, sorted(set(ranks))
    for i, (R, rank, piv) in enumerate(outs):
        r = ranks[i]
        pv = piv.cpu().numpy()[:r]
        # form checks on the device copy: pivot entries 1, rows past r zero
        assert not bool((R[r:] != 0).any()), f"instance {i}: rows past the rank"
        assert bool((R[torch.arange(r, device=dev), piv[:r].long()] == 1).all()), f"instance {i}"
        if i in keep:
            Rh = R.cpu().numpy().astype(np.uint32)
            A = keep[i]
            print(f"instance {i}: certificates", flush=True)
            assert certs.is_rref_form(Rh, r, pv), f"instance {i}: not an RREF"
            assert certs.freivalds_rank_factorisation(A, Rh, r, pv, P), f"instance {i}: A != C R"
            R1, r1, p1 = lx.rref(A, P)
            torch.cuda.synchronize()
            assert int(r1.item()) == r and np.array_equal(R1.cpu().numpy().astype(np.uint32), Rh)
            if i == 21:
                print("instance 21: C oracle at full size", flush=True)
                Ro, ro, po = oracle.rref(A, P)
                assert ro == r and np.array_equal(po, pv) and np.array_equal(Ro, Rh)
                print("instance 21: oracle agrees", flush=True)
