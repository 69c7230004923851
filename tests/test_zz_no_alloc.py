"""linac_solve_noalloc (the solve for callers that cannot allocate) against
linac_solve, through the C ABI, bit for bit.

Two calls in a row on one GPU share the library's fixed scratch array; the
second takes a smaller system, so anything it reads that the first call left
behind and it did not initialise would show up as a difference.  Both the
plain path and the blocked int8 path (which the no-alloc call runs without its
look-ahead side stream) are covered, plus the host-side refusals: a system
whose workspace exceeds the array, and opts->validate.
"""

from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
import workloads
import paper_2605_25863_amd as lx

pytestmark = pytest.mark.gpu


def _outputs(torch, dev, m, n, k):
    return (torch.full((n, k), -7, dtype=torch.int32, device=dev),
            torch.full((1,), -7, dtype=torch.int32, device=dev),
            torch.full((max(min(m, n), 1),), -7, dtype=torch.int32, device=dev),
            torch.full((max(k, 1),), 9, dtype=torch.uint8, device=dev))


def _host(torch, outs, n, k):
    X, rank, piv, cons = outs
    torch.cuda.synchronize()
    return (X.cpu().numpy(), int(rank.item()), piv.cpu().numpy(), cons.cpu().numpy()[:k])


def _run_pair(A, B, p, path, panel):
    import torch
    dev = torch.device("cuda", 0)
    At = torch.from_numpy(A.astype(np.int32)).to(dev)
    Bt = torch.from_numpy(B.astype(np.int32)).to(dev)
    m, n = A.shape
    k = B.shape[1]
    ref_outs = _outputs(torch, dev, m, n, k)
    lx.solve(At, Bt, p, path=path, panel_width=panel, out=ref_outs)
    got_outs = _outputs(torch, dev, m, n, k)
    lx.solve_noalloc(At, Bt, p, path=path, panel_width=panel, out=got_outs)
    ref = _host(torch, ref_outs, n, k)
    got = _host(torch, got_outs, n, k)
    for name, g, r in zip(("X", "rank", "pivots", "consistent"), got, ref):
        assert np.array_equal(np.asarray(g), np.asarray(r)), f"{name} differs"
    return got


@pytest.mark.parametrize("path,panel,sizes", [
    (lx.PATH_PLAIN, 0, [(700, 5), (300, 2)]),
    (lx.PATH_BLOCKED_INT8, 128, [(1500, 8), (520, 3)]),
    (lx.PATH_AUTO, 0, [(2600, 16), (257, 1)]),
])
def test_noalloc_matches_solve_two_calls(gpu, path, panel, sizes):
    for call, (n, k) in enumerate(sizes):
        A, B, p = workloads.dense_system(seed=500 + n, n=n, k=k)
        A[n // 2] = A[1]  # rank deficient: a free column and an inconsistent right-hand side
        print(f"noalloc call {call}: path={path} panel={panel} n={n} k={k}", flush=True)
        X, r, piv, cons = _run_pair(A, B, p, path, panel)
        assert r == n - 1
        if n <= 700:  # small enough for the oracle
            Xo, ro, po, co = oracle.solve(A, B, p)
            assert np.array_equal(X, Xo.astype(np.int32)) and np.array_equal(cons, co)


def test_noalloc_fp64_and_rectangular(gpu):
    rng = np.random.default_rng(5)
    p = 1048573
    for m, n, k in [(400, 300, 4), (90, 260, 2)]:
        A = workloads.uniform(rng, (m, n), p)
        B = workloads.uniform(rng, (m, k), p)
        print(f"noalloc fp64 {m}x{n} k={k}", flush=True)
        _run_pair(A, B, p, lx.PATH_BLOCKED_FP64, 64)


def test_noalloc_host_refusals(gpu):
    lib = lx._load()
    fake = ctypes.c_void_p(0x1000)
    # 8192 x 8192 needs about 270 MB of workspace: more than the array
    st = lib.linac_solve_noalloc(fake, 8192, 8192, 8192, fake, 1, 1, 7, fake, 1, fake, fake, fake,
                                 None, None)
    assert st == 5  # LINAC_E_WORKSPACE
    o = lx._opts(validate=True)
    st = lib.linac_solve_noalloc(fake, 8, 8, 8, fake, 1, 1, 7, fake, 1, fake, fake, fake,
                                 ctypes.byref(o), None)
    assert st == 2  # LINAC_E_UNSUPPORTED
