"""The C-ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before any device work (runs without a GPU: every call
here returns from the host-side checks)."""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2605_25863_amd as lx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "linac.h")

OK, INVALID, UNSUP, NOTPRIME, RANGE, WS, NOMEM, HIP = range(8)


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:linac_status|const char\*|int)\s+(linac_\w+)\s*\(",
                                 text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lx.library_path()):
        pytest.fail("library not built: run __graft_entry__.build() first")
    return lx._load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_strings(lib):
    assert lib.linac_version() >= 100
    for st in range(8):
        assert lib.linac_status_string(st)


def test_check_prime_matches_trial_division(lib):
    limit = 1 << 18
    sieve = np.ones(limit, dtype=bool)
    sieve[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = False
    for v in range(1, limit):
        want = OK if sieve[v] else NOTPRIME
        assert lib.linac_check_prime(v) == want, v
    # strong pseudoprimes to base 2 and Carmichael numbers are composite
    for v in (2047, 3277, 4033, 4681, 8321, 561, 1105, 1729, 2465, 25326001, 46337 * 46327):
        assert lib.linac_check_prime(v) == NOTPRIME, v
    assert lib.linac_check_prime(3215031751) == UNSUP  # spsp(2,3,5,7), above 2^31
    # random 31-bit values against trial division
    rng = np.random.default_rng(0)
    for v in rng.integers(1 << 30, 1 << 31, size=300):
        v = int(v)
        prime = all(v % d for d in range(2, int(v ** 0.5) + 1))
        assert lib.linac_check_prime(v) == (OK if prime else NOTPRIME), v
    assert lib.linac_check_prime((1 << 31) - 1) == OK
    assert lib.linac_check_prime(2147483629) == OK
    assert lib.linac_check_prime(0) == UNSUP
    assert lib.linac_check_prime(1 << 31) == UNSUP
    assert lib.linac_check_prime(0xFFFFFFFB) == UNSUP  # prime, but above 2^31


def _fake(n=1):
    # non-null addresses that the host checks never dereference
    return ctypes.c_void_p(0x1000 * n)


def _solve(lib, m=4, n=4, k=1, lda=4, ldb=1, ldx=1, p=7, ws_bytes=1 << 30, ws=True, A=True,
           X=True, rank=True, cons=True, piv=True):
    return lib.linac_solve(_fake(1) if A else None, m, n, lda, _fake(2), k, ldb, p,
                           _fake(3) if X else None, ldx, _fake(4) if rank else None,
                           _fake(5) if piv else None, _fake(6) if cons else None,
                           _fake(7) if ws else None, ws_bytes, None, None)


def test_solve_argument_errors(lib):
    assert _solve(lib, m=-1) == INVALID
    assert _solve(lib, lda=3) == INVALID
    assert _solve(lib, k=2, ldb=1) == INVALID
    assert _solve(lib, k=2, ldb=2, ldx=1) == INVALID
    assert _solve(lib, A=False) == INVALID
    assert _solve(lib, X=False) == INVALID
    assert _solve(lib, rank=False) == INVALID
    assert _solve(lib, cons=False) == INVALID
    assert _solve(lib, piv=False) == INVALID
    assert _solve(lib, p=0) == UNSUP
    assert _solve(lib, p=(1 << 31) + 11) == UNSUP
    assert _solve(lib, p=9) == NOTPRIME
    assert _solve(lib, p=561) == NOTPRIME
    assert _solve(lib, ws=False) == WS
    assert _solve(lib, ws_bytes=16) == WS
    assert _solve(lib, m=1 << 31) == NOMEM


def test_rref_argument_errors(lib):
    f = _fake
    assert lib.linac_rref(f(1), -1, 3, 3, 7, f(2), f(3), f(4), 1 << 20, None, None) == INVALID
    assert lib.linac_rref(f(1), 3, 3, 2, 7, f(2), f(3), f(4), 1 << 20, None, None) == INVALID
    assert lib.linac_rref(None, 3, 3, 3, 7, f(2), f(3), f(4), 1 << 20, None, None) == INVALID
    assert lib.linac_rref(f(1), 3, 3, 3, 7, None, f(3), f(4), 1 << 20, None, None) == INVALID
    assert lib.linac_rref(f(1), 3, 3, 3, 15, f(2), f(3), f(4), 1 << 20, None, None) == NOTPRIME
    assert lib.linac_rref(f(1), 3, 3, 3, 7, f(2), f(3), f(4), 8, None, None) == WS


def test_workspace_queries(lib):
    sz = ctypes.c_size_t()
    assert lib.linac_solve_workspace(8192, 8192, 16, None, ctypes.byref(sz)) == OK
    ld = (8192 + 16 + 63) // 64 * 64
    assert sz.value >= 8192 * ld * 4
    assert lib.linac_solve_workspace(-1, 3, 3, None, ctypes.byref(sz)) == INVALID
    assert lib.linac_rref_workspace(0, 0, None, ctypes.byref(sz)) == OK
    assert lib.linac_rref_workspace(5, 5, None, None) == INVALID


def test_binding_fails_loudly_without_gpu():
    """No CPU fallback: without a visible GPU the binding raises."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        lx.solve(np.eye(3, dtype=np.uint32), np.ones((3, 1), dtype=np.uint32), 7)


def test_tuning_table_parsing(lib):
    """linac_load_tuning: valid tables change the panel choice (seen through the
    workspace size), malformed ones are rejected and leave the table alone."""
    import json
    sz_default, sz = ctypes.c_size_t(), ctypes.c_size_t()
    opts = lx._opts(lx.PATH_BLOCKED_INT8)
    assert lib.linac_load_tuning(None) == OK
    assert lib.linac_solve_workspace(4096, 4096, 16, ctypes.byref(opts), ctypes.byref(sz_default)) == OK
    table = {"blocked_min": 2048, "panel": [{"n_max": 1024, "panel": 64},
                                            {"n_max": 1 << 30, "panel": 512}],
             "batched_per_cu": 2, "arch": "gfx950", "measured": {"x": [1, 2.5, None, True]}}
    assert lib.linac_load_tuning(json.dumps(table).encode()) == OK
    assert lib.linac_solve_workspace(4096, 4096, 16, ctypes.byref(opts), ctypes.byref(sz)) == OK
    assert sz.value > sz_default.value  # panel 512 needs larger panel buffers than 256
    # AUTO below the crossover is the plain path (smallest workspace)
    auto = lx._opts(lx.PATH_AUTO)
    plain = lx._opts(lx.PATH_PLAIN)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    lib.linac_solve_workspace(1500, 1500, 4, ctypes.byref(auto), ctypes.byref(a))
    lib.linac_solve_workspace(1500, 1500, 4, ctypes.byref(plain), ctypes.byref(b))
    assert a.value == b.value
    for bad in (b"{", b"[1,2", b'{"panel": [{"n_max": 10, "panel": 33}]}',
                b'{"batched_per_cu": 0}', b'{"lookahead": 2}', b"{} trailing"):
        assert lib.linac_load_tuning(bad) == INVALID
    # the previous valid table is still in force
    assert lib.linac_solve_workspace(4096, 4096, 16, ctypes.byref(opts), ctypes.byref(a)) == OK
    assert a.value == sz.value
    assert lib.linac_load_tuning(None) == OK
    lx.restore_tuning()


def test_plan(lib):
    """linac_plan reports the path AUTO takes and the panel width, from the
    caller's options and the tuning table, and rejects what the calls reject."""
    import json
    table = {"blocked_min": 2048, "panel": [{"n_max": 1024, "panel": 64},
                                            {"n_max": 1 << 30, "panel": 384}]}
    path, panel = ctypes.c_int(), ctypes.c_int()

    def plan(m, n, opts=None):
        st = lib.linac_plan(m, n, ctypes.byref(opts) if opts else None, ctypes.byref(path),
                            ctypes.byref(panel))
        return st, path.value, panel.value

    assert lib.linac_load_tuning(json.dumps(table).encode()) == OK
    try:
        assert plan(1500, 1500) == (OK, lx.PATH_PLAIN, 0)
        assert plan(4096, 5000) == (OK, lx.PATH_BLOCKED_INT8, 384)
        assert plan(5000, 2048) == (OK, lx.PATH_BLOCKED_INT8, 384)
        assert plan(800, 900, lx._opts(lx.PATH_BLOCKED_INT8)) == (OK, lx.PATH_BLOCKED_INT8, 64)
        assert plan(800, 900, lx._opts(lx.PATH_BLOCKED_FP64, 96)) == (OK, lx.PATH_BLOCKED_FP64, 96)
        assert plan(9000, 9000, lx._opts(lx.PATH_PLAIN, 96)) == (OK, lx.PATH_PLAIN, 0)
        assert plan(0, 0) == (OK, lx.PATH_PLAIN, 0)
        assert plan(800, 900, lx._opts(lx.PATH_BLOCKED_INT8, 100))[0] == INVALID
        assert plan(800, 900, lx._opts(lx.PATH_BLOCKED_INT8, 544))[0] == INVALID
        assert plan(-1, 5)[0] == INVALID
        assert lib.linac_plan(5, 5, None, None, ctypes.byref(panel)) == INVALID
        assert lib.linac_plan(5, 5, None, ctypes.byref(path), None) == INVALID
        assert plan(5, 5, lx._opts(7))[0] == UNSUP
    finally:
        lx.restore_tuning()


def test_load_matrix_argument_errors(lib):
    f = _fake
    lm = lib.linac_load_matrix
    # (bases, nrows, nbasis, ldbases, lindices, ncols, d, ldl, p, A, lda, stream)
    assert lm(f(1), -1, 4, 4, f(2), 5, 2, 2, 7, f(3), 5, None) == INVALID
    assert lm(f(1), 3, 4, 3, f(2), 5, 2, 2, 7, f(3), 5, None) == INVALID  # ldbases < nbasis
    assert lm(f(1), 3, 4, 4, f(2), 5, 2, 1, 7, f(3), 5, None) == INVALID  # ldl < d
    assert lm(f(1), 3, 4, 4, f(2), 5, 2, 2, 7, f(3), 4, None) == INVALID  # lda < ncols
    assert lm(None, 3, 4, 4, f(2), 5, 2, 2, 7, f(3), 5, None) == INVALID
    assert lm(f(1), 3, 4, 4, None, 5, 2, 2, 7, f(3), 5, None) == INVALID
    assert lm(f(1), 3, 4, 4, f(2), 5, 2, 2, 7, None, 5, None) == INVALID
    assert lm(f(1), 3, 4, 4, f(2), 5, -1, 1, 7, f(3), 5, None) == INVALID
    assert lm(f(1), 3, 4, 4, f(2), 5, 2, 2, 15, f(3), 5, None) == NOTPRIME
    assert lm(f(1), 3, 4, 4, f(2), 5, 2, 2, 0, f(3), 5, None) == UNSUP
    assert lm(f(1), 1 << 31, 4, 4, f(2), 5, 2, 2, 7, f(3), 5, None) == NOMEM
    # empty shapes need no pointers and launch nothing
    assert lm(None, 0, 4, 4, None, 0, 2, 2, 7, None, 1, None) == OK
    assert lm(None, 0, 0, 1, f(2), 5, 2, 2, 7, None, 5, None) == OK


def test_nullspace_and_column_basis_argument_errors(lib):
    f = _fake
    ns = lib.linac_nullspace
    # (R, m, n, ldr, rank, pivots, p, K, kcols, ldk, free_cols, stream)
    assert ns(f(1), 3, 4, 4, f(2), f(3), 7, f(4), 5, 5, None, None) == INVALID  # kcols > n
    assert ns(f(1), 3, 4, 3, f(2), f(3), 7, f(4), 4, 4, None, None) == INVALID  # ldr < n
    assert ns(f(1), 3, 4, 4, f(2), f(3), 7, f(4), 4, 3, None, None) == INVALID  # ldk < kcols
    assert ns(f(1), 3, 4, 4, None, f(3), 7, f(4), 4, 4, None, None) == INVALID
    assert ns(None, 3, 4, 4, f(2), f(3), 7, f(4), 4, 4, None, None) == INVALID
    assert ns(f(1), 3, 4, 4, f(2), None, 7, f(4), 4, 4, None, None) == INVALID
    assert ns(f(1), 3, 4, 4, f(2), f(3), 7, None, 4, 4, None, None) == INVALID
    assert ns(f(1), 3, 4, 4, f(2), f(3), 9, f(4), 4, 4, None, None) == NOTPRIME
    assert ns(None, 0, 0, 1, f(2), None, 7, None, 0, 1, None, None) == OK
    cb = lib.linac_column_basis
    # (A, m, n, lda, rank, pivots, C, ccols, ldc, stream)
    assert cb(f(1), 3, 4, 4, f(2), f(3), f(4), 4, 4, None) == INVALID  # ccols > min(m, n)
    assert cb(f(1), 3, 4, 3, f(2), f(3), f(4), 3, 3, None) == INVALID  # lda < n
    assert cb(f(1), 3, 4, 4, f(2), f(3), f(4), 3, 2, None) == INVALID  # ldc < ccols
    assert cb(f(1), 3, 4, 4, None, f(3), f(4), 3, 3, None) == INVALID
    assert cb(None, 3, 4, 4, f(2), f(3), f(4), 3, 3, None) == INVALID
    assert cb(f(1), 3, 4, 4, f(2), f(3), None, 3, 3, None) == INVALID
    assert cb(None, 0, 4, 4, f(2), None, None, 0, 1, None) == OK


def test_u64_and_lup_host_checks(lib):
    f = _fake
    OKP = 9223372036854775783  # 2^63 - 25
    assert lib.linac_check_prime_u64(OKP) == OK
    assert lib.linac_check_prime_u64(4611686018427387847) == OK
    assert lib.linac_check_prime_u64(4294967311) == OK
    assert lib.linac_check_prime_u64(2) == OK
    assert lib.linac_check_prime_u64(1 << 63) == UNSUP
    assert lib.linac_check_prime_u64((1 << 64) - 59) == UNSUP  # prime, but above 2^63
    assert lib.linac_check_prime_u64(0) == UNSUP
    assert lib.linac_check_prime_u64(3215031751) == NOTPRIME  # spsp(2,3,5,7)
    assert lib.linac_check_prime_u64(3825123056546413051) == NOTPRIME  # spsp to bases 2..23
    assert lib.linac_check_prime_u64(4294967297) == NOTPRIME  # 641 * 6700417
    for v in range(1, 2000):
        prime = v > 1 and all(v % q for q in range(2, int(v ** 0.5) + 1))
        assert lib.linac_check_prime_u64(v) == (OK if prime else (UNSUP if v == 0 else NOTPRIME)), v
    ws = ctypes.c_size_t()
    assert lib.linac_rref_u64_workspace(100, 50, ctypes.byref(ws)) == OK and ws.value > 100 * 50 * 8
    assert lib.linac_lup_workspace(100, 50, 0, ctypes.byref(ws)) == OK
    # (A, m, n, lda, p, rank, pivots, ws, ws_bytes, opts, stream)
    ru = lib.linac_rref_u64
    assert ru(f(1), 3, 4, 3, OKP, f(2), f(3), f(4), 1 << 20, None, None) == INVALID
    assert ru(f(1), 3, 4, 4, OKP, None, f(3), f(4), 1 << 20, None, None) == INVALID
    assert ru(f(1), 3, 4, 4, 1 << 63, f(2), f(3), f(4), 1 << 20, None, None) == UNSUP
    assert ru(f(1), 3, 4, 4, OKP - 2, f(2), f(3), f(4), 1 << 20, None, None) == NOTPRIME
    assert ru(f(1), 3, 4, 4, OKP, f(2), f(3), f(4), 16, None, None) == WS
    su = lib.linac_solve_u64
    assert su(f(1), 3, 4, 4, f(2), 2, 1, OKP, f(3), 2, f(4), f(5), f(6), f(7), 1 << 20, None,
              None) == INVALID
    assert su(f(1), 3, 4, 4, f(2), 2, 2, OKP, f(3), 2, f(4), f(5), None, f(7), 1 << 20, None,
              None) == INVALID
    lu = lib.linac_lup
    # (A, m, n, lda, p, perm, rank, pivots, ws, ws_bytes, opts, stream)
    assert lu(f(1), 3, 4, 4, 7, None, f(2), f(3), f(4), 1 << 20, None, None) == INVALID
    assert lu(f(1), 3, 4, 4, (1 << 31) + 11, f(5), f(2), f(3), f(4), 1 << 20, None, None) == UNSUP
    assert lib.linac_lup_u64(f(1), 3, 4, 4, 9, f(5), f(2), f(3), f(4), 1 << 20, None,
                             None) == NOTPRIME
