"""Test oracle for exact Gaussian elimination over F_p -- NOT part of the product.

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the library and its Python binding
never do.  It shares no code with the GPU path.

What it computes is the plain definition of the method's outputs (the paper,
Sec. 3.2 and Sec. 5.1-5.2): for A (m x n), B (m x k) and a prime p,

* R = RREF(A) over F_p in the original shape, zero rows at the bottom
  (Sec. 2.3, Basic Usage);
* the rank r and the ascending pivot columns J (Sec. 5.1);
* for each right-hand side t: consistent[t] iff rank(A) = rank([A | b_t]),
  and X[:, t] the particular solution whose free (non-pivot) variables are
  zero, or zero when inconsistent (Sec. 5.2).

Three independent implementations of one textbook Gauss-Jordan algorithm:
``c`` (oracle/gj.c: uint64 and ``%``, OpenMP over rows), ``numpy`` (int64,
vectorised row update; f*x < 2^62 is exact) and ``python`` (Python ints, for
tiny sizes and brute force).  The numpy and python versions also accept a
``pivot_rule`` ("first", "last", "random") to show the outputs do not depend
on which non-zero entry is chosen (Sec. 3.2, "Pivoting").

Readings where the paper is silent: pivots are searched only in A's columns;
several right-hand sides are carried as extra columns of the augmented
matrix; entries must already be canonical residues in [0, p).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gj.c")
_LIB = os.path.join(_HERE, "liboracle_gj.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle/gj.c with gcc (-O2, OpenMP) into oracle/liboracle_gj.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_gauss_jordan.restype = ctypes.c_int64
        lib.oracle_gauss_jordan.argtypes = [u64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_uint64, i64p, u64p, ctypes.c_int]
        lib.oracle_gauss_jordan_many.restype = None
        lib.oracle_gauss_jordan_many.argtypes = [u64p, i64p, i64p, i64p, i64p, u64p, i64p, i64p,
                                                 i64p, ctypes.c_int64, ctypes.c_int]
        lib.oracle_inv.restype = ctypes.c_uint64
        lib.oracle_inv.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_powmod.restype = ctypes.c_uint64
        lib.oracle_powmod.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_gauss_jordan_wide.restype = ctypes.c_int64
        lib.oracle_gauss_jordan_wide.argtypes = [u64p, ctypes.c_int64, ctypes.c_int64,
                                                 ctypes.c_int64, ctypes.c_uint64, i64p, ctypes.c_int]
        lib.oracle_lup.restype = ctypes.c_int64
        lib.oracle_lup.argtypes = [u64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, i64p, i64p,
                                   i64p, ctypes.c_int]
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def inv(a: int, p: int) -> int:
    """Extended-Euclid inverse of a mod p (0 when a is not invertible)."""
    return int(_load().oracle_inv(int(a), int(p)))


def powmod(a: int, e: int, p: int) -> int:
    return int(_load().oracle_powmod(int(a), int(e), int(p)))


# ---------------------------------------------------------------------------
# Gauss-Jordan in three independent implementations
# ---------------------------------------------------------------------------

def _gj_c(M: np.ndarray, nsearch: int, p: int, threads: int = 0, want_det: bool = False):
    M = np.ascontiguousarray(M, dtype=np.uint64).copy()
    m, ncols = M.shape
    piv = np.zeros(max(min(m, nsearch), 1), dtype=np.int64)
    det = ctypes.c_uint64(0)
    lib = _load()
    r = lib.oracle_gauss_jordan(M.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), m, ncols,
                                nsearch, p, piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                ctypes.byref(det) if want_det else None, int(threads))
    return M, int(r), piv[: int(r)].copy(), int(det.value)


def _gj_c_wide(M: np.ndarray, nsearch: int, p: int, threads: int = 0, want_det: bool = False):
    """oracle/gj.c's Gauss-Jordan with 128-bit products (primes up to 2^63)."""
    if want_det:
        raise ValueError("the wide C oracle does not track the determinant")
    M = np.ascontiguousarray(M, dtype=np.uint64).copy()
    m, ncols = M.shape
    piv = np.zeros(max(min(m, nsearch), 1), dtype=np.int64)
    r = _load().oracle_gauss_jordan_wide(M.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), m,
                                         ncols, nsearch, p,
                                         piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                         int(threads))
    return M, int(r), piv[: int(r)].copy(), 0


def _choose(rows_nonzero, rule, rng):
    if rule == "first":
        return rows_nonzero[0]
    if rule == "last":
        return rows_nonzero[-1]
    return rows_nonzero[int(rng.integers(0, len(rows_nonzero)))]


def _gj_numpy(M: np.ndarray, nsearch: int, p: int, pivot_rule: str = "first", seed: int = 0,
              want_det: bool = False):
    """int64 Gauss-Jordan: the row update is vectorised, nothing else."""
    if p >= 1 << 31:
        raise ValueError("the numpy oracle needs p < 2^31 (products must fit int64)")
    M = np.array(M, dtype=np.int64)
    m, ncols = M.shape
    rng = np.random.default_rng(seed)
    i = 0
    piv = []
    det, singular = 1 % p, False
    for j in range(nsearch):
        if i == m:
            singular = True
            break
        nz = np.nonzero(M[i:, j])[0]
        if len(nz) == 0:
            singular = True
            continue
        r = i + int(_choose(nz, pivot_rule, rng))
        if r != i:
            M[[i, r]] = M[[r, i]]
            det = (p - det) % p
        head = int(M[i, j])
        det = det * head % p
        M[i] = M[i] * pow(head, -1, p) % p
        f = M[:, j].copy()
        f[i] = 0
        rows = np.nonzero(f)[0]
        if len(rows):
            M[rows] = (M[rows] - (f[rows, None] * M[i][None, :]) % p) % p
        piv.append(j)
        i += 1
    return M.astype(np.uint64), i, np.array(piv, dtype=np.int64), (0 if singular else det)


def _gj_python(M, nsearch: int, p: int, pivot_rule: str = "first", seed: int = 0,
               want_det: bool = False):
    """Python-int Gauss-Jordan on lists: the plainest possible statement."""
    shape = np.asarray(M).shape
    M = [[int(x) for x in row] for row in np.asarray(M).tolist()]
    m, ncols = shape
    rng = np.random.default_rng(seed)
    i = 0
    piv = []
    det, singular = 1 % p, False
    for j in range(nsearch):
        if i == m:
            singular = True
            break
        nz = [q - i for q in range(i, m) if M[q][j] % p != 0]
        if not nz:
            singular = True
            continue
        r = i + _choose(nz, pivot_rule, rng)
        if r != i:
            M[i], M[r] = M[r], M[i]
            det = (-det) % p
        head = M[i][j]
        det = det * head % p
        hinv = pow(head, p - 2, p)  # Fermat: head^(p-2) = head^-1 in F_p
        M[i] = [x * hinv % p for x in M[i]]
        for q in range(m):
            if q != i and M[q][j] != 0:
                f = M[q][j]
                M[q] = [(a - f * b) % p for a, b in zip(M[q], M[i])]
        piv.append(j)
        i += 1
    arr = np.array(M, dtype=np.uint64).reshape(m, ncols)
    return arr, i, np.array(piv, dtype=np.int64), (0 if singular else det)


_IMPLS = {"c": _gj_c, "c_wide": _gj_c_wide, "numpy": _gj_numpy, "python": _gj_python}


def gauss_jordan(M, nsearch: int, p: int, impl: str = "c", **kw):
    """RREF of M over F_p with pivots searched in columns [0, nsearch).

    Returns (reduced matrix as uint64, rank, pivot columns, det).  ``det`` is
    meaningful only for a square searched block and when asked for.
    """
    M = np.asarray(M)
    if M.ndim != 2:
        raise ValueError("matrix must be 2-D")
    if M.size and int(M.max()) >= p:
        raise ValueError("entries must be canonical residues in [0, p)")
    if impl == "c" and p >= 1 << 32:
        impl = "c_wide"  # products of residues above 2^32 need 128 bits
    if impl in ("c", "c_wide"):
        kw.pop("pivot_rule", None)
        kw.pop("seed", None)
    return _IMPLS[impl](M, nsearch, int(p), **kw)


def _word(p: int):
    """Storage of residues: uint32 below 2^32, uint64 above (Sec. 3.2)."""
    return np.uint32 if p < 1 << 32 else np.uint64


def rref(A, p: int, impl: str = "c", **kw):
    """(R, rank, pivots): R in A's shape (uint32, or uint64 for p >= 2^32),
    zero rows at the bottom."""
    A = np.asarray(A)
    R, r, piv, _ = gauss_jordan(A, A.shape[1], p, impl, **kw)
    return R.astype(_word(p)), r, piv


def solve(A, B, p: int, impl: str = "c", **kw):
    """(X, rank, pivots, consistent) for A X = B over F_p (Sec. 5.2).

    The augmented matrix [A | B] is reduced with pivots only in A's columns.
    Column t is consistent iff every row at or below the rank is zero in
    B's part, which is rank(A) = rank([A | b_t]).  X takes the reduced B rows
    on the pivot variables and zero on the free ones; an inconsistent column
    of X is all zero.
    """
    A = np.asarray(A)
    B = np.asarray(B)
    m, n = A.shape
    k = B.shape[1]
    M = np.concatenate([A.astype(np.uint64), B.astype(np.uint64)], axis=1)
    R, r, piv, _ = gauss_jordan(M, n, p, impl, **kw)
    consistent = np.array([not np.any(R[r:, n + t]) for t in range(k)], dtype=np.uint8)
    X = np.zeros((n, k), dtype=np.uint64)
    for s, c in enumerate(piv):
        X[c, :] = R[s, n:]
    X[:, consistent == 0] = 0
    return X.astype(_word(p)), r, piv, consistent


def det(A, p: int, impl: str = "c", **kw) -> int:
    """Determinant of a square A over F_p (heads before scaling, sign of swaps)."""
    A = np.asarray(A)
    assert A.shape[0] == A.shape[1]
    return gauss_jordan(A, A.shape[1], p, impl, want_det=True, **kw)[3]


def solve_many(systems, threads: int = 0):
    """Oracle solves of many independent systems, one thread per system.

    ``systems`` is a list of dicts {A, B, p}.  Returns a list of
    (X, rank, pivots, consistent) in order.
    """
    lib = _load()
    mats, offs, rows, cols, ns, ps, pivoffs = [], [], [], [], [], [], []
    off = poff = 0
    for s in systems:
        A, B = np.asarray(s["A"]), np.asarray(s["B"])
        M = np.concatenate([A.astype(np.uint64), B.astype(np.uint64)], axis=1)
        mats.append(M.ravel())
        offs.append(off)
        rows.append(M.shape[0])
        cols.append(M.shape[1])
        ns.append(A.shape[1])
        ps.append(int(s["p"]))
        pivoffs.append(poff)
        off += M.size
        poff += max(min(A.shape), 1)
    buf = np.concatenate(mats) if mats else np.zeros(0, np.uint64)
    i64 = lambda v: np.array(v, dtype=np.int64)
    offs_a, rows_a, cols_a, ns_a, poffs_a = map(i64, (offs, rows, cols, ns, pivoffs))
    ps_a = np.array(ps, dtype=np.uint64)
    ranks = np.zeros(len(systems), dtype=np.int64)
    pivs = np.zeros(max(poff, 1), dtype=np.int64)
    P64 = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_gauss_jordan_many(buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 offs_a.ctypes.data_as(P64), rows_a.ctypes.data_as(P64),
                                 cols_a.ctypes.data_as(P64), ns_a.ctypes.data_as(P64),
                                 ps_a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 ranks.ctypes.data_as(P64), pivs.ctypes.data_as(P64),
                                 poffs_a.ctypes.data_as(P64), len(systems), int(threads))
    out = []
    for i, s in enumerate(systems):
        m, ncols, n = rows[i], cols[i], ns[i]
        R = buf[offs[i]: offs[i] + m * ncols].reshape(m, ncols)
        r = int(ranks[i])
        piv = pivs[pivoffs[i]: pivoffs[i] + r].copy()
        k = ncols - n
        consistent = np.array([not np.any(R[r:, n + t]) for t in range(k)], dtype=np.uint8)
        X = np.zeros((n, k), dtype=np.uint64)
        for srow, c in enumerate(piv):
            X[c, :] = R[srow, n:]
        X[:, consistent == 0] = 0
        out.append((X.astype(np.uint32), r, piv, consistent))
    return out


# ---------------------------------------------------------------------------
# Applications of the RREF (Sec. 5.1): used by the tests as certificates
# ---------------------------------------------------------------------------

def drop_bottom_zero_rows(R):
    """R without its trailing all-zero rows."""
    R = np.asarray(R)
    keep = R.shape[0]
    while keep and not np.any(R[keep - 1]):
        keep -= 1
    return R[:keep]


def canonical_kernel(R, pivots, n: int, p: int):
    """Null-space basis K (n x (n-r)) of the RREF R: free variables take -I.

    Column f of K corresponds to the f-th non-pivot column c: K[c, f] = -1 and
    K[pivots[s], f] = R[s, c], so that R K = 0 (Sec. 5.1).
    """
    R = np.asarray(R).astype(np.int64)
    piv = list(int(c) for c in pivots)
    free = [c for c in range(n) if c not in set(piv)]
    K = np.zeros((n, len(free)), dtype=np.int64)
    for f, c in enumerate(free):
        K[c, f] = p - 1
        for s, pc in enumerate(piv):
            K[pc, f] = R[s, c] % p
    return K.astype(np.uint64)


def matmul_mod(A, B, p: int) -> np.ndarray:
    """(A @ B) mod p exactly, for residues below 2^31 (16-bit split of B)."""
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    lo = B & 0xFFFF
    hi = B >> 16
    out = np.zeros((A.shape[0], B.shape[1]), dtype=np.int64)
    # each partial sum of at most 2^15 products below 2^47 stays below 2^62
    step = 1 << 14
    for k0 in range(0, A.shape[1], step):
        a = A[:, k0:k0 + step]
        out = (out + (a @ lo[k0:k0 + step]) % p) % p
        out = (out + ((a @ hi[k0:k0 + step]) % p) * (1 << 16) % p) % p
    return out.astype(np.uint64)


def rank_factor_columns(A, pivots):
    """C = A[:, J]: the columns of A at the pivot columns J of its RREF, so that
    A = C R with R the non-zero rows of the RREF (Sec. 5.1)."""
    A = np.asarray(A)
    return A[:, np.asarray(pivots, dtype=np.int64)].copy()


# ---------------------------------------------------------------------------
# Construction of a linear system from monomials (Sec. 3.3)
# ---------------------------------------------------------------------------

def load_matrix(bases, lindices, p: int, impl: str = "numpy"):
    """A[r, c] = prod_t bases[r, lindices[c, t]] mod p (Sec. 3.3, the matrix
    of a monomial ansatz evaluated at sampling points; Sec. 2.3 for the
    bases / lindices layout).

    bases: (nrows, nbasis) residues, one row per sampling point; lindices:
    (ncols, d) integer indices into a row of bases, one row per monomial.
    The empty product (d = 0) is 1.  An index outside [0, nbasis) is not
    defined by the paper; it is read here as a factor 0.

    ``numpy``: a running product reduced after every factor (int64; the
    product of two residues below 2^31 is below 2^62).  ``python``: Python
    ints, the product taken whole and reduced once (tiny sizes).
    """
    B = np.asarray(bases)
    L = np.asarray(lindices)
    if B.ndim != 2 or L.ndim != 2:
        raise ValueError("bases and lindices must be 2-D")
    if B.size and int(B.max()) >= p:
        raise ValueError("bases must be canonical residues in [0, p)")
    nrows, nb = B.shape
    ncols, d = L.shape
    if impl == "python":
        Bl = [[int(x) for x in row] for row in B.tolist()]
        Ll = [[int(x) for x in row] for row in L.tolist()]
        out = np.zeros((nrows, ncols), dtype=np.uint32)
        for r in range(nrows):
            for c in range(ncols):
                prod = 1
                for t in range(d):
                    i = Ll[c][t]
                    prod *= Bl[r][i] if 0 <= i < nb else 0
                out[r, c] = prod % p
        return out
    B = B.astype(np.int64)
    L = L.astype(np.int64)
    A = np.full((nrows, ncols), 1 % p, dtype=np.int64)
    for t in range(d):
        idx = L[:, t]
        ok = (idx >= 0) & (idx < nb)
        F = np.zeros((nrows, ncols), dtype=np.int64)
        F[:, ok] = B[:, idx[ok]]
        A = A * F % p
    return A.astype(np.uint32)



# ---------------------------------------------------------------------------
# LUP factorisation (the paper's future work, Sec. 6)
# ---------------------------------------------------------------------------

def lup(A, p: int, impl: str = "c"):
    """P A = L U over F_p by forward elimination with a fixed pivot rule.

    For each column j in turn the pivot is the first row, in the original row
    order, that is not a pivot yet and has a non-zero entry in column j;
    every other non-pivot row q takes g = A[q][j] / head, is replaced by
    row_q - g * (pivot row), and keeps g in column j.  Returns (LU, perm,
    rank, pivots): perm lists the pivot rows in pivot order, then the other
    rows in their original order, and LU = the worked matrix in that row
    order (L's entries at the pivot columns left of each row's own pivot,
    U's entries elsewhere; see ``lup_factors``).

    ``c``: oracle/gj.c (128-bit products); ``python``: Python ints.
    """
    A = np.asarray(A)
    m, n = A.shape
    if A.size and int(A.max()) >= p:
        raise ValueError("entries must be canonical residues in [0, p)")
    if impl == "c":
        M = np.ascontiguousarray(A, dtype=np.uint64).copy()
        step = np.zeros(max(m, 1), dtype=np.int64)
        prow = np.zeros(max(min(m, n), 1), dtype=np.int64)
        pcol = np.zeros(max(min(m, n), 1), dtype=np.int64)
        P64 = ctypes.POINTER(ctypes.c_int64)
        r = int(_load().oracle_lup(M.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), m, n, p,
                                   step.ctypes.data_as(P64), prow.ctypes.data_as(P64),
                                   pcol.ctypes.data_as(P64), 0))
        is_piv = step[:m] >= 0
        pivrows, pivots = prow[:r].tolist(), pcol[:r].copy()
        W = M
    else:
        W = [[int(x) for x in row] for row in A.tolist()]
        is_piv = [False] * m
        pivrows, piv_list = [], []
        for j in range(n):
            cand = [q for q in range(m) if not is_piv[q] and W[q][j] % p]
            if not cand:
                continue
            r0 = cand[0]
            inv = pow(W[r0][j], p - 2, p)
            for q in range(m):
                if q == r0 or is_piv[q] or W[q][j] == 0:
                    continue
                g = W[q][j] * inv % p
                W[q][j] = g
                for c in range(j + 1, n):
                    W[q][c] = (W[q][c] - g * W[r0][c]) % p
            is_piv[r0] = True
            pivrows.append(r0)
            piv_list.append(j)
        W = np.array(W, dtype=np.uint64).reshape(m, n)
        is_piv = np.array(is_piv, dtype=bool)
        pivots = np.array(piv_list, dtype=np.int64)
        r = len(pivrows)
    perm = np.array(list(pivrows) + [q for q in range(m) if not is_piv[q]], dtype=np.int64)
    LU = W[perm] if m else W
    return LU.astype(np.uint64), perm, int(r), np.asarray(pivots, dtype=np.int64)


def lup_factors(LU, perm, rank: int, pivots, p: int):
    """(Pmat, L, U) as dense uint64 arrays from the packed LUP output: Pmat is
    the m x m permutation with (Pmat A)[i] = A[perm[i]], L is unit lower
    triangular (m x m) with L[i][s] = LU[i][pivots[s]] for s < min(i, rank),
    and U (m x n) is LU with the L entries cleared and rows from the rank on
    zero."""
    LU = np.asarray(LU, dtype=np.uint64)
    m, n = LU.shape
    Pm = np.zeros((m, m), dtype=np.uint64)
    for i, q in enumerate(perm):
        Pm[i, int(q)] = 1
    L = np.eye(m, dtype=np.uint64)
    U = np.zeros((m, n), dtype=np.uint64)
    J = [int(c) for c in pivots]
    for i in range(m):
        for s in range(min(i, rank)):
            L[i, s] = LU[i, J[s]]
        if i < rank:
            U[i] = LU[i]
            for s in range(i):
                U[i, J[s]] = 0
    return Pm, L, U
