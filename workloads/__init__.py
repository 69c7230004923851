"""Seeded synthetic inputs for exact Gaussian elimination over F_p.

This module is shared by the test oracle and the GPU path.  It draws numbers
and shapes only: it holds no elimination arithmetic.  Every generator takes an
explicit seed and uses numpy's PCG64 (``numpy.random.default_rng``), so the
same call returns the same bytes on every machine.

Workloads follow the benchmark of the paper (Sec. 4.1): dense, fully random
square matrices with entries uniform in [0, p).  The five named workloads are

* ``c1`` -- one n=256 system, p = 2^31-1, one right-hand side (seed 1);
* ``c2`` -- one n=8192 system, a seeded 31-bit prime, 16 right-hand sides
  (seed 2);
* ``c3`` -- one n=16384 system, a seeded 31-bit prime, 64 right-hand sides
  (seed 3);
* ``c4`` -- 4096 independent systems, n uniform in [32, 512], 1..8 right-hand
  sides, one seeded 31-bit prime per system, 205 of them made rank deficient
  (seed 4);
* ``c5`` -- 64 instances of a 12000 x 10000 matrix sharing one sparsity
  pattern (200 non-zeros per independent row, 2500 dependent rows), p = 2^31-1
  (seed 5).  It stands in for the sample-point systems of the paper's
  applications (Sec. 5.5), whose data are not available.

Beside them, ``monomial_system`` draws the inputs of the system construction
(Sec. 3.3): the basis variables at each sampling point and the index lists of
the monomials of an ansatz (workload ``lm``: 20000 sampling points and 20000
monomials, the largest size the paper times for construction, Sec. 4.2).
"""

from __future__ import annotations

import numpy as np

MERSENNE31 = (1 << 31) - 1

__all__ = [
    "MERSENNE31",
    "is_prime_u32",
    "draw_prime31",
    "draw_prime_bits",
    "uniform",
    "dense_system",
    "config",
    "batched_systems",
    "sparse_pattern_instances",
    "sparse_pattern_instances_torch",
    "small_cases",
    "vandermonde_nodes",
    "monomial_system",
    "LM_CONFIG",
]


def _mr_witness(a: int, n: int, d: int, s: int) -> bool:
    """True when ``a`` proves ``n`` composite (one Miller-Rabin round)."""
    x = pow(a, d, n)
    if x == 1 or x == n - 1:
        return False
    for _ in range(s - 1):
        x = x * x % n
        if x == n - 1:
            return False
    return True


def is_prime_u32(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 4 759 123 141 (bases 2, 7, 61).

    Jaeschke (1993) showed that no composite below 4 759 123 141 is a strong
    pseudoprime to all three bases, which covers every 32-bit integer.
    """
    n = int(n)
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 61):
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    return not any(_mr_witness(a, n, d, s) for a in (2, 7, 61))


def draw_prime31(rng: np.random.Generator) -> int:
    """A prime in [2^30, 2^31): an odd seeded candidate, then step by 2.

    The walk ends because 2^31 - 1 is prime.
    """
    c = int(rng.integers(1 << 30, 1 << 31)) | 1
    while not is_prime_u32(c):
        c += 2
    return c


def draw_prime_bits(rng: np.random.Generator, bits: int) -> int:
    """A prime in [2^(bits-1), 2^bits): an odd seeded candidate, then step by 2."""
    c = int(rng.integers(1 << (bits - 1), 1 << bits)) | 1
    while not is_prime_u32(c):
        c += 2
    return c


def uniform(rng: np.random.Generator, shape, p: int, low: int = 0) -> np.ndarray:
    """Entries uniform in [low, p) as uint32 (canonical residues)."""
    return rng.integers(low, p, size=shape, dtype=np.uint64).astype(np.uint32)


def dense_system(seed: int, n: int, k: int, p: int | None = None, m: int | None = None):
    """A dense m x n system with k right-hand sides, entries uniform in [0, p).

    With ``p`` None the prime is drawn from the seed (31-bit, Miller-Rabin).
    Returns (A, B, p) with A, B uint32 arrays.
    """
    rng = np.random.default_rng(seed)
    if p is None:
        p = draw_prime31(rng)
    m = n if m is None else m
    A = uniform(rng, (m, n), p)
    B = uniform(rng, (m, k), p)
    return A, B, int(p)


CONFIGS = {
    "c1": dict(seed=1, n=256, k=1, p=MERSENNE31),
    "c2": dict(seed=2, n=8192, k=16, p=None),
    "c3": dict(seed=3, n=16384, k=64, p=None),
}


def config(name: str, n: int | None = None):
    """The dense single-system workloads c1..c3 (optionally resized).

    Resizing keeps the seed and the prime rule, so a smaller instance has the
    same value distribution as the named one.
    """
    cfg = dict(CONFIGS[name])
    if n is not None:
        cfg["n"] = n
    return dense_system(cfg["seed"], cfg["n"], cfg["k"], cfg["p"])


def _make_dependent(rng: np.random.Generator, A: np.ndarray, B: np.ndarray, p: int):
    """Overwrite one random row of [A | B] by a random combination of 3 others.

    Coefficients are uniform in [1, p); the combination is applied to the
    augmented row, so the system stays consistent and has rank n-1 with
    overwhelming probability.
    """
    m = A.shape[0]
    t = int(rng.integers(0, m))
    others = [r for r in range(m) if r != t]
    src = rng.choice(others, size=min(3, len(others)), replace=False)
    coef = rng.integers(1, p, size=len(src), dtype=np.uint64)
    aug = np.concatenate([A, B], axis=1).astype(object)
    row = [0] * aug.shape[1]
    for c, s in zip(coef, src):
        row = [(x + int(c) * int(y)) % p for x, y in zip(row, aug[s])]
    row = np.array(row, dtype=np.uint64).astype(np.uint32)
    A[t, :] = row[: A.shape[1]]
    B[t, :] = row[A.shape[1]:]
    return t


def batched_systems(seed: int = 4, count: int = 4096, n_lo: int = 32, n_hi: int = 512,
                    k_lo: int = 1, k_hi: int = 8, deficient_frac: float = 0.05):
    """The c4 batch: ``count`` square systems of uneven size.

    n ~ U{n_lo..n_hi}, k ~ U{k_lo..k_hi} (inclusive), one seeded 31-bit prime
    per system, entries uniform in [0, p).  round(deficient_frac*count)
    systems, chosen without replacement, get one row replaced by a random
    combination of three other rows (on the augmented matrix).
    Returns a list of dicts {A, B, p, n, k, deficient}.
    """
    root = np.random.SeedSequence(seed)
    top = np.random.default_rng(root)
    ns = top.integers(n_lo, n_hi + 1, size=count)
    ks = top.integers(k_lo, k_hi + 1, size=count)
    n_def = int(round(deficient_frac * count))
    deficient = set(top.choice(count, size=n_def, replace=False).tolist()) if n_def else set()
    out = []
    for s, child in enumerate(root.spawn(count)):
        rng = np.random.default_rng(child)
        p = draw_prime31(rng)
        n, k = int(ns[s]), int(ks[s])
        A = uniform(rng, (n, n), p)
        B = uniform(rng, (n, k), p)
        if s in deficient:
            _make_dependent(rng, A, B, p)
        out.append(dict(A=A, B=B, p=p, n=n, k=k, deficient=s in deficient))
    return out


def _sparse_pattern(seed: int, count: int, m: int, n: int, base_rows: int, nnz: int):
    """The shared structure of the c5 family: per base row its ``nnz`` column
    positions, per dependent row its two source base rows, the shared row
    permutation, and one seed sequence per instance."""
    root = np.random.SeedSequence(seed)
    pat_rng = np.random.default_rng(root.spawn(1)[0])
    cols = np.stack([pat_rng.choice(n, size=nnz, replace=False) for _ in range(base_rows)])
    dep = np.stack([pat_rng.choice(base_rows, size=2, replace=False)
                    for _ in range(m - base_rows)])
    perm = pat_rng.permutation(m)
    children = np.random.SeedSequence([seed, 1]).spawn(count)
    return cols, dep, perm, children


def _instance_draws(child, m: int, base_rows: int, nnz: int, p: int):
    """One instance's values at the shared positions and its dependent-row
    coefficients, both uniform in [1, p)."""
    rng = np.random.default_rng(child)
    vals = rng.integers(1, p, size=(base_rows, nnz), dtype=np.uint64)
    coef = rng.integers(1, p, size=(m - base_rows, 2), dtype=np.uint64)
    return vals, coef


def sparse_pattern_instances(seed: int = 5, count: int = 64, m: int = 12000, n: int = 10000,
                             base_rows: int = 9500, nnz: int = 200, p: int = MERSENNE31,
                             instances=None):
    """The c5 family: ``count`` instances sharing one sparsity pattern.

    ``base_rows`` rows carry exactly ``nnz`` distinct seeded column positions
    (shared by every instance) with values uniform in [1, p) drawn per
    instance.  The remaining m - base_rows rows are c1*R_a + c2*R_b of two
    distinct base rows (indices shared, coefficients per instance, uniform in
    [1, p)).  One shared permutation shuffles the rows.  ``instances`` selects
    a subset of instance indices to materialise (default: all).
    Yields (index, A) with A an m x n uint32 array.
    """
    cols, dep, perm, children = _sparse_pattern(seed, count, m, n, base_rows, nnz)
    wanted = range(count) if instances is None else instances
    for idx in wanted:
        vals, coef = _instance_draws(children[idx], m, base_rows, nnz, p)
        base = np.zeros((base_rows, n), dtype=np.uint64)
        np.put_along_axis(base, cols, vals, axis=1)
        A = np.zeros((m, n), dtype=np.uint64)
        A[:base_rows] = base
        for t in range(m - base_rows):
            a, b = dep[t]
            # products < 2^62 and their sum < 2^63 fit uint64
            A[base_rows + t] = (coef[t, 0] * base[a] % p + coef[t, 1] * base[b] % p) % p
        yield idx, A[perm].astype(np.uint32)


def sparse_pattern_instances_torch(device, seed: int = 5, count: int = 64, m: int = 12000,
                                   n: int = 10000, base_rows: int = 9500, nnz: int = 200,
                                   p: int = MERSENNE31, instances=None):
    """The same matrices as ``sparse_pattern_instances``, assembled with torch
    on ``device`` (the random draws stay on the host, in the same order), so
    that a full-size batch need not pass through host memory.  Yields
    (index, A) with A an m x n int32 tensor (residues below 2^31)."""
    import torch
    cols, dep, perm, children = _sparse_pattern(seed, count, m, n, base_rows, nnz)
    cols_t = torch.from_numpy(cols.astype(np.int64)).to(device)
    dep_t = torch.from_numpy(dep.astype(np.int64)).to(device)
    perm_t = torch.from_numpy(perm.astype(np.int64)).to(device)
    wanted = range(count) if instances is None else instances
    for idx in wanted:
        vals, coef = _instance_draws(children[idx], m, base_rows, nnz, p)
        vals_t = torch.from_numpy(vals.astype(np.int64)).to(device)
        coef_t = torch.from_numpy(coef.astype(np.int64)).to(device)
        A = torch.zeros((m, n), dtype=torch.int64, device=device)
        A[:base_rows].scatter_(1, cols_t, vals_t)
        step = 512
        for t0 in range(0, m - base_rows, step):
            t1 = min(t0 + step, m - base_rows)
            ra = A[dep_t[t0:t1, 0]]
            rb = A[dep_t[t0:t1, 1]]
            # products < 2^62 and their sum < 2^63 fit int64
            A[base_rows + t0: base_rows + t1] = (coef_t[t0:t1, :1] * ra % p
                                                 + coef_t[t0:t1, 1:] * rb % p) % p
            del ra, rb
        yield idx, A[perm_t].to(torch.int32)
        del A


SMALL_PRIMES = (2, 3, 5, 7, 65521, (1 << 20) + 7, MERSENNE31)


def small_cases(seed: int, count: int, max_dim: int = 64, max_k: int = 8):
    """Randomised small shapes and structures for parity tests.

    Each case is a dict {A, B, p, kind}.  Kinds: dense, rank-deficient
    (product of thin factors), duplicate rows, zero matrix, identity, first
    column zero, wide (m < n), tall (m > n).  Primes cycle through a fixed set
    plus seeded 31-bit primes.
    """
    rng = np.random.default_rng(seed)
    kinds = ["dense", "lowrank", "duprows", "zero", "identity", "col0zero", "wide", "tall"]
    out = []
    for i in range(count):
        kind = kinds[i % len(kinds)]
        if i % 9 == 8:
            p = draw_prime31(rng)
        else:
            p = SMALL_PRIMES[int(rng.integers(0, len(SMALL_PRIMES)))]
        m = int(rng.integers(1, max_dim + 1))
        n = int(rng.integers(1, max_dim + 1))
        if kind == "wide" and m >= n:
            m, n = min(m, n), max(m, n) + 1
        if kind == "tall" and m <= n:
            m, n = max(m, n) + 1, min(m, n)
        k = int(rng.integers(0, max_k + 1))
        if kind == "lowrank":
            r = int(rng.integers(0, min(m, n) + 1))
            L = uniform(rng, (m, r), p).astype(object)
            R = uniform(rng, (r, n), p).astype(object)
            A = (L.dot(R) % p if r else np.zeros((m, n), dtype=object)).astype(np.uint64)
            A = A.astype(np.uint32)
        elif kind == "zero":
            A = np.zeros((m, n), dtype=np.uint32)
        elif kind == "identity":
            A = np.eye(m, n, dtype=np.uint32)
        else:
            A = uniform(rng, (m, n), p)
            if kind == "duprows" and m > 1:
                src = rng.integers(0, m, size=m // 2)
                dst = rng.integers(0, m, size=m // 2)
                A[dst] = A[src]
            if kind == "col0zero":
                A[:, 0] = 0
        B = uniform(rng, (m, k), p)
        if kind in ("lowrank", "duprows") and k and m:
            # make half the right-hand sides consistent: B = A @ Y
            Y = uniform(rng, (n, k), p).astype(object)
            cons = (A.astype(object).dot(Y) % p).astype(np.uint64).astype(np.uint32)
            B[:, ::2] = cons[:, ::2]
        out.append(dict(A=A, B=B, p=int(p), kind=kind))
    return out


def vandermonde_nodes(seed: int, count: int, p: int, distinct: bool = True) -> np.ndarray:
    """Seeded evaluation nodes in [0, p); distinct unless asked otherwise."""
    rng = np.random.default_rng(seed)
    if distinct:
        assert count <= p
        if p < 1 << 20:
            return rng.permutation(p)[:count].astype(np.uint64)
        seen: list[int] = []
        s = set()
        while len(seen) < count:
            x = int(rng.integers(0, p))
            if x not in s:
                s.add(x)
                seen.append(x)
        return np.array(seen, dtype=np.uint64)
    return rng.integers(0, p, size=count, dtype=np.uint64)


# System construction (Sec. 3.3): square, like the paper's timings (Sec. 4.2).
LM_CONFIG = dict(seed=6, nrows=20000, ncols=20000, nbasis=48, d=12, p=MERSENNE31)


def monomial_system(seed: int = 6, nrows: int = 20000, ncols: int = 20000, nbasis: int = 48,
                    d: int = 12, p: int = MERSENNE31):
    """(bases, lindices, p) for the system construction.

    bases (nrows x nbasis, uint32): column 0 is the dummy variable 1 that pads
    shorter monomials (the paper's helper pads to one uniform degree); the
    other basis variables are uniform in [1, p) at each sampling point.
    lindices (ncols x d, int32): monomial c has a degree uniform in [1, d];
    its variables are uniform in [1, nbasis) and the remaining d - degree
    slots name the dummy variable 0.
    """
    rng = np.random.default_rng(seed)
    bases = uniform(rng, (nrows, nbasis), p, low=1)
    if nbasis:
        bases[:, 0] = 1
    deg = rng.integers(1, d + 1, size=ncols) if d else np.zeros(ncols, np.int64)
    hi = max(nbasis, 2)
    L = rng.integers(1, hi, size=(ncols, d)).astype(np.int32)
    L[np.arange(d)[None, :] >= deg[:, None]] = 0
    return bases, L, int(p)
