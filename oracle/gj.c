/*
 * Test oracle -- NOT part of the product.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.
 *
 * Plain, slow, obviously correct Gauss-Jordan elimination over F_p, written
 * from the paper's statement of the method (Sec. 3.2, "Chosen algorithm",
 * "Pivoting", "Conditional Rescale", "Row reduce", "Increment counters", and
 * Fig. 1) and of its applications (Sec. 5.1 rank factorisation, Sec. 5.2
 * solving linear systems).
 *
 * Arithmetic: residues are uint64 in [0, p) with p < 2^32, so every product
 * of two residues is below 2^64 and a plain `%` reduces it.  No Barrett, no
 * Montgomery, no blocking, no reordering: one pivot column at a time, every
 * other row eliminated (Gauss-Jordan, rows above and below the pivot).
 *
 * The only parallelism is OpenMP over the independent rows of one
 * elimination step (or over independent systems in the batch entry point);
 * it does not change any arithmetic.
 */
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Modular inverse by the extended Euclidean algorithm (a != 0 mod p). */
uint64_t oracle_inv(uint64_t a, uint64_t p)
{
    int64_t t = 0, newt = 1;
    int64_t r = (int64_t)p, newr = (int64_t)(a % p);
    while (newr != 0) {
        int64_t q = r / newr;
        int64_t tmp = t - q * newt; t = newt; newt = tmp;
        tmp = r - q * newr; r = newr; newr = tmp;
    }
    if (r != 1) return 0; /* not invertible */
    if (t < 0) t += (int64_t)p;
    return (uint64_t)t;
}

/* a^e mod p by square-and-multiply (used by the tests to cross-check the
 * inverse through Fermat's little theorem). */
uint64_t oracle_powmod(uint64_t a, uint64_t e, uint64_t p)
{
    uint64_t r = 1 % p, b = a % p;
    while (e) {
        if (e & 1) r = r * b % p;
        b = b * b % p;
        e >>= 1;
    }
    return r;
}

/*
 * Reduce the m x ncols row-major matrix M (leading dimension ncols) to reduced
 * row-echelon form over F_p, searching pivots only in columns [0, nsearch)
 * while carrying every column.  For each pivot column j, in order:
 *   a. the pivot is the first row r >= i with M[r][j] != 0 (any non-zero
 *      entry is a valid pivot over a field); if there is none the column is
 *      free and j advances alone;
 *   b. rows r and i are swapped;
 *   c. the head M[i][j] is inverted and row i is scaled so the head is 1;
 *   d. every other row q with f = M[q][j] != 0 gets row_q -= f * row_i;
 *   e. j is recorded as a pivot column and i advances.
 * Returns the rank and writes the ascending pivot columns to pivcols.
 * When det_out is non-NULL and the matrix is square in its searched part,
 * *det_out receives (-1)^swaps * prod(heads before scaling), or 0 when a
 * column has no pivot.
 */
int64_t oracle_gauss_jordan(uint64_t *M, int64_t m, int64_t ncols, int64_t nsearch,
                            uint64_t p, int64_t *pivcols, uint64_t *det_out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t i = 0;
    uint64_t det = 1 % p;
    int singular = 0;
    for (int64_t j = 0; j < nsearch; ++j) {
        if (i == m) { singular = 1; break; }
        int64_t r = -1;
        for (int64_t q = i; q < m; ++q)
            if (M[q * ncols + j] != 0) { r = q; break; }
        if (r < 0) { singular = 1; continue; }
        if (r != i) {
            for (int64_t c = 0; c < ncols; ++c) {
                uint64_t t = M[i * ncols + c];
                M[i * ncols + c] = M[r * ncols + c];
                M[r * ncols + c] = t;
            }
            det = (p - det) % p;
        }
        uint64_t *pr = M + i * ncols;
        uint64_t head = pr[j];
        det = det * head % p;
        uint64_t inv = oracle_inv(head, p);
        for (int64_t c = j; c < ncols; ++c) pr[c] = pr[c] * inv % p;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < m; ++q) {
            if (q == i) continue;
            uint64_t *row = M + q * ncols;
            uint64_t f = row[j];
            if (f == 0) continue;
            for (int64_t c = j; c < ncols; ++c)
                row[c] = (row[c] + p - f * pr[c] % p) % p;
        }
        pivcols[i] = j;
        ++i;
    }
    if (det_out) *det_out = singular ? 0 : det;
    return i;
}

/*
 * Many independent systems, one thread per system (OpenMP over systems).
 * System s is the row-major matrix at mats + offs[s] with rows[s] rows,
 * cols[s] columns and nsearch[s] searchable columns, modulus ps[s].  Its rank
 * goes to ranks[s] and its pivot columns to pivs + pivoffs[s].
 */
void oracle_gauss_jordan_many(uint64_t *mats, const int64_t *offs, const int64_t *rows,
                              const int64_t *cols, const int64_t *nsearch, const uint64_t *ps,
                              int64_t *ranks, int64_t *pivs, const int64_t *pivoffs,
                              int64_t count, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < count; ++s) {
        ranks[s] = oracle_gauss_jordan(mats + offs[s], rows[s], cols[s], nsearch[s], ps[s],
                                       pivs + pivoffs[s], NULL, 1);
    }
}

/* The number of threads OpenMP would use (reported next to timings). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * The same Gauss-Jordan for primes up to 2^63 (Sec. 3.2 "Number types": uint64
 * storage for primes beyond 32 bits): identical steps, with every product of
 * two residues formed in 128 bits before `%`.  The inverse is the extended
 * Euclidean algorithm of oracle_inv (its signed 64-bit values stay below p).
 */
static uint64_t mulmod_wide(uint64_t a, uint64_t b, uint64_t p)
{
    return (uint64_t)((unsigned __int128)a * b % p);
}

int64_t oracle_gauss_jordan_wide(uint64_t *M, int64_t m, int64_t ncols, int64_t nsearch,
                                 uint64_t p, int64_t *pivcols, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t i = 0;
    for (int64_t j = 0; j < nsearch && i < m; ++j) {
        int64_t r = -1;
        for (int64_t q = i; q < m; ++q)
            if (M[q * ncols + j] != 0) { r = q; break; }
        if (r < 0) continue;
        if (r != i) {
            for (int64_t c = 0; c < ncols; ++c) {
                uint64_t t = M[i * ncols + c];
                M[i * ncols + c] = M[r * ncols + c];
                M[r * ncols + c] = t;
            }
        }
        uint64_t *pr = M + i * ncols;
        uint64_t inv = oracle_inv(pr[j], p);
        for (int64_t c = j; c < ncols; ++c) pr[c] = mulmod_wide(pr[c], inv, p);
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < m; ++q) {
            if (q == i) continue;
            uint64_t *row = M + q * ncols;
            uint64_t f = row[j];
            if (f == 0) continue;
            for (int64_t c = j; c < ncols; ++c) {
                uint64_t t = mulmod_wide(f, pr[c], p);
                row[c] = row[c] >= t ? row[c] - t : row[c] + (p - t);
            }
        }
        pivcols[i] = j;
        ++i;
    }
    return i;
}

/*
 * LUP factorisation with the first-non-zero pivot rule in the original row
 * order (the paper names LU factorisation as future work, Sec. 6).  Rows are
 * never swapped in M: for each column j, the pivot is the smallest row index q
 * not yet a pivot with M[q][j] != 0; every other non-pivot row q gets the
 * multiplier g = M[q][j] / M[piv][j], which replaces M[q][j], and
 * M[q][c] -= g * M[piv][c] for c > j.  The pivot row is left as it is.
 * is_piv_step[q] receives the step at which row q became a pivot, or -1;
 * pivrows[s] / pivcols[s] the s-th pivot row and column.  Returns the rank.
 * Products are formed in 128 bits, so p may be any prime below 2^63.
 */
int64_t oracle_lup(uint64_t *M, int64_t m, int64_t n, uint64_t p, int64_t *is_piv_step,
                   int64_t *pivrows, int64_t *pivcols, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int64_t q = 0; q < m; ++q) is_piv_step[q] = -1;
    int64_t rank = 0;
    for (int64_t j = 0; j < n && rank < m; ++j) {
        int64_t piv = -1;
        for (int64_t q = 0; q < m; ++q)
            if (is_piv_step[q] < 0 && M[q * n + j] != 0) { piv = q; break; }
        if (piv < 0) continue;
        const uint64_t *u = M + piv * n;
        uint64_t inv = oracle_inv(u[j], p);
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < m; ++q) {
            if (q == piv || is_piv_step[q] >= 0) continue;
            uint64_t *row = M + q * n;
            if (row[j] == 0) continue;
            uint64_t g = mulmod_wide(row[j], inv, p);
            row[j] = g;
            for (int64_t c = j + 1; c < n; ++c) {
                uint64_t t = mulmod_wide(g, u[c], p);
                row[c] = row[c] >= t ? row[c] - t : row[c] + (p - t);
            }
        }
        is_piv_step[piv] = rank;
        pivrows[rank] = piv;
        pivcols[rank] = j;
        ++rank;
    }
    return rank;
}
