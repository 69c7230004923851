/*
 * linac-mi355x: exact Gaussian elimination over a prime field F_p on AMD
 * Instinct MI355X (gfx950).
 *
 * The operations follow the statement of the method in "Linac: linear algebra
 * with CUDA over finite fields" (De Laurentis, Franklin):
 *   - row reduction to reduced row-echelon form (RREF) in the original shape,
 *     zero rows at the bottom, with field_characteristic = p selecting exact
 *     arithmetic mod p (Sec. 2.3 "Basic Usage"; Sec. 3.2);
 *   - the rank and the pivot columns of the RREF (Sec. 5.1);
 *   - solving A X = B by reducing the augmented matrix [A | B]: a column of B
 *     is consistent iff rank(A) = rank([A | b]); the particular solution sets
 *     the free (non-pivot) variables to zero (Sec. 5.2).
 *
 * Conventions shared by every entry point
 *   - Residues are canonical: 0 <= a < p, stored as uint32.  p must be a prime
 *     with 2 <= p < 2^31 (so a residue is also a non-negative int32).
 *   - Matrices are row-major with an explicit leading dimension (elements
 *     between the starts of consecutive rows).
 *   - Every array pointer is a DEVICE pointer owned by the caller.  The library
 *     never allocates device memory: scratch space comes from the caller's
 *     workspace `ws` of `ws_bytes` bytes, sized by the matching *_workspace
 *     query.  No pointer is kept after a call returns.
 *   - Calls are asynchronous on the HIP stream `s` (NULL = the null stream);
 *     outputs are valid once the stream has been synchronised.  Calls on
 *     distinct streams with distinct workspaces may run concurrently and give
 *     the same results.  Two library-internal resources are shared per
 *     device: the blocked int8 path overlaps a panel's trailing update with
 *     the next panel on one side stream per device, so the trailing parts of
 *     concurrent blocked calls on one device queue behind each other there;
 *     and linac_rref_batched calls on one device take turns on its lanes.
 *   - Errors are returned, never thrown.  All argument checks run on the host
 *     before any device work, so a non-OK return from a check leaves every
 *     buffer untouched.  On LINAC_E_HIP the outputs are unspecified and
 *     linac_last_hip_error() gives the HIP error code.
 *   - m = 0, n = 0 or k = 0 are valid shapes (rank 0).
 */
#ifndef LINAC_H
#define LINAC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LINAC_OK = 0,
    LINAC_E_INVALID_ARG = 1, /* null pointer, negative size, leading dimension too small */
    LINAC_E_UNSUPPORTED = 2, /* p = 0 (floating-point mode), p >= 2^31, path not available */
    LINAC_E_NOT_PRIME = 3,   /* p is not prime (deterministic Miller-Rabin, bases 2, 7, 61) */
    LINAC_E_RANGE = 4,       /* an entry is >= p (checked only with opts.validate) */
    LINAC_E_WORKSPACE = 5,   /* ws is NULL or smaller than the workspace query */
    LINAC_E_NOMEM = 6,       /* problem does not fit in 64-bit byte counts */
    LINAC_E_HIP = 7          /* a HIP runtime call failed */
} linac_status;

enum {
    LINAC_PATH_AUTO = 0,
    LINAC_PATH_PLAIN = 1,        /* one fused Gauss-Jordan step kernel per pivot column */
    LINAC_PATH_BLOCKED_INT8 = 2, /* blocked, trailing update on int8 MFMA (balanced limbs) */
    LINAC_PATH_BLOCKED_FP64 = 3  /* blocked, trailing update on FP64 MFMA (p < 2^21) */
};

typedef struct {
    int path;          /* LINAC_PATH_*; AUTO picks by p and size */
    int panel_width;   /* blocked paths: panel width, 0 = tuned default */
    int validate;      /* non-zero: check 0 <= entry < p on the device first.  This
                          makes the call synchronous (it reads a flag back) and
                          returns LINAC_E_RANGE on failure */
    int verbose;       /* non-zero: print the chosen path and launch geometry */
    hipEvent_t ev_begin; /* optional (may be NULL): recorded on `s` immediately before
                            the first launch of the path's dominant kernel */
    hipEvent_t ev_end;   /* optional: recorded immediately after its last launch */
    int64_t* dominant_launches; /* optional HOST pointer: receives the number of
                                   launches of the dominant kernel */
    /* Optional per-launch timing (for profiling; adds an event record around
     * every hot-kernel launch).  launch_events: HOST array of 2 * launch_cap
     * caller-created events; pair i brackets the i-th recorded launch, whose
     * kind (LINAC_KERNEL_*) goes to launch_kinds[i] (HOST array of launch_cap).
     * *launch_used (HOST) receives the number of pairs recorded. */
    hipEvent_t* launch_events;
    int32_t* launch_kinds;
    int32_t launch_cap;
    int32_t* launch_used;
} linac_opts;

enum {
    LINAC_KERNEL_STEP = 1,          /* fused Gauss-Jordan step (plain path and panel leaves) */
    LINAC_KERNEL_LEAF_PRODUCT = 2,  /* blocked: leaf transform applied to the panel buffer */
    LINAC_KERNEL_TRAIL_PRODUCT = 3, /* blocked: panel transform applied to the trailing columns */
    LINAC_KERNEL_BATCHED = 4,       /* batched persistent launch */
    LINAC_KERNEL_SELECT = 5,        /* blocked: pivot selection of a leaf */
    LINAC_KERNEL_OPERANDS = 6,      /* blocked: building the MFMA operands of a product */
    LINAC_KERNEL_LEAF_FUSED = 7     /* blocked int8, leaf pipeline: a leaf's product on all rows
                                       but the next leaf's first chunk, in one launch with that
                                       leaf's first pivot selection */
};

/*
 * The plan a call on an m x n system would follow: *path receives the path
 * (LINAC_PATH_PLAIN, _BLOCKED_INT8 or _BLOCKED_FP64; AUTO resolved by size and
 * the tuning table) and *panel the panel width of a blocked path (0 for the
 * plain path).  Both are HOST pointers.  Depends only on the shape and opts
 * (never on p or the data), so it matches the workspace queries.  Returns
 * LINAC_E_INVALID_ARG for a NULL pointer or a negative size, and for a panel
 * width outside 32..512 or not a multiple of 32.
 */
linac_status linac_plan(int64_t m, int64_t n, const linac_opts* opts, int* path, int* panel);

/* Workspace (bytes) needed by linac_rref for an m x n matrix. */
linac_status linac_rref_workspace(int64_t m, int64_t n, const linac_opts* opts, size_t* bytes);

/*
 * RREF of A over F_p, in place (Sec. 2.3; Sec. 3.2; Fig. 1).
 *   A       device, m x n row-major, leading dimension lda >= max(n, 1); on
 *           return it holds the RREF: the rank r non-zero rows first, each with a
 *           leading 1 in its pivot column, pivot columns zero elsewhere, the
 *           remaining m - r rows zero.
 *   rank    device int32[1]: r.
 *   pivots  device int32[min(m, n)]: the pivot columns in ascending order,
 *           -1 from index r on.  May be NULL when min(m, n) = 0.
 */
linac_status linac_rref(uint32_t* A, int64_t m, int64_t n, int64_t lda, uint32_t p,
                        int32_t* rank, int32_t* pivots, void* ws, size_t ws_bytes,
                        const linac_opts* opts, hipStream_t s);

/* Workspace (bytes) needed by linac_solve for A m x n and B m x k. */
linac_status linac_solve_workspace(int64_t m, int64_t n, int64_t k, const linac_opts* opts,
                                   size_t* bytes);

/*
 * Solve A X = B over F_p by reducing [A | B] (Sec. 5.2).  A and B are not
 * modified.  Pivots are searched only in A's n columns.
 *   A           device, m x n, leading dimension lda >= max(n, 1).
 *   B           device, m x k, leading dimension ldb >= max(k, 1).
 *   X           device, n x k, leading dimension ldx >= max(k, 1): the
 *               particular solution with free variables zero; column t is all
 *               zero when it is inconsistent.
 *   rank        device int32[1]: rank(A).
 *   pivots      device int32[min(m, n)]: ascending pivot columns of A, -1 padded
 *               (may be NULL when min(m, n) = 0).
 *   consistent  device uint8[k]: 1 iff rank(A) = rank([A | b_t]) (may be NULL
 *               when k = 0).
 */
linac_status linac_solve(const uint32_t* A, int64_t m, int64_t n, int64_t lda,
                         const uint32_t* B, int64_t k, int64_t ldb, uint32_t p,
                         uint32_t* X, int64_t ldx, int32_t* rank, int32_t* pivots,
                         uint8_t* consistent, void* ws, size_t ws_bytes,
                         const linac_opts* opts, hipStream_t s);

/* One matrix of a batched RREF: the linac_rref arguments, with its own prime. */
typedef struct {
    uint32_t* A;      /* device, m x n, reduced in place */
    int64_t m, n, lda;
    uint32_t p;
    int32_t* rank;    /* device int32[1] */
    int32_t* pivots;  /* device int32[min(m, n)] (may be NULL when min(m, n) = 0) */
} linac_matrix;

/* Workspace (bytes) for linac_rref_batched on this host array of matrices: the
 * number of lanes (see below) times the largest single-matrix workspace. */
linac_status linac_rref_batched_workspace(const linac_matrix* mats, int32_t count,
                                          const linac_opts* opts, size_t* bytes);

/*
 * RREF of `count` independent matrices in one call (Sec. 2.3, Sec. 3.2 per
 * matrix; the paper reduces one matrix per call, and its applications reduce
 * many sample-point systems of one shape, Sec. 5.5).  Per matrix the results
 * equal those of linac_rref.  `mats` is a HOST array read during the call only.
 * The matrices are spread over "lanes" (tuning key rref_lanes, default 4,
 * at most 8): each lane is an internal stream of the library with its own
 * slice of ws, and takes its matrices one after another, largest first to the
 * least loaded lane; one host thread per lane enqueues that lane's launches.
 * The lanes start after the work already queued on `s` and `s` waits for all
 * of them before its later work, so the call is ordered on `s` like any other.
 * Concurrent lanes overlap one matrix's latency-bound pivot selections with
 * another's matrix products.  Inside a lane the blocked path runs without its
 * look-ahead side stream (one lane keeps it and runs on `s` itself).
 * Calls of this function on one device are serialised by the library (they
 * share the lanes).  opts->ev_begin / ev_end bracket the whole batch; per-launch
 * timing is not recorded.  Errors: as linac_rref for each matrix (checked on the
 * host before any device work); LINAC_E_WORKSPACE.
 */
linac_status linac_rref_batched(const linac_matrix* mats, int32_t count, void* ws, size_t ws_bytes,
                                const linac_opts* opts, hipStream_t s);

/* Size of the fixed scratch array behind linac_solve_noalloc (per GPU). */
#define LINAC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * linac_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and argument checks as linac_solve, without ws/ws_bytes:
 * the scratch space is a fixed array of LINAC_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held from the first call on that GPU until the process
 * ends.  The call allocates nothing (no hipMalloc or hipFree, no stream or
 * event created): the blocked int8 path runs without its look-ahead side
 * stream.  The caller still owns A, B and every output.
 *   - LINAC_E_WORKSPACE when the system needs more scratch than the array holds
 *     (linac_solve_workspace with the same opts gives the need; about
 *     n (n + k) * 4 bytes on the plain path, so up to n of about 4000);
 *   - LINAC_E_UNSUPPORTED with opts->validate (the range check reads a flag
 *     back through a host copy).
 * Every call on a GPU shares that GPU's array and leaves its contents behind;
 * each call initialises what it reads.  Calls that overlap in time on one GPU
 * (different streams, or different host threads without ordering) race on the
 * array: serialise them.
 */
linac_status linac_solve_noalloc(const uint32_t* A, int64_t m, int64_t n, int64_t lda,
                                 const uint32_t* B, int64_t k, int64_t ldb, uint32_t p, uint32_t* X,
                                 int64_t ldx, int32_t* rank, int32_t* pivots, uint8_t* consistent,
                                 const linac_opts* opts, hipStream_t s);

/* One system of a batch: the same meaning as the linac_solve arguments, with its
 * own prime.  Square or rectangular; all pointers are device pointers. */
typedef struct {
    const uint32_t* A;
    const uint32_t* B;
    uint32_t* X;
    int32_t m, n, k;
    int32_t lda, ldb, ldx;
    uint32_t p;
    int32_t* rank;
    int32_t* pivots;
    uint8_t* consistent;
} linac_system;

/* Workspace (bytes) for linac_solve_batched on this host array of systems. */
linac_status linac_solve_batched_workspace(const linac_system* sys, int32_t count,
                                           const linac_opts* opts, size_t* bytes);

/*
 * Solve `count` independent systems in one persistent launch (the paper solves
 * one matrix per call; batching many uneven systems is this library's
 * extension).  `sys` is a HOST array read during the call only.  The library
 * uploads the descriptors into ws and launches a graph that it captured for
 * this (ws, plan) pair on first use, replaying it on later calls.  Per system the
 * results equal those of linac_solve.  Each system must fit one workgroup's
 * bookkeeping: m <= 1024 and n + k <= 2048, else LINAC_E_UNSUPPORTED (before
 * any device work; larger systems go through linac_solve).  With
 * opts->validate every entry of every A and B is checked against its system's
 * prime first (synchronously); an entry >= p returns LINAC_E_RANGE before the
 * batch runs.
 */
linac_status linac_solve_batched(const linac_system* sys, int32_t count, void* ws,
                                 size_t ws_bytes, const linac_opts* opts, hipStream_t s);

/*
 * Matrix of a monomial ansatz evaluated at sampling points (Sec. 3.3, "Building
 * linear systems on GPUs"; the bases / lindices layout of Sec. 2.3):
 *     A[r][c] = prod_{t < d} bases[r][lindices[c][t]]  mod p.
 *   bases     device, nrows x nbasis residues (< p), leading dimension
 *             ldbases >= max(nbasis, 1): row r holds the basis variables at
 *             sampling point r.
 *   lindices  device int32, ncols x d, leading dimension ldl >= max(d, 1): row
 *             c lists the basis variables whose product is monomial c (the
 *             paper's kernel takes one degree d for all monomials; shorter
 *             monomials are padded with a variable equal to 1).  An index
 *             outside [0, nbasis) is a factor 0 (it never reads outside bases).
 *   A         device, nrows x ncols, leading dimension lda >= max(ncols, 1).
 * d = 0 gives A = 1 everywhere.  Entries of bases >= p give unspecified
 * residues (no fault).  Needs no workspace.  Errors: LINAC_E_INVALID_ARG
 * (negative size, leading dimension too small, NULL with a non-empty shape),
 * the modulus errors of the other calls, LINAC_E_NOMEM when a size reaches
 * 2^31, LINAC_E_HIP.
 */
linac_status linac_load_matrix(const uint32_t* bases, int64_t nrows, int64_t nbasis,
                               int64_t ldbases, const int32_t* lindices, int64_t ncols, int64_t d,
                               int64_t ldl, uint32_t p, uint32_t* A, int64_t lda, hipStream_t s);

/*
 * Canonical basis of the null space from an RREF (Sec. 5.1, "Rank
 * factorisation and null spaces"): ker(A) = ker(R), and with the free
 * (non-pivot) columns c_0 < c_1 < ... of R, column f of K is the solution of
 * R x = 0 whose free variables are minus the unit vector e_f:
 *     K[c_f][f] = p - 1,  K[pivots[s]][f] = R[s][c_f],  every other entry 0,
 * so that A K = 0.  The basis has n - r columns, r = *rank.
 *   R          device, m x n RREF as linac_rref returns it, leading dimension
 *              ldr >= max(n, 1); only its first r rows are read.
 *   rank       device int32[1] and pivots device int32[min(m, n)] as linac_rref
 *              returns them (rank is clamped to [0, min(m, n)], so no value
 *              makes the kernel read outside R).
 *   K          device, n x kcols, leading dimension ldk >= max(kcols, 1), with
 *              kcols <= n: columns f < n - r receive the basis, columns from
 *              n - r on are set to zero.  kcols = n always holds the whole
 *              basis (the rank is on the device, so the call never waits for
 *              it); a smaller kcols truncates it.
 *   free_cols  optional device int32[n]: c_f for f < n - r, then -1.
 * Errors as for linac_rref's argument checks.
 */
linac_status linac_nullspace(const uint32_t* R, int64_t m, int64_t n, int64_t ldr,
                             const int32_t* rank, const int32_t* pivots, uint32_t p, uint32_t* K,
                             int64_t kcols, int64_t ldk, int32_t* free_cols, hipStream_t s);

/*
 * The column basis of a rank factorisation (Sec. 5.1): C = A[:, J] for the
 * pivot columns J of A's RREF, so that A = C R with R the first r rows of the
 * RREF.
 *   A       device, m x n (the matrix before reduction), leading dimension
 *           lda >= max(n, 1).
 *   rank, pivots  device, as linac_rref returns them for A.
 *   C       device, m x ccols, leading dimension ldc >= max(ccols, 1), with
 *           ccols <= min(m, n): column s < r receives A's column pivots[s],
 *           columns from r on are zero.
 * Errors: LINAC_E_INVALID_ARG for bad sizes or NULL pointers, LINAC_E_HIP.
 */
linac_status linac_column_basis(const uint32_t* A, int64_t m, int64_t n, int64_t lda,
                                const int32_t* rank, const int32_t* pivots, uint32_t* C,
                                int64_t ccols, int64_t ldc, hipStream_t s);

/*
 * 64-bit primes (Sec. 3.2 "Number types": uint64 storage for primes beyond
 * 32 bits).  Residues are uint64 in [0, p) with p a prime, 2 <= p < 2^63
 * (p >= 2^63: LINAC_E_UNSUPPORTED; composite: LINAC_E_NOT_PRIME, by a
 * deterministic Miller-Rabin test with the first twelve primes as bases).
 * Same meaning, layouts and errors as linac_rref / linac_solve, on one
 * column-at-a-time Gauss-Jordan path: per pivot column one search launch and
 * one row-update launch (Sec. 3.2, Fig. 1).  opts: validate and verbose are
 * honoured, path and panel_width ignored.  Workspaces from the matching
 * queries.
 */
linac_status linac_rref_u64_workspace(int64_t m, int64_t n, size_t* bytes);
linac_status linac_rref_u64(uint64_t* A, int64_t m, int64_t n, int64_t lda, uint64_t p,
                            int32_t* rank, int32_t* pivots, void* ws, size_t ws_bytes,
                            const linac_opts* opts, hipStream_t s);
linac_status linac_solve_u64_workspace(int64_t m, int64_t n, int64_t k, size_t* bytes);
linac_status linac_solve_u64(const uint64_t* A, int64_t m, int64_t n, int64_t lda, const uint64_t* B,
                             int64_t k, int64_t ldb, uint64_t p, uint64_t* X, int64_t ldx,
                             int32_t* rank, int32_t* pivots, uint8_t* consistent, void* ws,
                             size_t ws_bytes, const linac_opts* opts, hipStream_t s);
/* Host-only check of a 64-bit modulus: LINAC_OK for a prime below 2^63. */
linac_status linac_check_prime_u64(uint64_t p);

/*
 * LUP factorisation P A = L U over F_p (the paper names it as future work,
 * Sec. 6), with a fixed pivot rule so that the factors are reproducible: for
 * each column j in turn, the pivot is the first row, in the ORIGINAL row order,
 * that is not a pivot yet and whose current entry in column j is non-zero (a
 * column without one is skipped).  Forward elimination only: a row that is not
 * a pivot yet becomes row - g * (pivot row) with g = its entry / the head.
 *   A      device, m x n, leading dimension lda >= max(n, 1), overwritten with
 *          the packed factors in P order: row i of the output belongs to the
 *          original row perm[i].  With r = rank and J = pivots:
 *            L (m x m, unit lower triangular): L[i][s] = A_out[i][J[s]] for
 *              s < min(i, r); L[i][i] = 1; every other entry 0;
 *            U (m x n, row echelon): for i < r, U[i][c] = A_out[i][c] except
 *              at the columns J[s], s < i, where U is 0; U[i][J[i]] is the
 *              pivot's head (not normalised); rows i >= r of U are zero.
 *          Then (P A)[i] = A[perm[i]] and P A = L U exactly.
 *   perm   device int32[m]: the pivot rows in pivot order, then the other rows
 *          in their original order.
 *   rank, pivots  device, as for linac_rref (J = the pivot columns of the RREF).
 * linac_lup takes 32-bit residues (p < 2^31), linac_lup_u64 64-bit ones
 * (p < 2^63).  Workspace: linac_lup_workspace(m, n, wide = 0 or 1).  opts:
 * validate and verbose are honoured.  Errors as for linac_rref.
 */
linac_status linac_lup_workspace(int64_t m, int64_t n, int wide, size_t* bytes);
linac_status linac_lup(uint32_t* A, int64_t m, int64_t n, int64_t lda, uint32_t p, int32_t* perm,
                       int32_t* rank, int32_t* pivots, void* ws, size_t ws_bytes,
                       const linac_opts* opts, hipStream_t s);
linac_status linac_lup_u64(uint64_t* A, int64_t m, int64_t n, int64_t lda, uint64_t p, int32_t* perm,
                           int32_t* rank, int32_t* pivots, void* ws, size_t ws_bytes,
                           const linac_opts* opts, hipStream_t s);

/* Load tuned parameters for later calls (process-wide); NULL restores the
 * built-in defaults.  Tuning only selects among configurations that give the
 * same results (paths and panel widths all compute the unique RREF).  The text
 * is a JSON object, as written by the autotuner (paper_2605_25863_amd/tune.py):
 *   "blocked_min":    AUTO takes the blocked int8 path once min(m, n) >= this;
 *   "panel":          array of {"n_max": N, "panel": w}: panel width w for
 *                     min(m, n) <= N (first match, ascending N; w a multiple of
 *                     32 in [32, 512]); larger sizes use the last entry;
 *   "batched_per_cu": resident workgroups per compute unit of the batched launch;
 *   "lookahead":      1 (default) or 0: whether the blocked int8 path overlaps the
 *                     next panel's pivot selection with the trailing update (on a
 *                     second stream that the call joins back to s);
 *   "rref_lanes":     1..8, the matrices linac_rref_batched reduces concurrently;
 *   "forward_min":    solves on the blocked int8 path eliminate forward and
 *                     back-substitute once min(m, n) >= this (below it, and for
 *                     every RREF, they run Gauss-Jordan);
 *   "leaf_blocks":    2, 3, 6 or 9: 16-column blocks per workgroup of the blocked
 *                     int8 path's leaf product (a tile shape);
 *   "leaf_pipeline":  1 (default) or 0: whether the blocked int8 path splits each
 *                     leaf's product so that the next leaf's first pivot
 *                     selection runs in the same launch as its larger half.
 * Unknown keys are ignored.  Returns LINAC_E_INVALID_ARG (and keeps the current
 * table) for malformed text or out-of-range values.  Host only. */
linac_status linac_load_tuning(const char* json);

/* Host-only primality check used by argument validation: LINAC_OK when p is a
 * prime below 2^31, LINAC_E_NOT_PRIME when not prime, LINAC_E_UNSUPPORTED when
 * p = 0 or p >= 2^31.  Touches no device. */
linac_status linac_check_prime(uint32_t p);

const char* linac_status_string(linac_status st);
int linac_last_hip_error(void);
int linac_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LINAC_H */
