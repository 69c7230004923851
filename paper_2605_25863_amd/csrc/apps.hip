// Around the elimination: building a system from monomials (before it) and
// reading bases off the RREF (after it).
//
//  * load_matrix_kernel: A[r][c] = prod_t bases[r][lindices[c][t]] mod p, the
//    matrix of a monomial ansatz evaluated at sampling points (Sec. 3.3, with
//    the bases / lindices layout of Sec. 2.3).  The paper gives a block one
//    sampling point, stages its bases row in shared memory and lets each
//    thread run through monomials.  Here a workgroup takes a tile of 32
//    sampling points x 256 monomials: each lane keeps its monomial's indices
//    in registers for the whole tile (they are re-read once per 32 rows, not
//    once per row), the tile's bases rows sit in LDS as FP64 values with one
//    extra zero slot per row, and the lane runs four sampling points at a
//    time as independent multiplication chains.  The store of a row is one
//    contiguous 256-column strip per workgroup.
//  * nullspace_kernel: the canonical basis K of ker(A) = ker(R) from the RREF
//    R: free variables take -I, pivot variables the entries of R (Sec. 5.1).
//  * column_basis_kernel: C = A[:, J] for the pivot columns J, the left factor
//    of the rank factorisation A = C R (Sec. 5.1).
//
// Arithmetic of the chains: a product of two residues in FP64 with a
// round-to-nearest quotient.  For |a| < 2^32 and 0 <= b < 2^31,
// h = fl(a b) and l = a b - h (exact by FMA); q = rint(h / p) is within one
// of the nearest quotient, and r = fma(-q, p, h) + l = a b - q p is an
// integer below 2^33 in magnitude, computed exactly.  The quotient error of
// fl(h * fl(1/p)) is below 2^-19, so |r| <= p/2 + 1: the chain keeps signed
// representatives of size ~p/2 and is made canonical once at the end.
#include <algorithm>

#include "internal.h"

namespace linac {

namespace {

constexpr int kLmThreads = 256;
constexpr int kLmRows = 32;               // sampling points per workgroup
constexpr int kLmRowGroup = 4;            // independent chains per lane
constexpr int kLmLdsBytes = 64 * 1024;    // bases staged per workgroup

__device__ __forceinline__ double mulmod_signed(double a, double b, double p, double pinv) {
    const double h = a * b;
    const double l = __fma_rn(a, b, -h);
    const double q = rint(h * pinv);
    return __fma_rn(-q, p, h) + l;
}

__device__ __forceinline__ uint32_t canonical(double r, double p) {
    if (r < 0.0) r += p;
    if (r >= p) r -= p;
    return (uint32_t)r;
}

// kDM: the largest monomial degree this instance keeps in registers (d <= kDM).
// kStaged: bases rows in LDS (nb + 1 doubles each fit kLmLdsBytes), else they
// are read from global memory (L1/L2) with the same zero for bad indices.
template <int kDM, bool kStaged>
__global__ __launch_bounds__(kLmThreads) void load_matrix_kernel(
    const uint32_t* __restrict__ bases, int32_t nrows, int32_t nb, int64_t ldbases,
    const int32_t* __restrict__ lind, int32_t ncols, int32_t d, int64_t ldl, FieldConst F,
    uint32_t* __restrict__ A, int64_t lda, int32_t rows_per_stage) {
    extern __shared__ double s_b[];  // rows_per_stage x (nb + 1); slot nb holds 0
    const int64_t c = (int64_t)blockIdx.x * kLmThreads + threadIdx.x;
    const bool col_ok = c < ncols;
    const int32_t stride = nb + 1;
    const double p = F.dp, pinv = F.pinv;

    // indices of this lane's monomial; anything outside [0, nb) names slot nb (0)
    uint32_t idx[kDM];
#pragma unroll
    for (int t = 0; t < kDM; ++t) {
        const int32_t v = (t < d && col_ok) ? lind[c * ldl + t] : 0;
        idx[t] = min((uint32_t)v, (uint32_t)nb);
    }

    for (int32_t r0 = blockIdx.y * kLmRows; r0 < nrows; r0 += gridDim.y * kLmRows) {
        const int32_t r1 = min(r0 + kLmRows, nrows);
        for (int32_t rs = r0; rs < r1; rs += rows_per_stage) {
            const int32_t nrs = min(rows_per_stage, r1 - rs);
            if constexpr (kStaged) {
                __syncthreads();  // the previous stage has been consumed
                for (int32_t i = threadIdx.x; i < nrs * stride; i += kLmThreads) {
                    const int32_t rr = i / stride, v = i - rr * stride;
                    s_b[i] = v < nb ? (double)bases[(int64_t)(rs + rr) * ldbases + v] : 0.0;
                }
                __syncthreads();
            }
            for (int32_t rr = 0; rr < nrs; rr += kLmRowGroup) {
                double acc[kLmRowGroup];
                auto factor = [&](int u, int t) -> double {
                    const int32_t row = min(rr + u, nrs - 1);  // clamped: always a valid row
                    if constexpr (kStaged) {
                        return s_b[row * stride + idx[t]];
                    } else {
                        const uint32_t i = idx[t];
                        const uint32_t v = bases[(int64_t)(rs + row) * ldbases + min(i, (uint32_t)(nb - 1))];
                        return i < (uint32_t)nb ? (double)v : 0.0;
                    }
                };
                if (d == 0) {
#pragma unroll
                    for (int u = 0; u < kLmRowGroup; ++u) acc[u] = 1.0;
                } else {
#pragma unroll
                    for (int u = 0; u < kLmRowGroup; ++u) acc[u] = factor(u, 0);
                }
#pragma unroll
                for (int t = 1; t < kDM; ++t) {
                    if (t < d) {
                        double f[kLmRowGroup];
#pragma unroll
                        for (int u = 0; u < kLmRowGroup; ++u) f[u] = factor(u, t);
#pragma unroll
                        for (int u = 0; u < kLmRowGroup; ++u) acc[u] = mulmod_signed(acc[u], f[u], p, pinv);
                    }
                }
                if (col_ok) {
#pragma unroll
                    for (int u = 0; u < kLmRowGroup; ++u)
                        if (rr + u < nrs)
                            A[(int64_t)(rs + rr + u) * lda + c] = (d == 0) ? (1u % F.p) : canonical(acc[u], p);
                }
            }
        }
    }
}

// Generic degree: indices read from global memory (L1-resident) for every row.
__global__ __launch_bounds__(kLmThreads) void load_matrix_any_kernel(
    const uint32_t* __restrict__ bases, int32_t nrows, int32_t nb, int64_t ldbases,
    const int32_t* __restrict__ lind, int32_t ncols, int32_t d, int64_t ldl, FieldConst F,
    uint32_t* __restrict__ A, int64_t lda) {
    const int64_t c = (int64_t)blockIdx.x * kLmThreads + threadIdx.x;
    if (c >= ncols) return;
    const double p = F.dp, pinv = F.pinv;
    for (int32_t r = blockIdx.y; r < nrows; r += gridDim.y) {
        double acc = 1.0;
        for (int32_t t = 0; t < d; ++t) {
            const uint32_t i = (uint32_t)lind[c * ldl + t];
            const double f = i < (uint32_t)nb ? (double)bases[(int64_t)r * ldbases + i] : 0.0;
            acc = t == 0 ? f : mulmod_signed(acc, f, p, pinv);
        }
        A[(int64_t)r * lda + c] = canonical(acc, p);
    }
}

// The number of pivots i < r with pivots[i] - i <= f, i.e. pivots before the
// (f+1)-th free column (pivots[i] - i counts the free columns before pivot i
// and does not decrease).  Binary search; r is small next to the work.
__device__ __forceinline__ int32_t pivots_before_free(const int32_t* piv, int32_t r, int32_t f) {
    int32_t lo = 0, hi = r;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (piv[mid] - mid <= f) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First index i in [0, r) with piv[i] >= j (r when none).
__device__ __forceinline__ int32_t lower_bound_piv(const int32_t* piv, int32_t r, int32_t j) {
    int32_t lo = 0, hi = r;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (piv[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int32_t clamp_rank(const int32_t* rank, int32_t cap) {
    const int32_t r = *rank;
    return r < 0 ? 0 : (r > cap ? cap : r);
}

// K (n x kcols, row-major): column f < n - r is the basis vector of the f-th
// free column c_f: K[c_f][f] = p - 1 (that is -1), K[pivots[s]][f] = R[s][c_f],
// every other entry 0; columns from n - r on are zero.  free_cols (optional,
// n entries) receives c_f, then -1.
__global__ __launch_bounds__(256) void nullspace_kernel(const uint32_t* __restrict__ R, int64_t ldr,
                                                        int32_t n, int32_t rcap,
                                                        const int32_t* __restrict__ rank,
                                                        const int32_t* __restrict__ piv, uint32_t p,
                                                        uint32_t* __restrict__ K, int64_t ldk,
                                                        int32_t kcols, int32_t* __restrict__ free_cols) {
    const int32_t r = clamp_rank(rank, rcap);
    const int32_t f = blockIdx.x * 256 + threadIdx.x;
    const int32_t nfree = n - r;
    const int32_t cf = f < nfree ? f + pivots_before_free(piv, r, f) : -1;
    if (free_cols && blockIdx.y == 0 && f < n) free_cols[f] = cf;
    if (f >= kcols) return;
    for (int32_t j = blockIdx.y; j < n; j += gridDim.y) {
        const int32_t s = lower_bound_piv(piv, r, j);  // uniform over the workgroup
        const bool is_pivot = s < r && piv[s] == j;
        uint32_t v = 0;
        if (f < nfree) {
            if (is_pivot) v = R[(int64_t)s * ldr + cf];
            else v = (j == cf) ? p - 1 : 0u;
        }
        K[(int64_t)j * ldk + f] = v;
    }
}

// C (m x ccols): C[i][s] = A[i][pivots[s]] for s < r, zero for s >= r.
__global__ __launch_bounds__(256) void column_basis_kernel(const uint32_t* __restrict__ A, int64_t lda,
                                                           int32_t m, int32_t n, int32_t rcap,
                                                           const int32_t* __restrict__ rank,
                                                           const int32_t* __restrict__ piv,
                                                           uint32_t* __restrict__ C, int64_t ldc,
                                                           int32_t ccols) {
    const int32_t r = clamp_rank(rank, rcap);
    const int32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= ccols) return;
    int32_t col = s < r ? piv[s] : -1;
    if (col >= n) col = -1;  // never read outside A, whatever the pivots hold
    for (int32_t i = blockIdx.y; i < m; i += gridDim.y)
        C[(int64_t)i * ldc + s] = col >= 0 ? A[(int64_t)i * lda + col] : 0u;
}

}  // namespace

hipError_t launch_load_matrix(const uint32_t* bases, int64_t nrows, int64_t nb, int64_t ldbases,
                              const int32_t* lind, int64_t ncols, int64_t d, int64_t ldl,
                              const FieldConst& F, uint32_t* A, int64_t lda, hipStream_t s) {
    if (nrows == 0 || ncols == 0) return hipSuccess;
    const dim3 grid((unsigned)ceil_div(ncols, kLmThreads),
                    (unsigned)std::min<int64_t>(ceil_div(nrows, kLmRows), 65535));
    const int64_t row_bytes = (nb + 1) * (int64_t)sizeof(double);
    const bool staged = row_bytes <= kLmLdsBytes;
    const int32_t rps = staged ? (int32_t)std::min<int64_t>(kLmRows, kLmLdsBytes / row_bytes) : kLmRows;
    const size_t lds = staged ? (size_t)rps * row_bytes : 0;
    const int32_t nrows32 = (int32_t)nrows, nb32 = (int32_t)nb, ncols32 = (int32_t)ncols,
                  d32 = (int32_t)d;
#define LM_LAUNCH(DM, ST)                                                                         \
    hipLaunchKernelGGL((load_matrix_kernel<DM, ST>), grid, dim3(kLmThreads), lds, s, bases, nrows32, \
                       nb32, ldbases, lind, ncols32, d32, ldl, F, A, lda, rps)
    if (nb == 0 || d > 32) {
        const dim3 grid1(grid.x, (unsigned)std::min<int64_t>(nrows, 65535));
        hipLaunchKernelGGL(load_matrix_any_kernel, grid1, dim3(kLmThreads), 0, s, bases, nrows32, nb32,
                           ldbases, lind, ncols32, d32, ldl, F, A, lda);
    } else if (d <= 8) {
        if (staged) LM_LAUNCH(8, true); else LM_LAUNCH(8, false);
    } else if (d <= 16) {
        if (staged) LM_LAUNCH(16, true); else LM_LAUNCH(16, false);
    } else {
        if (staged) LM_LAUNCH(32, true); else LM_LAUNCH(32, false);
    }
#undef LM_LAUNCH
    return hipGetLastError();
}

hipError_t launch_nullspace(const uint32_t* R, int64_t m, int64_t n, int64_t ldr, const int32_t* rank,
                            const int32_t* pivots, uint32_t p, uint32_t* K, int64_t kcols, int64_t ldk,
                            int32_t* free_cols, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t width = kcols > n ? kcols : n;
    const dim3 grid((unsigned)ceil_div(width, 256), (unsigned)std::min<int64_t>(n, 65535));
    const int32_t rcap = (int32_t)(m < n ? m : n);
    hipLaunchKernelGGL(nullspace_kernel, grid, dim3(256), 0, s, R, ldr, (int32_t)n, rcap, rank, pivots,
                       p, K, ldk, (int32_t)kcols, free_cols);
    return hipGetLastError();
}

hipError_t launch_column_basis(const uint32_t* A, int64_t m, int64_t n, int64_t lda, const int32_t* rank,
                               const int32_t* pivots, uint32_t* C, int64_t ccols, int64_t ldc,
                               hipStream_t s) {
    if (m == 0 || ccols == 0) return hipSuccess;
    const dim3 grid((unsigned)ceil_div(ccols, 256), (unsigned)std::min<int64_t>(m, 65535));
    const int32_t rcap = (int32_t)(m < n ? m : n);
    hipLaunchKernelGGL(column_basis_kernel, grid, dim3(256), 0, s, A, lda, (int32_t)m, (int32_t)n, rcap,
                       rank, pivots, C, ldc, (int32_t)ccols);
    return hipGetLastError();
}

}  // namespace linac
