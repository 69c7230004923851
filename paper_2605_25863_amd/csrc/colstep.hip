// A column-at-a-time elimination engine for two outputs the 32-bit paths do
// not give:
//
//  * 64-bit primes (Sec. 3.2 "Number types": residues stored as uint64 for
//    p up to 2^64 - 1; here 2 <= p < 2^63): Gauss-Jordan RREF and solve, as
//    the paper's loop does it (Sec. 3.2, Fig. 1), with uint64 storage;
//  * the LUP factorisation P A = L U (named as future work in Sec. 6) for
//    32-bit and 64-bit primes: forward elimination that keeps every
//    multiplier, with a fixed pivot rule so that the factors are reproducible.
//
// Per pivot column j two launches:
//  1. search_kernel (one workgroup): records column j of every row (the
//     multipliers of this step, so the update never reads a column it is
//     writing), picks the pivot row -- the first row, in the original row
//     order, that is not a pivot yet and has a non-zero entry (any non-zero
//     entry is a valid pivot over a field, Sec. 3.2 "Pivoting") -- inverts its
//     head and stages the pivot row with Shoup quotients of its entries;
//  2. update_kernel (rows x column chunks): every row that takes part is
//     updated from the staged pivot row.  Gauss-Jordan: all rows but the
//     pivot row, x <- x - f * pn[c] with pn the normalised pivot row, and the
//     pivot row is written normalised.  LUP: only rows that are not pivots
//     yet, x <- x - g * u[c] with g = f / head, and g itself is stored at
//     column j (the L entry); the pivot row stays as it is (a row of U).
// Rows are never moved; pivrow[s] names the s-th pivot row.  Rows whose entry
// in column j is zero are skipped (a wave-uniform test: a wave updates one row
// at a time).
//
// Arithmetic: the update multiplies by the fixed pivot-row entry w with its
// Shoup quotient w' = floor(w 2^B / p) (B = 32 or 64): q = hi(a w'), and
// a w - q p (mod 2^B) lies in [0, 2p), which fits B bits for p < 2^(B-1)
// (V. Shoup; D. Harvey, "Faster arithmetic for number-theoretic transforms",
// 2014).  For 64 bits, w' comes from a 128-by-64-bit long division (once per
// pivot-row entry and step) and the inverse from the extended Euclidean
// algorithm on signed 64-bit values.
#include <algorithm>

#include "internal.h"

namespace linac {

namespace {

constexpr int kCsThreads = 256;
constexpr int kCsRowsPerWave = 8;
constexpr int kCsTileRows = 4 * kCsRowsPerWave;

// ---------------------------------------------------------------------------
// Field operations per word size
// ---------------------------------------------------------------------------
template <typename W>
struct CsField;

template <>
struct CsField<uint32_t> {
    FieldConst F;
    __device__ uint32_t p() const { return F.p; }
    __device__ uint32_t quot(uint32_t w) const { return shoup_quot(w, F); }
    __device__ uint32_t mul_fixed(uint32_t a, uint32_t w, uint32_t wq) const {
        return reduce_2p(shoup_mul_lazy(a, w, wq, F.p), F.p);
    }
    __device__ uint32_t inv(uint32_t a) const { return inv_mod(a, F.p); }
};

__device__ __forceinline__ uint64_t sub_mod64(uint64_t x, uint64_t t, uint64_t p) {
    return x >= t ? x - t : x + (p - t);
}

template <>
struct CsField<uint64_t> {
    uint64_t P;
    __device__ uint64_t p() const { return P; }
    // floor(w 2^64 / p) for w < p < 2^63 by long division: the running
    // remainder stays below p, so doubling it never overflows.
    __device__ uint64_t quot(uint64_t w) const {
        uint64_t rem = w, q = 0;
        for (int i = 0; i < 64; ++i) {
            rem <<= 1;
            q <<= 1;
            if (rem >= P) {
                rem -= P;
                q |= 1;
            }
        }
        return q;
    }
    __device__ uint64_t mul_fixed(uint64_t a, uint64_t w, uint64_t wq) const {
        const uint64_t q = __umul64hi(a, wq);
        const uint64_t r = a * w - q * P;  // in [0, 2p), below 2^64 for p < 2^63
        return r >= P ? r - P : r;
    }
    __device__ uint64_t inv(uint64_t a) const {
        int64_t t = 0, nt = 1;
        uint64_t r = P, nr = a;
        while (nr != 0) {
            const uint64_t q = r / nr;
            const int64_t tmp = t - (int64_t)q * nt;  // |t| <= p / 2 < 2^62 throughout
            t = nt;
            nt = tmp;
            const uint64_t rr = r - q * nr;
            r = nr;
            nr = rr;
        }
        return t < 0 ? (uint64_t)(t + (int64_t)P) : (uint64_t)t;
    }
};

__device__ __forceinline__ uint32_t sub_any(uint32_t x, uint32_t t, uint32_t p) { return sub_mod(x, t, p); }
__device__ __forceinline__ uint64_t sub_any(uint64_t x, uint64_t t, uint64_t p) { return sub_mod64(x, t, p); }

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
template <typename W>
struct CsArgs {
    W* M;          // m x ld working copy
    int64_t ld;
    int32_t m, ncols, nsearch;  // right-hand sides: ncols - nsearch
    W* fcol;       // column j of every row at the start of step j
    W* pn;         // staged pivot row (normalised for Gauss-Jordan)
    W* pnq;        // Shoup quotients of pn
    int32_t* is_piv;   // -1, or the step at which the row became a pivot
    int32_t* pivrow;   // s-th pivot row
    int32_t* pivcol;   // s-th pivot column
    int32_t* state;    // [0] rank, [1] this step's pivot row or -1
    W* inv;            // [0] inverse of this step's head, [1] its Shoup quotient
    uint32_t* incons;  // per right-hand side: 1 once a residual is non-zero
};

template <typename W>
__global__ __launch_bounds__(kCsThreads) void cs_init_kernel(CsArgs<W> a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.m;
         i += (int64_t)gridDim.x * blockDim.x)
        a.is_piv[i] = -1;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < a.ncols - a.nsearch;
         t += (int64_t)gridDim.x * blockDim.x)
        a.incons[t] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 2) a.state[threadIdx.x] = threadIdx.x == 0 ? 0 : -1;
}

template <typename W>
__global__ __launch_bounds__(kCsThreads) void cs_pack_kernel(CsArgs<W> a, const W* A, int64_t lda,
                                                              const W* B, int64_t ldb, int32_t n) {
    const int64_t total = (int64_t)a.m * a.ld;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / a.ld, c = i - r * a.ld;
        W v = 0;
        if (c < n) v = A[r * lda + c];
        else if (c < a.ncols) v = B[r * ldb + (c - n)];
        a.M[i] = v;
    }
}

template <typename W, bool kLU>
__global__ __launch_bounds__(1024) void cs_search_kernel(CsArgs<W> a, CsField<W> f, int32_t j) {
    __shared__ int32_t s_best[16];
    __shared__ int32_t s_piv;
    const int tid = threadIdx.x;
    int32_t best = INT32_MAX;
    for (int32_t r = tid; r < a.m; r += 1024) {
        const W v = a.M[(int64_t)r * a.ld + j];
        a.fcol[r] = v;
        if (v != 0 && a.is_piv[r] < 0 && r < best) best = r;
    }
    for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
    if ((tid & 63) == 0) s_best[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
        int32_t b = INT32_MAX;
        for (int w = 0; w < 16; ++w) b = min(b, s_best[w]);
        const int32_t rank = a.state[0];
        if (b == INT32_MAX || rank >= a.m) {
            s_piv = -1;
            a.state[1] = -1;
        } else {
            s_piv = b;
            a.state[1] = b;
            a.is_piv[b] = rank;
            a.pivrow[rank] = b;
            a.pivcol[rank] = j;
            a.state[0] = rank + 1;
            const W iv = f.inv(a.M[(int64_t)b * a.ld + j]);
            a.inv[0] = iv;
            a.inv[1] = f.quot(iv);
        }
    }
    __syncthreads();
    const int32_t piv = s_piv;
    if (piv < 0) return;
    const W iv = a.inv[0], ivq = a.inv[1];
    const W* prow = a.M + (int64_t)piv * a.ld;
    for (int32_t c = j + tid; c < a.ncols; c += 1024) {
        W v = prow[c];
        if (!kLU) v = f.mul_fixed(v, iv, ivq);  // Gauss-Jordan: the normalised pivot row
        a.pn[c] = v;
        a.pnq[c] = f.quot(v);
    }
}

// Rows [blockIdx.x * 32, +32) x columns [cbase + blockIdx.y * chunk, +chunk),
// chunk = 64 lanes x kVec words (one 16-byte access per lane and row).
template <typename W, bool kLU>
__global__ __launch_bounds__(kCsThreads) void cs_update_kernel(CsArgs<W> a, CsField<W> f, int32_t j,
                                                                int64_t cbase) {
    constexpr int kVec = 16 / (int)sizeof(W);
    const int32_t piv = a.state[1];
    if (piv < 0) return;  // free column: nothing to do
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t c0 = cbase + (int64_t)blockIdx.y * 64 * kVec + lane * kVec;
    const W p = f.p();
    W pn[kVec], pnq[kVec];
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
        const int64_t c = c0 + e;
        const bool live = c > j && c < a.ncols;
        pn[e] = live ? a.pn[c] : (W)0;
        pnq[e] = live ? a.pnq[c] : (W)0;
    }
    const W iv = a.inv[0], ivq = a.inv[1];
    const int32_t r0 = blockIdx.x * kCsTileRows + wave * kCsRowsPerWave;
    for (int rr = 0; rr < kCsRowsPerWave; ++rr) {
        const int32_t r = r0 + rr;
        if (r >= a.m) break;
        W* row = a.M + (int64_t)r * a.ld;
        if (r == piv) {
            if (!kLU) {  // write the normalised pivot row (column j becomes 1)
#pragma unroll
                for (int e = 0; e < kVec; ++e) {
                    const int64_t c = c0 + e;
                    if (c == j) row[c] = 1;
                    else if (c > j && c < a.ncols) row[c] = pn[e];
                }
            }
            continue;
        }
        if (kLU && a.is_piv[r] >= 0) continue;  // LUP: rows of U stay
        const W fr = a.fcol[r];
        if (fr == 0) continue;
        const W g = kLU ? f.mul_fixed(fr, iv, ivq) : fr;  // LUP multiplier f / head
        if (c0 + kVec <= a.ld) {
            W x[kVec];
            __builtin_memcpy(x, row + c0, 16);
#pragma unroll
            for (int e = 0; e < kVec; ++e) {
                const int64_t c = c0 + e;
                if (c > j && c < a.ncols) x[e] = sub_any(x[e], f.mul_fixed(g, pn[e], pnq[e]), p);
                else if (c == j) x[e] = kLU ? g : (W)0;
            }
            __builtin_memcpy(row + c0, x, 16);
        }
    }
}

// Gauss-Jordan outputs.  RREF: row s of A is pivot row s, rows from the rank
// on are zero (only the first n columns).
template <typename W>
__global__ __launch_bounds__(kCsThreads) void cs_rref_out_kernel(CsArgs<W> a, W* A, int64_t lda,
                                                                  int32_t n, int32_t* rank,
                                                                  int32_t* pivots, int32_t pcount) {
    const int32_t r = a.state[0];
    const int64_t total = (int64_t)a.m * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / n, c = i - s * n;
        A[s * lda + c] = s < r ? a.M[(int64_t)a.pivrow[s] * a.ld + c] : (W)0;
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pcount;
         g += (int64_t)gridDim.x * blockDim.x)
        pivots[g] = g < r ? a.pivcol[g] : -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) *rank = r;
}

// Solve: a right-hand side is inconsistent iff some row without a pivot keeps a
// non-zero entry in it (Sec. 5.2).
template <typename W>
__global__ __launch_bounds__(kCsThreads) void cs_incons_kernel(CsArgs<W> a, int32_t n, int32_t k) {
    const int64_t total = (int64_t)a.m * k;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / k, t = i - r * k;
        if (a.is_piv[r] < 0 && a.M[r * a.ld + n + t] != 0) a.incons[t] = 1;
    }
}

template <typename W>
__global__ __launch_bounds__(kCsThreads) void cs_solve_out_kernel(CsArgs<W> a, int32_t n, int32_t k,
                                                                   W* X, int64_t ldx, int32_t* rank,
                                                                   int32_t* pivots, int32_t pcount,
                                                                   uint8_t* consistent) {
    const int32_t r = a.state[0];
    const int64_t total = (int64_t)n * k;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / k, t = i - c * k;
        W v = 0;
        if (!a.incons[t]) {
            // the pivot of column c, if any: pivcol is ascending over [0, r)
            int32_t lo = 0, hi = r;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (a.pivcol[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            if (lo < r && a.pivcol[lo] == c) v = a.M[(int64_t)a.pivrow[lo] * a.ld + n + t];
        }
        X[c * ldx + t] = v;
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pcount;
         g += (int64_t)gridDim.x * blockDim.x)
        pivots[g] = g < r ? a.pivcol[g] : -1;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < k;
         g += (int64_t)gridDim.x * blockDim.x)
        consistent[g] = a.incons[g] ? 0 : 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) *rank = r;
}

// LUP outputs: perm (the pivot rows in pivot order, then the other rows in
// their original order) and the packed factors, row i of A = working row
// perm[i]: L's entries sit at the pivot columns left of row i's own pivot,
// U's entries everywhere else.
template <typename W>
__global__ __launch_bounds__(1024) void cs_perm_kernel(CsArgs<W> a, int32_t* perm) {
    // the non-pivot rows: position rank + (number of non-pivot rows before them)
    __shared__ int32_t s_count[1024];
    const int32_t r = a.state[0];
    const int tid = threadIdx.x;
    const int32_t per = (a.m + 1023) / 1024;
    const int32_t lo = min(a.m, tid * per), hi = min(a.m, lo + per);
    int32_t cnt = 0;
    for (int32_t q = lo; q < hi; ++q) cnt += a.is_piv[q] < 0;
    s_count[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
        const int32_t v = tid >= off ? s_count[tid - off] : 0;
        __syncthreads();
        s_count[tid] += v;
        __syncthreads();
    }
    int32_t pos = r + s_count[tid] - cnt;
    for (int32_t q = lo; q < hi; ++q)
        if (a.is_piv[q] < 0) perm[pos++] = q;
    for (int32_t s = tid; s < r; s += 1024) perm[s] = a.pivrow[s];
}

template <typename W>
__global__ __launch_bounds__(kCsThreads) void cs_lu_out_kernel(CsArgs<W> a, W* A, int64_t lda, int32_t n,
                                                                const int32_t* perm, int32_t* rank,
                                                                int32_t* pivots, int32_t pcount) {
    const int64_t total = (int64_t)a.m * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / n, c = i - s * n;
        A[s * lda + c] = a.M[(int64_t)perm[s] * a.ld + c];
    }
    const int32_t r = a.state[0];
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pcount;
         g += (int64_t)gridDim.x * blockDim.x)
        pivots[g] = g < r ? a.pivcol[g] : -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) *rank = r;
}

template <typename W>
__global__ void cs_range_kernel(const W* M, int64_t rows, int64_t cols, int64_t ld, W p, uint32_t* flag) {
    const int64_t total = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols, c = i - r * cols;
        if (M[r * ld + c] >= p) *flag = 1;
    }
}

unsigned grid_for(int64_t total) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, kCsThreads), 4096));
}

template <typename W>
size_t cs_carve(void* ws, int64_t m, int64_t n, int64_t k, CsArgs<W>& a) {
    Carver c(ws);
    a.ld = round_up(n + k > 0 ? n + k : 1, 256 / (int64_t)sizeof(W));  // 256-byte rows
    a.M = c.take<W>(m * a.ld);
    a.fcol = c.take<W>(m > 0 ? m : 1);
    a.pn = c.take<W>(a.ld);
    a.pnq = c.take<W>(a.ld);
    a.is_piv = c.take<int32_t>(m > 0 ? m : 1);
    a.pivrow = c.take<int32_t>(n > 0 ? n : 1);
    a.pivcol = c.take<int32_t>(n > 0 ? n : 1);
    a.state = c.take<int32_t>(8);
    a.inv = c.take<W>(2);
    a.incons = c.take<uint32_t>(k > 0 ? k : 1);
    a.m = (int32_t)m;
    a.ncols = (int32_t)(n + k);
    a.nsearch = (int32_t)n;
    return c.off + 256;
}

template <typename W>
CsField<W> make_cs_field(W p);
template <>
CsField<uint32_t> make_cs_field<uint32_t>(uint32_t p) {
    return CsField<uint32_t>{make_field(p)};
}
template <>
CsField<uint64_t> make_cs_field<uint64_t>(uint64_t p) {
    return CsField<uint64_t>{p};
}

// The elimination loop over the n searched columns (stream-ordered, no host
// synchronisation; the host stays blind as in the paper).
template <typename W, bool kLU>
hipError_t cs_eliminate(const CsArgs<W>& a, const CsField<W>& f, hipStream_t s) {
    constexpr int kVec = 16 / (int)sizeof(W);
    constexpr int64_t kChunk = 64 * kVec;
    const unsigned tiles = (unsigned)ceil_div(a.m, kCsTileRows);
    const int32_t steps = a.nsearch;
    for (int32_t j = 0; j < steps; ++j) {
        hipLaunchKernelGGL((cs_search_kernel<W, kLU>), dim3(1), dim3(1024), 0, s, a, f, j);
        const int64_t cbase = j / kVec * kVec;
        const unsigned chunks = (unsigned)ceil_div(a.ncols - cbase, kChunk);
        hipLaunchKernelGGL((cs_update_kernel<W, kLU>), dim3(tiles, chunks), dim3(kCsThreads), 0, s, a,
                           f, j, cbase);
    }
    return hipGetLastError();
}

template <typename W>
hipError_t cs_prepare(CsArgs<W>& a, const W* A, int64_t lda, const W* B, int64_t ldb, int32_t n,
                      hipStream_t s) {
    hipLaunchKernelGGL((cs_init_kernel<W>), dim3(grid_for(std::max(a.m, a.ncols - a.nsearch))),
                       dim3(kCsThreads), 0, s, a);
    if (a.m > 0)
        hipLaunchKernelGGL((cs_pack_kernel<W>), dim3(grid_for((int64_t)a.m * a.ld)), dim3(kCsThreads), 0,
                           s, a, A, lda, B, ldb, n);
    return hipGetLastError();
}

}  // namespace

size_t colstep_workspace(int64_t m, int64_t n, int64_t k, bool wide) {
    if (wide) {
        CsArgs<uint64_t> a;
        return cs_carve<uint64_t>(nullptr, m, n, k, a);
    }
    CsArgs<uint32_t> a;
    return cs_carve<uint32_t>(nullptr, m, n, k, a);
}

template <typename W>
hipError_t colstep_range(const W* M, int64_t rows, int64_t cols, int64_t ld, W p, uint32_t* flag,
                         hipStream_t s) {
    if (rows * cols == 0) return hipSuccess;
    hipLaunchKernelGGL((cs_range_kernel<W>), dim3(grid_for(rows * cols)), dim3(kCsThreads), 0, s, M, rows,
                       cols, ld, p, flag);
    return hipGetLastError();
}

template <typename W>
hipError_t colstep_rref(W* A, int64_t m, int64_t n, int64_t lda, W p, int32_t* rank, int32_t* pivots,
                        void* ws, hipStream_t s) {
    CsArgs<W> a;
    cs_carve<W>(ws, m, n, 0, a);
    const CsField<W> f = make_cs_field<W>(p);
    hipError_t e = cs_prepare<W>(a, A, lda, nullptr, 1, (int32_t)n, s);
    if (e == hipSuccess && m > 0) e = cs_eliminate<W, false>(a, f, s);
    const int32_t pc = (int32_t)std::min(m, n);
    if (e == hipSuccess) {
        hipLaunchKernelGGL((cs_rref_out_kernel<W>), dim3(grid_for(std::max<int64_t>(m * n, pc + 1))),
                           dim3(kCsThreads), 0, s, a, A, lda, (int32_t)n, rank, pivots, pc);
        e = hipGetLastError();
    }
    return e;
}

template <typename W>
hipError_t colstep_solve(const W* A, int64_t m, int64_t n, int64_t lda, const W* B, int64_t k,
                         int64_t ldb, W p, W* X, int64_t ldx, int32_t* rank, int32_t* pivots,
                         uint8_t* consistent, void* ws, hipStream_t s) {
    CsArgs<W> a;
    cs_carve<W>(ws, m, n, k, a);
    const CsField<W> f = make_cs_field<W>(p);
    hipError_t e = cs_prepare<W>(a, A, lda, B, ldb, (int32_t)n, s);
    if (e == hipSuccess && m > 0) e = cs_eliminate<W, false>(a, f, s);
    if (e == hipSuccess && m * k > 0) {
        hipLaunchKernelGGL((cs_incons_kernel<W>), dim3(grid_for(m * k)), dim3(kCsThreads), 0, s, a,
                           (int32_t)n, (int32_t)k);
        e = hipGetLastError();
    }
    const int32_t pc = (int32_t)std::min(m, n);
    if (e == hipSuccess) {
        const int64_t work = std::max<int64_t>(std::max<int64_t>(n * k, pc + 1), k + 1);
        hipLaunchKernelGGL((cs_solve_out_kernel<W>), dim3(grid_for(work)), dim3(kCsThreads), 0, s, a,
                           (int32_t)n, (int32_t)k, X, ldx, rank, pivots, pc, consistent);
        e = hipGetLastError();
    }
    return e;
}

template <typename W>
hipError_t colstep_lup(W* A, int64_t m, int64_t n, int64_t lda, W p, int32_t* perm, int32_t* rank,
                       int32_t* pivots, void* ws, hipStream_t s) {
    CsArgs<W> a;
    cs_carve<W>(ws, m, n, 0, a);
    const CsField<W> f = make_cs_field<W>(p);
    hipError_t e = cs_prepare<W>(a, A, lda, nullptr, 1, (int32_t)n, s);
    if (e == hipSuccess && m > 0) e = cs_eliminate<W, true>(a, f, s);
    const int32_t pc = (int32_t)std::min(m, n);
    if (e == hipSuccess && m > 0) {
        hipLaunchKernelGGL((cs_perm_kernel<W>), dim3(1), dim3(1024), 0, s, a, perm);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL((cs_lu_out_kernel<W>), dim3(grid_for(std::max<int64_t>(m * n, pc + 1))),
                           dim3(kCsThreads), 0, s, a, A, lda, (int32_t)n, (const int32_t*)perm, rank,
                           pivots, pc);
        e = hipGetLastError();
    }
    return e;
}

template hipError_t colstep_range<uint32_t>(const uint32_t*, int64_t, int64_t, int64_t, uint32_t,
                                            uint32_t*, hipStream_t);
template hipError_t colstep_range<uint64_t>(const uint64_t*, int64_t, int64_t, int64_t, uint64_t,
                                            uint32_t*, hipStream_t);
template hipError_t colstep_rref<uint64_t>(uint64_t*, int64_t, int64_t, int64_t, uint64_t, int32_t*,
                                           int32_t*, void*, hipStream_t);
template hipError_t colstep_solve<uint64_t>(const uint64_t*, int64_t, int64_t, int64_t, const uint64_t*,
                                            int64_t, int64_t, uint64_t, uint64_t*, int64_t, int32_t*,
                                            int32_t*, uint8_t*, void*, hipStream_t);
template hipError_t colstep_lup<uint32_t>(uint32_t*, int64_t, int64_t, int64_t, uint32_t, int32_t*,
                                          int32_t*, int32_t*, void*, hipStream_t);
template hipError_t colstep_lup<uint64_t>(uint64_t*, int64_t, int64_t, int64_t, uint64_t, int32_t*,
                                          int32_t*, int32_t*, void*, hipStream_t);

}  // namespace linac
