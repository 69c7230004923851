// Plain Gauss-Jordan elimination over F_p: one fused launch per pivot column.
//
// The paper's GPU loop (Sec. 3.2, "Looping" to "Increment counters", Fig. 1)
// runs about seven kernels per column: a two-level argmax pivot search, a row
// swap, a zero test of the head, a conditional rescale, the row update
// ("RowReduce", over 90 % of the time, Sec. 4.1.1) and a counter increment.
// Over F_p any non-zero entry is a valid pivot (Sec. 3.2, "Pivoting"), which
// lets this design fold all of them into a single kernel per column:
//
//  * Look-ahead pivot search.  Step j writes column j+1 anyway, so the blocks
//    that own it also record its values (fcol, with bit 31 marking rows that
//    are already pivots) and post the smallest non-pivot row with a non-zero
//    entry, packed with the inverse of that entry, through one 64-bit
//    atomicMin into slot[j+1].  Step j+1 reads the slot at launch: the pivot
//    row and its inverse are known with no extra launch and no host round trip
//    (the host stays blind, as in the paper).
//  * Virtual row swap.  Rows never move.  The pivot row q of step j is only
//    read during step j, so every block can form its normalised values
//    inv * W[q][c] on the fly; writing it back is deferred to step j+1, which
//    rescales row q before its own update (the "pending" row).  The final
//    gather writes rows in pivot order.
//  * The row update x <- x - f * pn[c] uses Shoup's precomputed-quotient
//    multiplication with the normalised pivot entry pn[c] as the fixed operand
//    (three 32-bit multiplies), or the Mersenne fold for p = 2^31 - 1.  Rows
//    with f = 0 are skipped (Sec. 3.4, conditional skipping).
//
// Launch shape: 256 threads (4 wave64); a block updates a 32-row x 256-column
// tile; each lane owns 4 consecutive columns (one 128-bit access per row, the
// paper's uint4 access of Sec. 3.4) and 8 rows, so 8 independent 128-bit loads
// are in flight per lane.  Column chunks start at j rounded down to 64, and
// grid.x runs over row tiles so the blocks of the chunk holding column j+1
// (the look-ahead) are dispatched first.
#include "internal.h"

namespace linac {

namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerWave = 8;
constexpr int kTileRows = 4 * kRowsPerWave;
constexpr int kChunkCols = 256;

template <bool kMersenne>
__device__ __forceinline__ uint32_t mul_mod_t(uint32_t a, uint32_t b, const FieldConst& F) {
    if constexpr (kMersenne) {
        return mersenne_reduce((uint64_t)a * b);
    } else {
        return mul_mod(a, b, F);
    }
}

__device__ __forceinline__ uint32_t pick(const uint4& v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

// Block-wide minimum of per-wave pivot candidates (row, head value), posted to
// `slot` as (row << 32) | inverse of the head: the smallest row wins.  The
// inverse is skipped when a smaller row has already been posted.
__device__ void block_candidate(int wave, int lane, int src_lane, int best, uint32_t bestv,
                                int* s_row, uint32_t* s_val, unsigned long long* slot,
                                uint32_t p) {
    best = __shfl(best, src_lane);
    bestv = __shfl(bestv, src_lane);
    if (lane == 0) {
        s_row[wave] = best;
        s_val[wave] = bestv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = s_row[0];
        uint32_t v = s_val[0];
        for (int w = 1; w < 4; ++w)
            if (s_row[w] < r) {
                r = s_row[w];
                v = s_val[w];
            }
        if (r != INT32_MAX) {
            const unsigned long long cur =
                __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((cur >> 32) > (unsigned long long)r)
                atomicMin(slot, ((unsigned long long)r << 32) | inv_mod(v, p));
        }
    }
}

__global__ void plain_init_kernel(PlainArgs a, int32_t k) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i <= a.nsearch; i += stride) a.slots[i] = kNoPivot;
    for (int64_t i = tid; i < a.nsearch; i += stride) a.colpiv[i] = -1;
    for (int64_t i = tid; i < a.m; i += stride) {
        a.is_piv[i] = 0;
        a.rowcol[i] = -1;
    }
    for (int64_t i = tid; i < k; i += stride) a.incons[i] = 0;
    if (tid < 8) a.state[tid] = 0;
}

// Copy [A | B] into the padded working matrix W and run the look-ahead for
// column 0.
__global__ __launch_bounds__(kThreads) void plain_pack_kernel(PlainArgs a, const uint32_t* A,
                                                              int64_t lda, const uint32_t* B,
                                                              int64_t ldb, int32_t n) {
    __shared__ int s_row[4];
    __shared__ uint32_t s_val[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)blockIdx.y * kChunkCols + lane * 4;
    const int row0 = blockIdx.x * kTileRows + wave * kRowsPerWave;
    int best = INT32_MAX;
    uint32_t bestv = 0;
    for (int rr = 0; rr < kRowsPerWave; ++rr) {
        int r = row0 + rr;
        if (r >= a.m || c0 >= a.ld) continue;
        uint32_t v[4];
        for (int e = 0; e < 4; ++e) {
            int64_t c = c0 + e;
            v[e] = c < n ? A[(int64_t)r * lda + c]
                         : (c < a.ncols ? B[(int64_t)r * ldb + (c - n)] : 0u);
        }
        *(uint4*)(a.W + (int64_t)r * a.ld + c0) = make_uint4(v[0], v[1], v[2], v[3]);
        if (blockIdx.y == 0 && lane == 0 && a.nsearch > 0) {
            a.fcol[0][r] = v[0];
            if (v[0] != 0 && r < best) {
                best = r;
                bestv = v[0];
            }
        }
    }
    if (blockIdx.y == 0 && a.nsearch > 0)
        block_candidate(wave, lane, 0, best, bestv, s_row, s_val, &a.slots[0], a.F.p);
}

// One Gauss-Jordan step for local pivot column j (see the file comment).  Only
// local columns below ncols_eff are touched (the blocked path's transform block
// is still zero beyond the current step).
template <bool kMersenne>
__global__ __launch_bounds__(kThreads) void plain_step_kernel(PlainArgs a, int32_t j,
                                                              int32_t ncols_eff) {
    __shared__ int s_row[4];
    __shared__ uint32_t s_val[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const FieldConst F = a.F;
    const uint32_t p = F.p;
    const int jg = a.coloff + j;

    const unsigned long long sj = a.slots[jg];
    const unsigned long long sprev = j > 0 ? a.slots[jg - 1] : kNoPivot;
    const bool have_piv = sj != kNoPivot;
    const int q = have_piv ? (int)(sj >> 32) : -1;
    const uint32_t inv = (uint32_t)sj;
    const int qpend = sprev != kNoPivot ? (int)(sprev >> 32) : -1;
    const uint32_t spend = (uint32_t)sprev;
    const bool lookahead = blockIdx.y == 0 && j + 1 < a.nsearch;

    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && have_piv) {
        int s = a.state[0];
        a.pivrow[s] = q;
        a.pivcol[s] = jg;
        a.colpiv[jg] = s;
        a.rowcol[q] = jg;
        a.is_piv[q] = 1;
        a.state[0] = s + 1;
    }
    if (!have_piv && qpend < 0 && !lookahead) return;

    const int cbase = j & ~63;
    const int64_t c0 = cbase + (int64_t)blockIdx.y * kChunkCols + lane * 4;
    const bool lane_on = c0 < a.ld;
    const int64_t ecol = a.einject >= 0 ? (int64_t)a.einject + j : -1;

    // normalised pivot row entries for this lane's columns, and their quotients
    uint32_t pn[4] = {0u, 0u, 0u, 0u}, pq[4] = {0u, 0u, 0u, 0u};
    if (have_piv && lane_on) {
        uint4 v = *(const uint4*)(a.W + (int64_t)q * a.ld + c0);
        uint32_t raw[4] = {v.x, v.y, v.z, v.w};
        if (ecol >= c0 && ecol < c0 + 4) raw[ecol - c0] = 1u;  // the pivot row's own E entry
        for (int e = 0; e < 4; ++e) pn[e] = mul_mod_t<kMersenne>(raw[e], inv, F);
        if constexpr (!kMersenne) {
            for (int e = 0; e < 4; ++e) pq[e] = shoup_quot(pn[e], F);
        }
    }

    const uint32_t* fcur = a.fcol[j & 1];
    const int row0 = blockIdx.x * kTileRows + wave * kRowsPerWave;
    // the pivot row is read-only during this step; its E entry 1 is stored for the next
    if (have_piv && ecol >= c0 && ecol < c0 + 4 && q >= row0 && q < row0 + kRowsPerWave)
        a.W[(int64_t)q * a.ld + ecol] = 1u;
    const bool col_on = lane_on && c0 < ncols_eff;
    uint4 x[kRowsPerWave];
    uint32_t f[kRowsPerWave];
    bool act[kRowsPerWave];
    uint32_t pivmask = 0;  // bit rr: row row0 + rr is already a pivot row
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) {
        const int r = row0 + rr;
        const bool valid = r < a.m;
        const uint32_t fr = valid ? fcur[r] : 0u;
        pivmask |= (fr >> 31) << rr;
        f[rr] = fr & 0x7fffffffu;
        const bool pend = r == qpend;
        bool on = valid && r != q;
        if (blockIdx.y != 0) on = on && (pend || (have_piv && f[rr] != 0));
        act[rr] = on;
        if (!have_piv) f[rr] = 0;
        if (on && col_on) x[rr] = *(const uint4*)(a.W + (int64_t)r * a.ld + c0);
        else x[rr] = make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) {
        if (!act[rr] || !col_on) continue;
        const int r = row0 + rr;
        uint32_t v[4] = {x[rr].x, x[rr].y, x[rr].z, x[rr].w};
        if (r == qpend) {
            for (int e = 0; e < 4; ++e) v[e] = mul_mod_t<kMersenne>(v[e], spend, F);
        }
        const uint32_t fr = f[rr];
        if (fr == 0 && r != qpend) continue;  // unchanged row (loaded for the look-ahead)
        {
            for (int e = 0; e < 4; ++e) {
                uint32_t t;
                if constexpr (kMersenne) {
                    t = mersenne_reduce((uint64_t)fr * pn[e]);
                } else {
                    t = reduce_2p(shoup_mul_lazy(fr, pn[e], pq[e], p), p);
                }
                v[e] = sub_mod(v[e], t, p);
            }
        }
        x[rr] = make_uint4(v[0], v[1], v[2], v[3]);
        *(uint4*)(a.W + (int64_t)r * a.ld + c0) = x[rr];
    }

    if (lookahead) {
        const int jn = j + 1;
        const int src_lane = (jn - cbase) >> 2;
        const int e = (jn - cbase) & 3;
        uint32_t* fnext = a.fcol[jn & 1];
        int best = INT32_MAX;
        uint32_t bestv = 0;
        if (lane == src_lane) {
            for (int rr = 0; rr < kRowsPerWave; ++rr) {
                const int r = row0 + rr;
                if (r >= a.m) break;
                const uint32_t v = r == q ? pick(make_uint4(pn[0], pn[1], pn[2], pn[3]), e)
                                          : pick(x[rr], e);
                const bool piv = ((pivmask >> rr) & 1u) || r == q;
                fnext[r] = v | ((uint32_t)piv << 31);
                if (v != 0 && !piv && r < best) {
                    best = r;
                    bestv = v;
                }
            }
        }
        block_candidate(wave, lane, src_lane, best, bestv, s_row, s_val, &a.slots[a.coloff + jn],
                        p);
    }
}

// Residual test of the right-hand sides: a non-pivot row with a non-zero entry
// in B's part makes that column inconsistent (Sec. 5.2).  One thread per
// (row, rhs).
__global__ void plain_incons_kernel(PlainArgs a, int32_t n, int32_t k) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.m * k) return;
    int r = (int)(idx / k), t = (int)(idx % k);
    if (a.is_piv[r]) return;
    if (a.W[(int64_t)r * a.ld + n + t] != 0) a.incons[t] = 1;
}

// Logical value of working-matrix entry (r, c): the last pivot row may still
// carry its deferred normalisation.
__device__ __forceinline__ uint32_t logical(const PlainArgs& a, int r, int64_t c, int qlast,
                                            uint32_t slast) {
    uint32_t v = a.W[(int64_t)r * a.ld + c];
    return r == qlast ? mul_mod(v, slast, a.F) : v;
}

__device__ __forceinline__ void last_pending(const PlainArgs& a, int& qlast, uint32_t& slast) {
    qlast = -1;
    slast = 1;
    if (a.nsearch > 0 && !a.resolved) {
        unsigned long long s = a.slots[a.nsearch - 1];
        if (s != kNoPivot) {
            qlast = (int)(s >> 32);
            slast = (uint32_t)s;
        }
    }
}

// X, consistency, rank and pivot outputs of a solve.
__global__ void plain_outputs_solve_kernel(PlainArgs a, int32_t n, int32_t k, uint32_t* X,
                                           int64_t ldx, int32_t* rank, int32_t* pivots,
                                           uint8_t* consistent) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int qlast;
    uint32_t slast;
    last_pending(a, qlast, slast);
    const int r = a.state[0];
    if (idx < (int64_t)n * k) {
        int v = (int)(idx / k), t = (int)(idx % k);
        int s = a.colpiv[v];
        uint32_t val = 0;
        if (s >= 0 && a.incons[t] == 0) val = logical(a, a.pivrow[s], (int64_t)n + t, qlast, slast);
        X[(int64_t)v * ldx + t] = val;
    }
    if (idx < k) consistent[idx] = a.incons[idx] ? 0 : 1;
    int mn = min(a.m, n);
    if (idx < mn) pivots[idx] = idx < r ? a.pivcol[idx] : -1;
    if (idx == 0) *rank = r;
}

// Gather the RREF into A (row s = pivot row s, zero rows below the rank).  Pivot
// columns are written as unit vectors.  One block per output row.
__global__ __launch_bounds__(kThreads) void plain_outputs_rref_kernel(PlainArgs a, uint32_t* A,
                                                                      int64_t lda, int32_t* rank,
                                                                      int32_t* pivots) {
    int qlast;
    uint32_t slast;
    last_pending(a, qlast, slast);
    const int r = a.state[0];
    const int n = a.nsearch;
    const int s = blockIdx.x;
    if (s < a.m) {
        const int prow = s < r ? a.pivrow[s] : 0;
        for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
            uint32_t val = 0;
            if (s < r) {
                int cp = a.colpiv[c];
                val = cp >= 0 ? (cp == s ? 1u : 0u) : logical(a, prow, c, qlast, slast);
            }
            A[(int64_t)s * lda + c] = val;
        }
    }
    if (s == 0) {
        int mn = min(a.m, n);
        for (int i = threadIdx.x; i < mn; i += blockDim.x) pivots[i] = i < r ? a.pivcol[i] : -1;
        if (threadIdx.x == 0) *rank = r;
    }
}

__global__ void range_check_kernel(const uint32_t* M, int64_t rows, int64_t cols, int64_t ld,
                                   uint32_t p, uint32_t* flag) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < rows * cols; i += stride) {
        if (M[(i / cols) * ld + i % cols] >= p) *flag = 1;
    }
}

}  // namespace

size_t plain_workspace(int64_t m, int64_t n, int64_t k) {
    PlainArgs a;
    Carver c(nullptr);
    int64_t ld = round_up(n + k > 0 ? n + k : 1, 64);
    c.take<uint32_t>(m * ld);
    c.take<uint32_t>(m);
    c.take<uint32_t>(m);
    c.take<uint32_t>(m);
    c.take<unsigned long long>(n + 1);
    c.take<int32_t>(n);
    c.take<int32_t>(n);
    c.take<int32_t>(n);
    c.take<int32_t>(m);
    c.take<int32_t>(8);
    c.take<uint32_t>(k > 0 ? k : 1);
    (void)a;
    return c.off + 256;
}

void plain_carve(void* ws, int64_t m, int64_t n, int64_t k, PlainArgs& a) {
    Carver c(ws);
    a.ld = round_up(n + k > 0 ? n + k : 1, 64);
    a.W = c.take<uint32_t>(m * a.ld);
    a.fcol[0] = c.take<uint32_t>(m);
    a.fcol[1] = c.take<uint32_t>(m);
    a.is_piv = c.take<uint32_t>(m);
    a.slots = c.take<unsigned long long>(n + 1);
    a.pivrow = c.take<int32_t>(n);
    a.pivcol = c.take<int32_t>(n);
    a.colpiv = c.take<int32_t>(n);
    a.rowcol = c.take<int32_t>(m);
    a.state = c.take<int32_t>(8);
    a.incons = c.take<uint32_t>(k > 0 ? k : 1);
    a.m = (int32_t)m;
    a.ncols = (int32_t)(n + k);
    a.nsearch = (int32_t)n;
    a.coloff = 0;
    a.einject = -1;
    a.resolved = 0;
}

hipError_t plain_prepare(const PlainArgs& a, const uint32_t* A, int64_t lda, const uint32_t* B,
                         int64_t ldb, int32_t n, int32_t k, hipStream_t s) {
    int64_t work = a.m > a.nsearch + 1 ? a.m : a.nsearch + 1;
    int blocks = (int)(ceil_div(work, 256) < 1024 ? ceil_div(work, 256) : 1024);
    hipLaunchKernelGGL(plain_init_kernel, dim3(blocks), dim3(256), 0, s, a, k);
    if (a.m > 0) {
        dim3 grid((unsigned)ceil_div(a.m, kTileRows), (unsigned)ceil_div(a.ld, kChunkCols));
        hipLaunchKernelGGL(plain_pack_kernel, grid, dim3(kThreads), 0, s, a, A, lda, B, ldb, n);
    }
    return hipGetLastError();
}

hipError_t launch_gj_step(const PlainArgs& a, int32_t j, int32_t ncols_eff, hipStream_t s) {
    const unsigned tiles = (unsigned)ceil_div(a.m, kTileRows);
    const int64_t cbase = j & ~63;
    dim3 grid(tiles, (unsigned)ceil_div(ncols_eff - cbase, kChunkCols));
    if (a.F.p == kMersenne31)
        hipLaunchKernelGGL(plain_step_kernel<true>, grid, dim3(kThreads), 0, s, a, j, ncols_eff);
    else
        hipLaunchKernelGGL(plain_step_kernel<false>, grid, dim3(kThreads), 0, s, a, j, ncols_eff);
    return hipGetLastError();
}

hipError_t plain_eliminate(const PlainArgs& a, const linac_opts* opts, hipStream_t s) {
    if (opts && opts->ev_begin) {
        hipError_t e = hipEventRecord(opts->ev_begin, s);
        if (e != hipSuccess) return e;
    }
    if (a.m > 0) {
        LaunchTimer lt(opts, s);
        for (int32_t j = 0; j < a.nsearch; ++j) {
            lt.before(LINAC_KERNEL_STEP);
            hipError_t e = launch_gj_step(a, j, a.ncols, s);
            lt.after();
            if (e != hipSuccess) return e;
        }
    }
    if (opts && opts->ev_end) {
        hipError_t e = hipEventRecord(opts->ev_end, s);
        if (e != hipSuccess) return e;
    }
    if (opts && opts->dominant_launches) *opts->dominant_launches = a.m > 0 ? a.nsearch : 0;
    return hipGetLastError();
}

hipError_t plain_finish_solve(const PlainArgs& a, int32_t n, int32_t k, uint32_t* X, int64_t ldx,
                              int32_t* rank, int32_t* pivots, uint8_t* consistent, hipStream_t s) {
    if ((int64_t)a.m * k > 0) {
        int64_t tot = (int64_t)a.m * k;
        hipLaunchKernelGGL(plain_incons_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s,
                           a, n, k);
    }
    int64_t tot = (int64_t)n * k;
    if (tot < k) tot = k;
    int64_t mn = a.m < n ? a.m : n;
    if (tot < mn) tot = mn;
    if (tot < 1) tot = 1;
    hipLaunchKernelGGL(plain_outputs_solve_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0,
                       s, a, n, k, X, ldx, rank, pivots, consistent);
    return hipGetLastError();
}

hipError_t plain_finish_rref(const PlainArgs& a, uint32_t* A, int64_t lda, int32_t* rank,
                             int32_t* pivots, hipStream_t s) {
    unsigned g = (unsigned)(a.m > 0 ? a.m : 1);
    hipLaunchKernelGGL(plain_outputs_rref_kernel, dim3(g), dim3(kThreads), 0, s, a, A, lda, rank,
                       pivots);
    return hipGetLastError();
}

hipError_t launch_range_check(const uint32_t* M, int64_t rows, int64_t cols, int64_t ld, uint32_t p,
                              uint32_t* flag, hipStream_t s) {
    if (rows * cols == 0) return hipSuccess;
    int64_t b = ceil_div(rows * cols, 256);
    hipLaunchKernelGGL(range_check_kernel, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s,
                       M, rows, cols, ld, p, flag);
    return hipGetLastError();
}

}  // namespace linac
