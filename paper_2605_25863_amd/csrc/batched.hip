// Many independent systems in one persistent launch.
//
// The paper solves one matrix per call (Sec. 2.3) and pays a launch per
// pivot column (Sec. 3.2).  For thousands of small systems that launch
// latency dominates, so here one workgroup solves a whole system with
// workgroup barriers between steps, and a persistent grid pulls systems from
// an atomic queue.  The host orders the queue by decreasing estimated cost
// (largest systems first: longest-processing-time scheduling).
//
// Per system, Gauss-Jordan (Sec. 3.2) in passes of kPB pivot columns, so that
// the system streams through the memory system once per pass, not once per
// column (with a thousand systems in flight they do not stay in cache):
//   1. the pass's columns of every row are copied to LDS and reduced there:
//      pivot = the smallest non-pivot row with a non-zero entry, one modular
//      inverse per pivot, every other eligible row updated; each row also
//      tracks the coefficients of its current values over the pass's pivot
//      rows as they were at the pass start;
//   2. the pass's pivot rows fully reduced (unit vectors at the pass's pivot
//      columns): PN_t = sum_s T[q_t][s] row_{q_s}, kPB-term dot products over
//      the full width;
//   3. every other row r (earlier pivots included) becomes r - sum_t
//      r[col_t] PN_t, the unique row of its coset with zeros at the pass's
//      pivot columns, and the pivot rows become PN.
// The dot products run in FP64 with the multiplier split into 16-bit halves,
// so every partial sum is exact (below 2^53).  Rows are never moved: pivot s
// is recorded in LDS.  Finally rank, pivots, X (free variables 0) and
// consistency are written.
#include <vector>

#include "internal.h"

namespace linac {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxRows = 1024;   // LDS bookkeeping bound per system
constexpr int kMaxCols = 2048;   // n + k bound
constexpr int kPB = 8;           // pivot columns per pass

struct SysDesc {
    const uint32_t* A;
    const uint32_t* B;
    uint32_t* X;
    int32_t* rank;
    int32_t* pivots;
    uint8_t* consistent;
    uint32_t* W;       // working region in the workspace (m rows, then kPB scratch rows)
    int32_t m, n, k;
    int32_t lda, ldb, ldx;
    int32_t ldw;       // multiple of 4
    int32_t pad;
    FieldConst F;
};

__device__ __forceinline__ int block_min(int v, int* red) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    v = min(min(red[0], red[1]), min(red[2], red[3]));
    __syncthreads();
    return v;
}

// (s1 2^16 + s0) mod p for the exact partial sums of a split dot product
// (s1 < 2^50, s0 < 2^51).
__device__ __forceinline__ uint32_t split_reduce(double s1, double s0, const FieldConst& F) {
    double q = floor(s1 * F.pinv);
    const double h = __fma_rn(-q, F.dp, s1);  // (-p, 2p)
    double y = __fma_rn(h, 65536.0, s0);      // |y| < 2^52
    q = floor(y * F.pinv);
    y = __fma_rn(-q, F.dp, y);  // (-p, 2p)
    if (y < 0.0) y += F.dp;
    if (y >= F.dp) y -= F.dp;
    return (uint32_t)y;
}

// LDS of one system: pivot state per row (0 candidate, 1 pivot of an earlier
// pass, 2 pivot of this pass), the pivot list, the pass's panel (later the
// rows' multipliers) and coefficient tracks, and each pass pivot's index.
struct BatchLds {
    uint8_t piv[kMaxRows];
    int8_t pt[kMaxRows];
    int32_t pivrow[kMaxRows];
    int32_t pivcol[kMaxRows];
    uint32_t P[kMaxRows * kPB];
    uint32_t T[kMaxRows * kPB];
    int red[4];
};

__device__ void solve_one(const SysDesc& d, BatchLds& L) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = d.m, n = d.n, k = d.k, ncols = n + k, ldw = d.ldw;
    const FieldConst F = d.F;
    const uint32_t p = F.p;
    uint32_t* PN = d.W + (int64_t)m * ldw;  // the pass's reduced pivot rows
    // stage [A | B] (padding columns zero); one wave per row
    for (int r = wave; r < m; r += 4) {
        for (int c = lane; c < ldw; c += 64) {
            d.W[(int64_t)r * ldw + c] = c < n ? d.A[(int64_t)r * d.lda + c]
                                              : (c < ncols ? d.B[(int64_t)r * d.ldb + (c - n)] : 0u);
        }
    }
    for (int r = tid; r < m; r += kThreads) L.piv[r] = 0;
    __syncthreads();
    int rank = 0;
    for (int j0 = 0; j0 < n && rank < m; j0 += kPB) {
        const int bw = min(kPB, n - j0);
        // 1. the pass's columns of the candidate rows, and empty tracks
        for (int i = tid; i < m * kPB; i += kThreads) {
            const int r = i / kPB, c = i % kPB;
            L.P[i] = (c < bw && L.piv[r] == 0) ? d.W[(int64_t)r * ldw + j0 + c] : 0u;
            L.T[i] = 0u;
        }
        __syncthreads();
        int np = 0;
        for (int c = 0; c < bw && rank + np < m; ++c) {
            int cand = INT32_MAX;
            for (int r = tid; r < m; r += kThreads)
                if (L.piv[r] == 0 && L.P[r * kPB + c] != 0 && r < cand) cand = r;
            const int q = block_min(cand, L.red);  // its barriers also publish the panel
            if (q == INT32_MAX) continue;          // free column
            const uint32_t inv = inv_mod_fermat(__builtin_amdgcn_readfirstlane(L.P[q * kPB + c]), F);
            // row q becomes pivot np of the pass: its own term turns into an
            // explicit coefficient, then the row is scaled to a leading 1
            if (tid < kPB) {
                const uint32_t tq = tid == np ? 1u : L.T[q * kPB + tid];
                L.T[q * kPB + tid] = mul_mod(tq, inv, F);
                L.P[q * kPB + tid] = mul_mod(L.P[q * kPB + tid], inv, F);
            }
            if (tid == 0) {
                L.piv[q] = 2;
                L.pt[q] = (int8_t)np;
                L.pivrow[rank + np] = q;
                L.pivcol[rank + np] = j0 + c;
            }
            __syncthreads();
            // column c out of the other candidates and the pass's earlier pivots
            for (int r = tid; r < m; r += kThreads) {
                if (r == q || L.piv[r] == 1) continue;
                const uint32_t f = L.P[r * kPB + c];
                if (f == 0) continue;
                for (int cc = 0; cc < kPB; ++cc)
                    L.P[r * kPB + cc] = sub_mod(L.P[r * kPB + cc], mul_mod(f, L.P[q * kPB + cc], F), p);
                for (int t = 0; t < kPB; ++t)
                    L.T[r * kPB + t] = sub_mod(L.T[r * kPB + t], mul_mod(f, L.T[q * kPB + t], F), p);
            }
            ++np;
            __syncthreads();
        }
        if (np == 0) continue;
        // 2. PN_t = sum_s T[q_t][s] row_{q_s} over 4-column groups from c0 (the
        // rows are zero before j0, so PN is too)
        const int c0 = j0 & ~3;
        const int ngroups = (ncols - c0 + 3) >> 2;
        // (all kPB terms are evaluated with every load issued first: beyond np
        // the coefficients are zero and the row index is clamped to pivot 0)
        for (int i = tid; i < np * ngroups; i += kThreads) {
            const int t = i / ngroups, c = c0 + 4 * (i % ngroups);
            const int qt = L.pivrow[rank + t];
            uint4 wv[kPB];
#pragma unroll
            for (int sidx = 0; sidx < kPB; ++sidx)
                wv[sidx] = *(const uint4*)(d.W + (int64_t)L.pivrow[rank + (sidx < np ? sidx : 0)] * ldw + c);
            double s1[4] = {0.0, 0.0, 0.0, 0.0}, s0[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int sidx = 0; sidx < kPB; ++sidx) {
                const uint32_t tv = L.T[qt * kPB + sidx];
                const double hi = (double)(tv >> 16), lo = (double)(tv & 0xffffu);
                const uint32_t w4[4] = {wv[sidx].x, wv[sidx].y, wv[sidx].z, wv[sidx].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    s1[e] = __fma_rn(hi, (double)w4[e], s1[e]);
                    s0[e] = __fma_rn(lo, (double)w4[e], s0[e]);
                }
            }
            uint32_t o[4];
            for (int e = 0; e < 4; ++e) o[e] = split_reduce(s1[e], s0[e], F);
            *(uint4*)(PN + (int64_t)t * ldw + c) = make_uint4(o[0], o[1], o[2], o[3]);
        }
        // the rows' multipliers: their pass-start values at the pass's pivot columns
        for (int i = tid; i < m * kPB; i += kThreads) {
            const int r = i / kPB, t = i % kPB;
            L.P[i] = (t < np && L.piv[r] != 2) ? d.W[(int64_t)r * ldw + L.pivcol[rank + t]] : 0u;
        }
        __threadfence_block();
        __syncthreads();
        // 3. r <- r - sum_t a_r[t] PN_t for every other row; the pivots take PN
        for (int i = tid; i < m * ngroups; i += kThreads) {
            const int r = i / ngroups, c = c0 + 4 * (i % ngroups);
            uint4* dst = (uint4*)(d.W + (int64_t)r * ldw + c);
            if (L.piv[r] == 2) {
                *dst = *(const uint4*)(PN + (int64_t)L.pt[r] * ldw + c);
                continue;
            }
            uint32_t a[kPB];  // zero beyond np
            bool any = false;
#pragma unroll
            for (int t = 0; t < kPB; ++t) {
                a[t] = L.P[r * kPB + t];
                any |= a[t] != 0;
            }
            if (!any) continue;
            uint4 pv[kPB];
#pragma unroll
            for (int t = 0; t < kPB; ++t) pv[t] = *(const uint4*)(PN + (int64_t)(t < np ? t : 0) * ldw + c);
            const uint4 x = *dst;
            double s1[4] = {0.0, 0.0, 0.0, 0.0}, s0[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < kPB; ++t) {
                const double hi = (double)(a[t] >> 16), lo = (double)(a[t] & 0xffffu);
                const uint32_t p4[4] = {pv[t].x, pv[t].y, pv[t].z, pv[t].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    s1[e] = __fma_rn(hi, (double)p4[e], s1[e]);
                    s0[e] = __fma_rn(lo, (double)p4[e], s0[e]);
                }
            }
            const uint32_t x4[4] = {x.x, x.y, x.z, x.w};
            uint32_t o[4];
            for (int e = 0; e < 4; ++e) o[e] = sub_mod(x4[e], split_reduce(s1[e], s0[e], F), p);
            *dst = make_uint4(o[0], o[1], o[2], o[3]);
        }
        __threadfence_block();
        __syncthreads();
        for (int r = tid; r < m; r += kThreads)
            if (L.piv[r] == 2) L.piv[r] = 1;
        rank += np;
        __syncthreads();
    }
    // outputs: rank, pivots (ascending by construction), consistency, X
    const int mn = min(m, n);
    if (tid == 0) *d.rank = rank;
    for (int s = tid; s < mn; s += kThreads) d.pivots[s] = s < rank ? L.pivcol[s] : -1;
    for (int t = tid; t < k; t += kThreads) d.consistent[t] = 1;
    for (int64_t i = tid; i < (int64_t)n * k; i += kThreads) d.X[(i / k) * d.ldx + (i % k)] = 0u;
    __syncthreads();
    // a non-pivot row with a non-zero right-hand side entry makes its column inconsistent
    for (int r = wave; r < m; r += 4) {
        if (L.piv[r]) continue;
        for (int t = lane; t < k; t += 64)
            if (d.W[(int64_t)r * ldw + n + t] != 0) d.consistent[t] = 0;
    }
    __syncthreads();
    for (int s = wave; s < rank; s += 4) {
        const int col = L.pivcol[s];
        const uint32_t* row = d.W + (int64_t)L.pivrow[s] * ldw + n;
        for (int t = lane; t < k; t += 64)
            if (d.consistent[t]) d.X[(int64_t)col * d.ldx + t] = row[t];
    }
    __syncthreads();
}

// Persistent kernel: every workgroup takes the next system from the queue until
// the queue is exhausted (each workgroup exits once the counter passes count).
__global__ __launch_bounds__(kThreads) void batched_kernel(const SysDesc* sys, int32_t count,
                                                           unsigned int* counter) {
    __shared__ BatchLds L;
    __shared__ uint32_t s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1u);
        __syncthreads();
        const unsigned int idx = s_idx;
        __syncthreads();
        if (idx >= (unsigned int)count) break;
        const SysDesc d = sys[idx];
        solve_one(d, L);
    }
}

__global__ void reset_counter_kernel(unsigned int* counter) { *counter = 0u; }

}  // namespace

size_t batched_desc_bytes() { return sizeof(SysDesc); }

bool batched_fits(int64_t m, int64_t n, int64_t k) {
    return m <= kMaxRows && n + k <= kMaxCols;
}

// Layout: [counter | descriptors | working regions]
size_t batched_workspace(const linac_system* sys, int32_t count) {
    size_t off = 256 + round_up((int64_t)count * sizeof(SysDesc), 256);
    for (int32_t i = 0; i < count; ++i) {
        const int64_t ldw = round_up(sys[i].n + sys[i].k > 0 ? sys[i].n + sys[i].k : 1, 4);
        off += round_up(((int64_t)sys[i].m + kPB) * ldw * 4, 256);
    }
    return off + 256;
}

// Fill host descriptors in queue order (decreasing cost).
void batched_describe(const linac_system* sys, int32_t count, void* ws, void* host_desc,
                      int32_t* order) {
    SysDesc* h = (SysDesc*)host_desc;
    char* base = (char*)ws;
    size_t off = 256 + round_up((int64_t)count * sizeof(SysDesc), 256);
    // working regions follow the caller's order; the queue follows cost
    std::vector<size_t> region(count);
    for (int32_t i = 0; i < count; ++i) {
        region[i] = off;
        const int64_t ldw = round_up(sys[i].n + sys[i].k > 0 ? sys[i].n + sys[i].k : 1, 4);
        off += round_up(((int64_t)sys[i].m + kPB) * ldw * 4, 256);
    }
    for (int32_t qi = 0; qi < count; ++qi) {
        const int32_t i = order[qi];
        const linac_system& s = sys[i];
        SysDesc& d = h[qi];
        d.A = s.A;
        d.B = s.B;
        d.X = s.X;
        d.rank = s.rank;
        d.pivots = s.pivots;
        d.consistent = s.consistent;
        d.W = (uint32_t*)(base + region[i]);
        d.m = s.m;
        d.n = s.n;
        d.k = s.k;
        d.lda = s.lda;
        d.ldb = s.ldb;
        d.ldx = s.ldx;
        d.ldw = (int32_t)round_up(s.n + s.k > 0 ? s.n + s.k : 1, 4);
        d.pad = 0;
        d.F = make_field(s.p);
    }
}

hipError_t batched_launch(void* ws, int32_t count, int32_t grid, hipStream_t s) {
    unsigned int* counter = (unsigned int*)ws;
    const SysDesc* desc = (const SysDesc*)((char*)ws + 256);
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    hipLaunchKernelGGL(batched_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, desc, count,
                       counter);
    return hipGetLastError();
}

void* batched_desc_ptr(void* ws) { return (char*)ws + 256; }

}  // namespace linac
