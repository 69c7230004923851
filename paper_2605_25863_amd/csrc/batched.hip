// Many independent systems in one persistent launch.
//
// The paper solves one matrix per call (Sec. 2.3) and pays a launch per
// pivot column (Sec. 3.2).  For thousands of small systems that launch
// latency dominates, so here one workgroup solves a whole system with
// workgroup barriers between pivot steps, and a persistent grid pulls systems
// from an atomic queue.  The host orders the queue by decreasing estimated
// cost (largest systems first: longest-processing-time scheduling).
//
// Per system (Gauss-Jordan, as in the plain path, Sec. 3.2):
//   copy [A | B] into a private working region of the workspace;
//   for each column j < n: the smallest non-pivot row with a non-zero entry is
//   the pivot (workgroup min-reduction), its inverse is taken by one thread,
//   the normalised pivot row is staged in LDS with its Shoup quotients, every
//   other row with f = W[r][j] != 0 is updated with 128-bit accesses, and the
//   pivot row is written back normalised (rows are never moved: the s-th pivot
//   row is recorded in LDS);
//   finally rank, pivots, X (free variables 0) and consistency are written.
#include <vector>

#include "internal.h"

namespace linac {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxRows = 1024;   // LDS bookkeeping bound per system
constexpr int kMaxCols = 2048;   // n + k bound (staged pivot row)

struct SysDesc {
    const uint32_t* A;
    const uint32_t* B;
    uint32_t* X;
    int32_t* rank;
    int32_t* pivots;
    uint8_t* consistent;
    uint32_t* W;       // working region in the workspace
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

__device__ void solve_one(const SysDesc& d, uint8_t* s_piv, int32_t* s_pivrow, int32_t* s_pivcol,
                          uint32_t* s_pn, uint32_t* s_pq, uint32_t* s_f, int* s_red,
                          uint32_t* s_bcast) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = d.m, n = d.n, k = d.k, ncols = n + k, ldw = d.ldw;
    const int nvec_row = ldw >> 2;
    const FieldConst F = d.F;
    const uint32_t p = F.p;
    // stage [A | B] (padding columns zero); one wave per row
    for (int r = wave; r < m; r += 4) {
        for (int c = lane; c < ldw; c += 64) {
            d.W[(int64_t)r * ldw + c] = c < n ? d.A[(int64_t)r * d.lda + c]
                                              : (c < ncols ? d.B[(int64_t)r * d.ldb + (c - n)] : 0u);
        }
    }
    for (int r = tid; r < m; r += kThreads) s_piv[r] = 0;
    __syncthreads();
    int rank = 0;
    for (int j = 0; j < n && rank < m; ++j) {
        // pivot search and multipliers of column j
        int cand = INT32_MAX;
        for (int r = tid; r < m; r += kThreads) {
            const uint32_t v = d.W[(int64_t)r * ldw + j];
            s_f[r] = v;
            if (v != 0 && !s_piv[r] && r < cand) cand = r;
        }
        const int q = block_min(cand, s_red);  // its barriers also publish s_f
        if (q == INT32_MAX) continue;          // free column
        // every wave takes the (wave-uniform) inverse itself on the scalar unit
        const uint32_t inv = inv_mod_fermat(__builtin_amdgcn_readfirstlane(s_f[q]), F);
        if (tid == 0) {
            s_piv[q] = 1;
            s_pivrow[rank] = q;
            s_pivcol[rank] = j;
        }
        __syncthreads();
        const int v0 = j >> 2;  // first 4-column vector touched
        for (int c = 4 * v0 + tid; c < ldw; c += kThreads) {
            const uint32_t v = c < ncols ? mul_mod(d.W[(int64_t)q * ldw + c], inv, F) : 0u;
            s_pn[c] = v;
            s_pq[c] = shoup_quot(v, F);
        }
        __syncthreads();
        // pivot row written back normalised; other rows with f != 0 updated
        for (int r = wave; r < m; r += 4) {
            const uint32_t f = s_f[r];
            if (r != q && f == 0) continue;
            uint4* row = (uint4*)(d.W + (int64_t)r * ldw);
            for (int vi = v0 + lane; vi < nvec_row; vi += 64) {
                const int c = 4 * vi;
                if (r == q) {
                    row[vi] = make_uint4(s_pn[c], s_pn[c + 1], s_pn[c + 2], s_pn[c + 3]);
                    continue;
                }
                uint4 x = row[vi];
                uint32_t v[4] = {x.x, x.y, x.z, x.w};
                for (int e = 0; e < 4; ++e) {
                    const uint32_t t =
                        reduce_2p(shoup_mul_lazy(f, s_pn[c + e], s_pq[c + e], p), p);
                    v[e] = sub_mod(v[e], t, p);
                }
                row[vi] = make_uint4(v[0], v[1], v[2], v[3]);
            }
        }
        ++rank;
        __syncthreads();
    }
    // outputs: rank, pivots (ascending by construction), consistency, X
    const int mn = min(m, n);
    if (tid == 0) *d.rank = rank;
    for (int s = tid; s < mn; s += kThreads) d.pivots[s] = s < rank ? s_pivcol[s] : -1;
    for (int t = tid; t < k; t += kThreads) d.consistent[t] = 1;
    for (int64_t i = tid; i < (int64_t)n * k; i += kThreads) d.X[(i / k) * d.ldx + (i % k)] = 0u;
    __syncthreads();
    // a non-pivot row with a non-zero right-hand side entry makes its column inconsistent
    for (int r = wave; r < m; r += 4) {
        if (s_piv[r]) continue;
        for (int t = lane; t < k; t += 64)
            if (d.W[(int64_t)r * ldw + n + t] != 0) d.consistent[t] = 0;
    }
    __syncthreads();
    for (int s = wave; s < rank; s += 4) {
        const int col = s_pivcol[s];
        const uint32_t* row = d.W + (int64_t)s_pivrow[s] * ldw + n;
        for (int t = lane; t < k; t += 64)
            if (d.consistent[t]) d.X[(int64_t)col * d.ldx + t] = row[t];
    }
    __syncthreads();
}

// Persistent kernel: every workgroup takes the next system from the queue until
// the queue is exhausted (each workgroup exits once the counter passes count).
__global__ __launch_bounds__(kThreads) void batched_kernel(const SysDesc* sys, int32_t count,
                                                           unsigned int* counter) {
    __shared__ uint8_t s_piv[kMaxRows];
    __shared__ int32_t s_pivrow[kMaxRows];
    __shared__ int32_t s_pivcol[kMaxRows];
    __shared__ uint32_t s_pn[kMaxCols];
    __shared__ uint32_t s_pq[kMaxCols];
    __shared__ uint32_t s_f[kMaxRows];
    __shared__ int s_red[4];
    __shared__ uint32_t s_bcast[2];
    for (;;) {
        if (threadIdx.x == 0) s_bcast[1] = atomicAdd(counter, 1u);
        __syncthreads();
        const unsigned int idx = s_bcast[1];
        __syncthreads();
        if (idx >= (unsigned int)count) break;
        const SysDesc d = sys[idx];
        solve_one(d, s_piv, s_pivrow, s_pivcol, s_pn, s_pq, s_f, s_red, s_bcast);
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
        off += round_up((int64_t)sys[i].m * ldw * 4, 256);
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
        off += round_up((int64_t)sys[i].m * ldw * 4, 256);
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
