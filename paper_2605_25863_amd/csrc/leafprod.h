// The int8 leaf product of the blocked path, as a workgroup body shared by
// the product kernel (blocked.hip) and by the launch that runs its larger half
// beside the next leaf's first pivot selection (leaf.hip).
#pragma once
#include "internal.h"

namespace linac {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// Forward elimination (the solve): a row that became a pivot in an earlier
// panel (its pivot column below skip_below, the panel start) takes no part in
// a panel -- not in the leaf products, not in the trailing product, not in the
// write-back -- so it keeps its entries right of its own panel (the U part
// that back-substitution reads).  skip_below = 0 is Gauss-Jordan.
__device__ __forceinline__ bool earlier_pivot(int32_t rowcol, int32_t skip_below) {
    return rowcol >= 0 && rowcol < skip_below;
}

// sum_s 256^s S_s reduced mod p, plus `add` (a residue, or 0).  With K <= 512
// and |digit| <= 128 every |S_s| < 2^25, so T_lo = S_0 + ... + 2^24 S_3 (below
// 2^50) and T_hi = S_4 + 256 S_5 + 65536 S_6 (below 2^40) are exact in FP64.
// T_hi times c32 = 2^32 mod p (below 2^71) is split exactly by an FMA into its
// rounded head h and an integer tail l (|l| <= 2^18); h is reduced once into
// [-p, 2p) (h / p < 2^40, so the floor of h / p is off by at most one and the
// FMA's difference, an integer below 2p, is exact).  The sum of that, l, T_lo
// and `add` stays an integer below 2^51, and one more reduction with two
// corrections gives the residue.
__device__ __forceinline__ uint32_t fold7s(int32_t s0, int32_t s1, int32_t s2, int32_t s3, int32_t s4,
                                           int32_t s5, int32_t s6, uint32_t add, double c32,
                                           const FieldConst& F) {
    const double lo = __fma_rn(16777216.0, (double)s3,
                               __fma_rn(65536.0, (double)s2, __fma_rn(256.0, (double)s1, (double)s0)));
    const double hi = __fma_rn(65536.0, (double)s6, __fma_rn(256.0, (double)s5, (double)s4));
    const double h = hi * c32;
    const double l = __fma_rn(hi, c32, -h);
    const double t = __fma_rn(-floor(h * F.pinv), F.dp, h) + l + lo + (double)add;
    double r2 = __fma_rn(-floor(t * F.pinv), F.dp, t);
    if (r2 < 0.0) r2 += F.dp;
    if (r2 >= F.dp) r2 -= F.dp;
    return (uint32_t)r2;
}

__device__ __forceinline__ uint32_t fold7(const v4i* acc, int r, uint32_t add, double c32,
                                          const FieldConst& F) {
    return fold7s(acc[0][r], acc[1][r], acc[2][r], acc[3][r], acc[4][r], acc[5][r], acc[6][r], add,
                  c32, F);
}

constexpr int kLeafAll = 0, kLeafChunk = 1, kLeafRest = 2;

// Leaf product on int8 MFMA: PR columns [l0, l0 + N) of every row become
// C + A . Y, and Y itself for the leaf's pivot rows, where A = -(the row's
// values at the leaf's pivot columns) and Y = P^-1 R, R being the pivot rows as
// the selection saw them, with each pivot's implicit 1 in the transform block.
// 16x16x32 MFMA tiles keep a wave at seven 4-register accumulators, so the
// kernel fits in 128 VGPRs and shares SIMDs with a concurrent trailing product.
// Workgroup: kWaves waves over 16 rows each and kLeafBlocks 16-column blocks,
// taken one after the other with the same multipliers (int8 digits built in
// registers).
// Operand lanes of the 16x16x32 int8 MFMA: A(i, k) in lane i + 16 (k / 8), byte
// k % 8; B(k, j) in lane j + 16 (k / 8), byte k % 8; C(i, j) in lane j + 16 (i /
// 4), register i % 4.  Y's fragments (plane l of 16-column block b at
// (4 b + l) * 512 bytes, 8 per lane) come from the selection when it built
// them (out->yready: the first chunk decided the leaf); otherwise every block
// forms its own slices of Y (32 x 16 x t products in FP64 with exact 16-bit
// splits) from the rows the selection saved.  In a pipelined leaf the chunk
// launch (ymode 1, one workgroup per column group) stores the slices it forms,
// and the launch of the other rows (ymode 2) reads them instead of forming
// its own in every workgroup.  The leaf's pivot columns are not written (their
// unit-vector form is implied by the bookkeeping), so no multiplier is
// overwritten while other blocks still read it.  The launch also builds the next leaf's candidate list
// (one entry per thread).
// kLeafBlocks: 16-column blocks per workgroup (a tuned shape: 2, 3, 6 or 9;
// the multipliers' digits are built once and reused across the blocks, and
// every block's current values are loaded up front).
// kMode splits the rows so that the next leaf's first selection can start
// early: kLeafAll updates every row; kLeafChunk only the next leaf's first
// chunk (the first 32 entries of the next candidate list, workgroup row 0,
// which also stores that chunk for the selection); kLeafRest every row but
// those.  The two halves write disjoint rows, and only kLeafAll and kLeafRest
// compact the candidate list.
// bx: the workgroup's row block (kWaves x 16 rows), by: its column group,
// flat: its index among all workgroups of the product (for the compaction).
template <int kLeafBlocks, int kMode, int kWaves>
__device__ __forceinline__ void leaf_product_block(const LeafProdArgs& a, int64_t bx, int64_t by,
                                                   int64_t flat) {
    constexpr int kT = kWaves * 64;  // threads of the workgroup
    constexpr int kRows = kWaves * 16;
    const PlainArgs& w = a.w;
    const struct {
        uint32_t* M;
        int64_t ld;
    } pr{a.PR, a.ldpr};
    const int32_t l0 = a.l0, wl = a.wl, wj = a.wj, gcol0 = a.gcol0;
    const int64_t N = a.N;
    const LeafOut* out = a.out;
    const uint32_t* rsave = a.rsave;
    const int64_t ldr = a.ldr;
    const double c32 = a.c32;
    const int32_t skip_below = a.skip_below;
    __shared__ uint32_t sP[32][33];
    __shared__ uint32_t sR[32][17];
    __shared__ __attribute__((aligned(16))) int8_t sB[4][64][8];
    __shared__ int32_t slist[32];     // kLeafChunk: the chunk's rows
    __shared__ uint32_t smask[kRows / 32];  // kLeafRest: this workgroup's rows that are in the chunk
    __shared__ int32_t sn;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t rb = bx * kWaves + wave;  // 16-row block
    const int64_t cb0 = by * kLeafBlocks;
    const int64_t NB = ceil_div(N, 16);
    const int t = out->t;
    const uint32_t p = w.F.p;
    const int E = *a.count;
    if (kMode != kLeafChunk) {
        const int64_t i = flat * kT + tid;
        if (i == 0) *a.count_next = E - t;
        leaf_compact_entry(out, t, a.cand, a.cand_next, E, i);
    }
    if (kMode != kLeafAll) {
        if (tid < kRows / 32) smask[tid] = 0u;
        __syncthreads();
        if (wave == 0) {
            int32_t crow;
            int rank;
            const int n = next_chunk_entry(out, t, a.cand, E, lane, &crow, &rank);
            if (kMode == kLeafChunk) {
                if (rank < 32) slist[rank] = crow;
                if (lane == 0) sn = n;
                if (by == 0) {
                    if (rank < 32) a.chunk[rank] = crow;
                    if (lane == 0) a.chunk[32] = E - t;
                }
            } else if (rank < 32) {
                const int64_t off = (int64_t)crow - bx * kRows;
                if (off >= 0 && off < kRows) atomicOr(&smask[off >> 5], 1u << (off & 31));
            }
        }
        __syncthreads();
    }
    // row of local index r (16 rb + r): through the chunk's list for kLeafChunk
    // (entries past its length map to m, out of range)
    auto row_at = [&](int64_t r) -> int64_t {
        if (kMode != kLeafChunk) return r;
        return r < sn ? (int64_t)slist[r] : (int64_t)w.m;
    };
    auto in_chunk = [&](int64_t row) -> bool {
        if (kMode != kLeafRest) return false;
        const int64_t off = row - bx * kRows;
        return (smask[off >> 5] >> (off & 31)) & 1u;
    };
    if (kMode != kLeafChunk && skip_below > 0) {  // forward elimination: earlier pivot rows need nothing
        const int64_t row = bx * kRows + tid;
        int keep = 0;
        if (tid < kRows && row < w.m) keep = !earlier_pivot(w.rowcol[row], skip_below);
        if (__syncthreads_or(keep) == 0) return;
    }
    // All loads below use addresses clamped into their arrays and are issued
    // unconditionally (values out of range are discarded afterwards), so they
    // overlap instead of waiting one by one.
    const bool yready = a.ymode == 2 || out->yready != 0;
    // multipliers of this lane's A row (row 16 rb + L%16, k = 8 (L/16) + e)
    const int64_t arow = row_at(rb * 16 + (lane & 15));
    const int64_t arowc = arow < w.m ? arow : w.m - 1;
    const int kg = 8 * (lane >> 4);
    uint32_t av[8];
    int sel = -1;
    {
        int colv[32];  // the leaf's pivot columns (the array always has 32 entries)
        bool ident = true;  // pivot columns 0 .. t-1 (dense data): contiguous loads
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            colv[k] = out->col[k] & 31;
            ident = ident && (k >= t || colv[k] == k);
        }
        const int rc = w.rowcol[arowc] - gcol0;
        if (ident) {
            const uint4* src = (const uint4*)(pr.M + arowc * pr.ld + l0 + kg);
            for (int q4 = 0; q4 < 2; ++q4) {
                const uint4 v4 = src[q4];
                av[4 * q4] = v4.x;
                av[4 * q4 + 1] = v4.y;
                av[4 * q4 + 2] = v4.z;
                av[4 * q4 + 3] = v4.w;
            }
        } else {  // (rare) gather by the pivot columns, read per lane
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = pr.M[arowc * pr.ld + l0 + (out->col[kg + e] & 31)];
        }
#pragma unroll
        for (int s2 = 0; s2 < 32; ++s2)  // the row's own pivot of this leaf, if any
            if (s2 < t && rc >= 0 && rc < wl && colv[s2] == rc) sel = s2;
        for (int e = 0; e < 8; ++e)
            if (arow >= w.m || kg + e >= t) av[e] = 0u;
        if (arow >= w.m) sel = -1;
    }
    // epilogue rows (16 rb + 4 (L/16) + r): rowcol and current values, loaded
    // before any computation
    int rcv[4];
    uint32_t cur[kLeafBlocks][4];
    int64_t erow[4];
    for (int r = 0; r < 4; ++r) {
        erow[r] = row_at(rb * 16 + 4 * (lane >> 4) + r);
        rcv[r] = w.rowcol[erow[r] < w.m ? erow[r] : w.m - 1];
    }
#pragma unroll
    for (int cbi = 0; cbi < kLeafBlocks; ++cbi) {
        const int64_t col = (cb0 + cbi) * 16 + (lane & 15);
        const int64_t colc = col < N ? col : N - 1;
        for (int r = 0; r < 4; ++r)
            cur[cbi][r] = pr.M[(erow[r] < w.m ? erow[r] : w.m - 1) * pr.ld + l0 + colc];
    }
    long af[4];
    {
        int8_t outa[4][8];
        for (int e = 0; e < 8; ++e) {
            const int k = kg + e;
            uint32_t x = sel >= 0 ? (k == sel ? 1u : 0u) : (av[e] == 0 ? 0u : p - av[e]);
            int8_t d[4];
            digits4(centre(x, p), d);
            for (int l = 0; l < 4; ++l) outa[l][e] = d[l];
        }
        for (int l = 0; l < 4; ++l) __builtin_memcpy(&af[l], outa[l], 8);
    }
#pragma unroll
    for (int cbi = 0; cbi < kLeafBlocks; ++cbi) {
        const int64_t cb = cb0 + cbi;
        if (cb >= NB) continue;  // uniform over the block
        long bf[4];
        if (yready) {
            for (int l = 0; l < 4; ++l) bf[l] = *(const long*)(a.yfrag + (cb * 4 + l) * 512 + lane * 8);
        } else {
            __syncthreads();  // the previous slice's LDS is free
            for (int i = tid; i < 32 * 32; i += kT) {
                const int s = i >> 5, c = i & 31;
                sP[s][c] = (s < t && c < t) ? out->pinv[s * 32 + c] : 0u;
            }
            for (int i = tid; i < 32 * 16; i += kT) {
                const int s = i >> 4, c = i & 15;
                const int64_t col = cb * 16 + c;
                const uint32_t rv = rsave[s * ldr + (col < N ? col : N - 1)];
                const int cs = out->col[s];
                sR[s][c] = (s < t && col < N) ? (col == (int64_t)wj + cs ? 1u : rv) : 0u;
            }
            __syncthreads();
            for (int i = tid; i < 32 * 16; i += kT) {  // Y(s, c) in FP64 with 16-bit splits
                const int s = i >> 4, c = i & 15;
                double s1 = 0.0, s0 = 0.0;
                for (int k = 0; k < t; ++k) {
                    const uint32_t pv = sP[s][k];
                    const double rv = (double)sR[k][c];
                    s1 = __fma_rn((double)(pv >> 16), rv, s1);
                    s0 = __fma_rn((double)(pv & 0xffffu), rv, s0);
                }
                // s1 < 2^51, s0 < 2^52: exact; reduce s1, recombine below 2^53, reduce
                double q = floor(s1 * w.F.pinv);
                double h = __fma_rn(-q, w.F.dp, s1);
                q = floor(h * w.F.pinv);
                h = __fma_rn(-q, w.F.dp, h);
                double y = __fma_rn(h, 65536.0, s0);
                q = floor(y * w.F.pinv);
                y = __fma_rn(-q, w.F.dp, y);
                q = floor(y * w.F.pinv);
                y = __fma_rn(-q, w.F.dp, y);
                if (y < 0.0) y += w.F.dp;
                if (y >= w.F.dp) y -= w.F.dp;
                int8_t d[4];
                digits4(centre((uint32_t)y, p), d);
                for (int l = 0; l < 4; ++l) sB[l][c + 16 * (s >> 3)][s & 7] = d[l];
            }
            __syncthreads();
            for (int l = 0; l < 4; ++l) __builtin_memcpy(&bf[l], sB[l][lane], 8);
            if (a.ymode == 1 && wave == 0)  // the slice for the launch of the other rows
                for (int l = 0; l < 4; ++l) *(long*)(a.ystore + (cb * 4 + l) * 512 + lane * 8) = bf[l];
        }
        v4i acc[7];
        for (int g = 0; g < 7; ++g)
            for (int r = 0; r < 4; ++r) acc[g][r] = 0;
        for (int l = 0; l < 4; ++l)
            for (int lp = 0; lp < 4; ++lp)
                acc[l + lp] = __builtin_amdgcn_mfma_i32_16x16x32_i8(af[l], bf[lp], acc[l + lp], 0, 0, 0);
        const int64_t col = cb * 16 + (lane & 15);
        const bool pivcol = col < wl && w.colpiv[gcol0 + (col < wl ? col : 0)] >= 0;
        if (col < N && !pivcol) {
            for (int r = 0; r < 4; ++r) {
                const int64_t row = erow[r];
                if (row >= w.m || earlier_pivot(rcv[r], skip_below) || in_chunk(row)) continue;
                const bool fresh = rcv[r] >= gcol0 && rcv[r] < gcol0 + wl;  // a pivot row of this leaf
                pr.M[row * pr.ld + l0 + col] = fold7(acc, r, fresh ? 0u : cur[cbi][r], c32, w.F);
            }
        }
    }
}

}  // namespace
}  // namespace linac
