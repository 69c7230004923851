// Many independent systems in one persistent launch.
//
// The paper solves one matrix per call (Sec. 2.3) and pays a launch per
// pivot column (Sec. 3.2).  For thousands of small systems that launch
// latency dominates, so here one workgroup solves a whole system with
// workgroup barriers between steps, and a persistent grid pulls systems from
// an atomic queue.  The host orders the queue by decreasing estimated cost
// (largest systems first: longest-processing-time scheduling).
//
// Per system, elimination with the paper's pivot rule (Sec. 3.2) in passes of
// kPB pivot columns, so that the system streams through the memory system once
// per pass, not once per column (with a thousand systems in flight they do not
// stay in cache).  The outputs are X, rank, pivots and consistency, not the
// reduced matrix, so a pass updates only the rows that are still candidates
// (forward elimination) and X is found by back-substitution at the end: the
// same results as Gauss-Jordan (X on the pivot variables is the unique solution
// of the echelon system with free variables 0).  A pass:
//   1. the pass's columns of every row are loaded once into LDS; one wave
//      finds the pivots (pivot of a column = the first candidate row whose
//      reduced value there is non-zero), keeping the first candidates reduced
//      fraction-free in registers (no inverse on this serial chain);
//   2. the pass's pivot rows fully reduced (unit vectors at the pass's pivot
//      columns): PN_t = sum_s T[t][s] row_{q_s}, with T the inverse of the
//      pivot block M[s][u] = row_{q_s}[col_u] (one wave, one inverse per pivot
//      in parallel), kPB-term dot products over the columns after the pass;
//   3. every candidate row r becomes r - sum_t r[col_t] PN_t, the unique row
//      of its coset with zeros at the pass's pivot columns, and the pass's
//      pivot rows become PN; pivot rows of earlier passes are not touched.
// The dot products run in FP64 with one factor split into 16-bit halves, so
// every partial sum is exact (below 2^53); step 3, a product of the rows'
// multipliers by the reduced pivot rows, runs on the FP64 matrix cores.  Rows
// are never moved: pivot s is recorded in LDS.  Finally rank, pivots,
// consistency and X (by back-substitution, free variables 0) are written.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace linac {

// The rows' multipliers of the current pass (kPB per row), in dynamic LDS
// sized at launch to the batch's largest system, so that batches of smaller
// systems fit more workgroups per CU.
extern __shared__ uint32_t g_mult[];

namespace {

constexpr int kThreads = 256;
constexpr int kMaxRows = 1024;   // LDS bookkeeping bound per system
constexpr int kMaxCols = 2048;   // n + k bound
constexpr int kPB = 16;          // pivot columns per pass (a multiple of 8)

// Global-memory views of the descriptor's pointers.  The descriptor is read
// from memory, so through its generic pointers every access would compile to a
// flat access, which counts against both the vector-memory and the LDS wait
// counters and so serialises loads with LDS traffic.
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4u gu4;
typedef __attribute__((address_space(1))) int32_t gi32;
typedef __attribute__((address_space(1))) uint8_t gu8;

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
    int32_t ldw;       // words per row, a multiple of 32
    int32_t pad;
    FieldConst F;
};

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

typedef double v4d __attribute__((ext_vector_type(4)));

// (d x - f y) mod p for residues d, x, f, y: each product is reduced exactly
// as in mul_mod (to [-p, 2p)), then the difference (-3p, 3p) is reduced.
__device__ __forceinline__ uint32_t mul_sub_mod(double d, uint32_t x, double f, double y,
                                                const FieldConst& F) {
    const double dx = (double)x;
    const double h1 = d * dx, l1 = __fma_rn(d, dx, -h1);
    const double h2 = f * y, l2 = __fma_rn(f, y, -h2);
    const double r1 = __fma_rn(-floor(h1 * F.pinv), F.dp, h1) + l1;
    const double r2 = __fma_rn(-floor(h2 * F.pinv), F.dp, h2) + l2;
    double r = r1 - r2;
    r = __fma_rn(-floor(r * F.pinv), F.dp, r);  // [-p, 2p)
    if (r < 0.0) r += F.dp;
    if (r >= F.dp) r -= F.dp;
    return (uint32_t)r;
}

// x - (s1 2^16 + s0) mod p for x < p and the exact sums s1 < 2^50, s0 < 2^51.
__device__ __forceinline__ uint32_t sub_split(uint32_t x, double s1, double s0, const FieldConst& F) {
    double q = floor(s1 * F.pinv);
    const double h = __fma_rn(-q, F.dp, s1);           // (-p, 2p)
    double y = __fma_rn(-h, 65536.0, (double)x - s0);  // |y| < 2^52
    q = floor(y * F.pinv);
    y = __fma_rn(-q, F.dp, y);  // [-p, 2p)
    if (y < 0.0) y += F.dp;
    if (y >= F.dp) y -= F.dp;
    return (uint32_t)y;
}

// LDS of one system (the pass's panel and multipliers are in g_mult): pivot
// state per row (0 candidate, 1 pivot of an earlier pass, 2 pivot of this
// pass), each pass pivot's index, the pivot list, the coefficients T of the
// reduced pivot rows over the pass-start pivot rows, the consistency flags, the
// passes' first pivots, and the pivot search's state.
struct BatchLds {
    uint8_t piv[kMaxRows];
    int8_t pt[kMaxRows];
    int16_t pivrow[kMaxRows];
    int16_t pivcol[kMaxRows];
    uint32_t T[kPB * kPB];
    uint8_t cons[kMaxCols];
    int16_t pstart[kMaxCols / kPB + 2];  // rank at the start of each pass with pivots
    // pivot search of a pass: the window's rows, and each pivot's panel row
    // (reduced by the pass's earlier pivots), leading value and pass column
    int32_t win[16];
    int16_t beyond[kMaxRows];  // the other candidate rows with a non-zero pass panel
    uint8_t nz[kMaxRows];      // candidate row with a non-zero pass panel
    uint32_t upan[kPB * kPB];
    uint32_t mst[kPB * kPB];  // each pivot's pass-start panel row
    uint32_t ud[kPB];
    int32_t upc[kPB];
    int32_t npp[2];  // the pass's pivot count, by pass parity
};

// T = M^-1 for the pass's pivot block M[s][u] = row_{q_s}[col_u] (pass-start
// values), by one wave: Gauss-Jordan on [M | I] in the pivot order (every
// leading block is invertible: it is what the pass eliminated), fraction-free
// (row_r <- d_s row_r - M[r][s] row_s, no inverse per step), then each row
// scaled by the inverse of its diagonal entry.  Entry (s, u) of M and of I
// lives in lane s * kLpr + u / kEpl, element u % kEpl.
constexpr int kLpr = 64 / kPB;    // lanes per row of the block
constexpr int kEpl = kPB / kLpr;  // entries per lane
static_assert(kEpl == 4, "the block inverse keeps four entries per lane");

__device__ void pivot_block_inverse(const SysDesc& d, BatchLds& L, int rank, int np) {
    const int lane = threadIdx.x & 63, s = lane / kLpr, ub = (lane % kLpr) * kEpl;
    const FieldConst& F = d.F;
    // vectors, not arrays: an element picked by a run-time index stays in
    // registers.  M comes from the pivots' pass-start panel rows, which the
    // pivot search recorded.
    v4u mv, iv;
#pragma unroll
    for (int e = 0; e < kEpl; ++e) {
        const int u = ub + e;
        const uint32_t w = L.mst[min(s, np - 1) * kPB + L.upc[min(u, np - 1)]];
        mv[e] = s < np && u < np ? w : 0u;
        iv[e] = s == u ? 1u : 0u;
    }
    for (int t = 0; t < np; ++t) {
        const int tl = t / kEpl, te = t % kEpl;  // column t: lane offset, element
        const uint32_t colt = mv[te];
        const uint32_t dt = __shfl(colt, t * kLpr + tl);
        const uint32_t f = __shfl(colt, s * kLpr + tl);
        v4u my, iy;
#pragma unroll
        for (int e = 0; e < kEpl; ++e) {
            my[e] = __shfl(mv[e], t * kLpr + lane % kLpr);
            iy[e] = __shfl(iv[e], t * kLpr + lane % kLpr);
        }
        if (s != t) {
#pragma unroll
            for (int e = 0; e < kEpl; ++e) {
                mv[e] = mul_sub_mod((double)dt, mv[e], (double)f, (double)my[e], F);
                iv[e] = mul_sub_mod((double)dt, iv[e], (double)f, (double)iy[e], F);
            }
        }
    }
    // the diagonal entry of row s sits in lane s * kLpr + s / kEpl, element s % kEpl
    const uint32_t ds = __shfl(mv[s % kEpl], s * kLpr + s / kEpl);
    const uint32_t inv = inv_mod_fermat(ds, F);
#pragma unroll
    for (int e = 0; e < kEpl; ++e)
        if (s < np && ub + e < np) L.T[s * kPB + ub + e] = mul_mod(iv[e], inv, F);
}

// Step 3 of a pass: r <- r - sum_t a_r[t] PN_t for the candidate rows with a
// non-zero multiplier, as the transposed product (width x kPB) by (kPB x 16 rows) on
// the 16x16x4 FP64 MFMA, the multipliers split into 16-bit halves (a = hi
// 2^16 + lo, two products).  Lane L (j = L % 16, g = L / 16) supplies
// PN[4 kb + g][tile column 4 (j % 4) + j / 4] and the halves of a[16 rb + j]
// [4 kb + g]; its four results are then row 16 rb + j at the tile columns 4 g
// .. 4 g + 3, one 16-byte load and store.  Products are below 2^47 and sums of
// kPB = 16 of them below 2^51, so the MFMA sums are exact.  A wave takes 16 rows by
// kStrip tiles, all loads issued first.
constexpr int kStrip = 4;

__device__ void update_rows(const SysDesc& d, const BatchLds& L, const gu32* PN, int np,
                            int c0) {
    constexpr int KB = kPB / 4;  // k-blocks of the MFMA
    gu32* W = (gu32*)d.W;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = d.m, ncols = d.n + d.k, ldw = d.ldw;
    const int nrb = (m + 15) >> 4, nct = (ncols - c0 + 15) >> 4;
    const int nst = (nct + kStrip - 1) / kStrip;
    const int j = lane & 15, g = lane >> 4;
    const int acol = 4 * (j & 3) + (j >> 2);
    int tk[KB];  // the PN row of each k-block (clamped beyond np: its multiplier is 0)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) tk[kb] = min(4 * kb + g, np - 1);
    for (int item = wave; item < nrb * nst; item += kThreads / 64) {
        const int rb = item / nst, st = item - rb * nst;
        const int row = rb * 16 + j;
        const bool rin = row < m;
        // every load below is unconditional, from a clamped address (a load
        // under a branch would be waited for before the join)
        const int rowc = rin ? row : m - 1;
        uint32_t a[KB];
        uint32_t any = 0u;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            a[kb] = rin ? g_mult[rowc * kPB + 4 * kb + g] : 0u;
            any |= a[kb];
        }
        const int state = L.piv[rowc];
        const bool pivot = rin && state == 2, keep = rin && state != 1;
        const int prow = L.pt[rowc];
        if (!__any(any != 0u || pivot)) continue;
        // a pivot row of the pass (zero multipliers) reads its PN row and so
        // takes it unchanged; a pivot row of an earlier pass is not written
        const gu32* xrow = state == 0 ? W + (int64_t)rowc * ldw : PN + (int64_t)(pivot ? prow : 0) * ldw;
        uint32_t pb[kStrip][KB];
#pragma unroll
        for (int e = 0; e < kStrip; ++e) {  // PN first: the MFMAs need it first
            const int ca = min(c0 + (st * kStrip + e) * 16 + acol, ldw - 1);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) pb[e][kb] = PN[(int64_t)tk[kb] * ldw + ca];
        }
        v4u x[kStrip];
#pragma unroll
        for (int e = 0; e < kStrip; ++e)
            x[e] = *(const gu4*)(xrow + min(c0 + (st * kStrip + e) * 16 + 4 * g, ldw - 4));
        double ah[KB], al[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            ah[kb] = (double)(a[kb] >> 16);
            al[kb] = (double)(a[kb] & 0xffffu);
        }
#pragma unroll
        for (int e = 0; e < kStrip; ++e) {
            const int tc = c0 + (st * kStrip + e) * 16;
            if (tc >= ncols) break;
            v4d hi = (v4d){0.0, 0.0, 0.0, 0.0}, lo = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const double b = (double)pb[e][kb];
                hi = __builtin_amdgcn_mfma_f64_16x16x4f64(b, ah[kb], hi, 0, 0, 0);
                lo = __builtin_amdgcn_mfma_f64_16x16x4f64(b, al[kb], lo, 0, 0, 0);
            }
            const int cx = tc + 4 * g;
            if (keep && cx < ncols)
                *(gu4*)(W + (int64_t)row * ldw + cx) =
                    (v4u){sub_split(x[e].x, hi[0], lo[0], d.F), sub_split(x[e].y, hi[1], lo[1], d.F),
                          sub_split(x[e].z, hi[2], lo[2], d.F), sub_split(x[e].w, hi[3], lo[3], d.F)};
        }
    }
}

// dst[r][c] = src[r][c] for r < rows, c < cols: a wave per row, a lane per
// column, kStageRows rows of loads in flight before their stores.
constexpr int kStageRows = 16;

__device__ void copy_block(gu32* dst, int ldd, const gu32* src, int lds, int rows, int cols) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int nw = kThreads / 64;
    for (int c0 = 0; c0 < cols; c0 += 64) {
        const int c = c0 + lane, cc = min(c, cols - 1);
        for (int r0 = wave; r0 < rows; r0 += nw * kStageRows) {
            uint32_t v[kStageRows];
#pragma unroll
            for (int u = 0; u < kStageRows; ++u)
                v[u] = src[(int64_t)min(r0 + nw * u, rows - 1) * lds + cc];
#pragma unroll
            for (int u = 0; u < kStageRows; ++u)
                if (r0 + nw * u < rows && c < cols) dst[(int64_t)(r0 + nw * u) * ldd + c] = v[u];
        }
    }
}

constexpr int kRowsPerThread = kMaxRows / kThreads;

// The pass columns j0 .. j0 + kPB - 1 of the thread's rows tid + kThreads u
// (u < nri), as one vector per row (so that a column picked by a run-time
// index stays in registers), every load issued before any is used; rows past
// m are clamped, and a group that would start past ldw is clamped (it then
// holds no column of the pass: j0 + 4 h < n <= ldw for every column the pass
// has).
typedef uint32_t vpu __attribute__((ext_vector_type(kPB)));
static_assert(kPB == 16, "the pass columns are four 16-byte groups");

__device__ __forceinline__ void load_pass_cols(const gu32* W, int ldw, int m, int nri, int j0,
                                               vpu (&raw)[kRowsPerThread]) {
    v4u g[kRowsPerThread][4];
#pragma unroll
    for (int u = 0; u < kRowsPerThread; ++u) {
        const gu32* rp = W + (int64_t)min((int)threadIdx.x + kThreads * min(u, nri - 1), m - 1) * ldw;
#pragma unroll
        for (int h = 0; h < 4; ++h) g[u][h] = *(const gu4*)(rp + min(j0 + 4 * h, ldw - 4));
    }
#pragma unroll
    for (int u = 0; u < kRowsPerThread; ++u)
        raw[u] = __builtin_shufflevector(
            __builtin_shufflevector(g[u][0], g[u][1], 0, 1, 2, 3, 4, 5, 6, 7),
            __builtin_shufflevector(g[u][2], g[u][3], 0, 1, 2, 3, 4, 5, 6, 7), 0, 1, 2, 3, 4, 5, 6,
            7, 8, 9, 10, 11, 12, 13, 14, 15);
}

// Pivot search of a pass by one wave; returns the number of pivots (the same
// in every lane) and records them.  The pivot of column c is the first
// candidate row, in row order, whose value at c after eliminating the pass's
// earlier pivots is non-zero.  The first kWin candidate rows (the window) are
// kept reduced in registers, fraction-free (r <- d r - f q on the later
// columns: the zero pattern is that of the normalised elimination, which is
// all the search needs); lane L holds columns 4 (L % 4) .. 4 (L % 4) + 3 of
// window row L / 4, so a column costs a ballot and at most four updates per
// lane.  Only candidates that are non-zero somewhere in the pass's columns
// are considered (a zero row stays zero).  When every live window row is
// zero at c and such candidates remain after the window, those are scanned
// 64 at a time, each replaying the pass's pivots so far on its pass-start
// values (every pivot's panel row, reduced by the pivots before it, is kept in
// LDS); window rows are zero at c, so such a pivot changes nothing in the
// window.
constexpr int kWin = 16;
static_assert(kWin * 4 == 64 && kPB == 16, "window: 16 rows by 4 groups of 4 columns");

__device__ int search_pass(const SysDesc& d, BatchLds& L, int j0, int bw, int rank) {
    const int lane = threadIdx.x & 63, slot = lane >> 2, g = lane & 3;
    const int m = d.m;
    const FieldConst F = d.F;
    // the candidates that can give a pivot (a row that is zero at every
    // column of the pass stays zero), in row order: the first kWin form the
    // window, the others are listed for the scans
    int nlist = 0;
    for (int r0 = 0; r0 < m; r0 += 64) {
        const int r = r0 + lane;
        const bool c = r < m && L.piv[r] == 0 && L.nz[r];
        const uint64_t b = __ballot(c);
        const int pos = nlist + (int)__popcll(b & ((1ull << lane) - 1ull));
        if (c) {
            if (pos < kWin)
                L.win[pos] = r;
            else
                L.beyond[pos - kWin] = (int16_t)r;
        }
        nlist += (int)__popcll(b);
    }
    if (nlist == 0) return 0;
    const int nwin = min(nlist, kWin), nbeyond = nlist - nwin;
    bool live = slot < nwin;
    const int wr = L.win[min(slot, nwin - 1)];
    const v4u x0 = *(const v4u*)&g_mult[wr * kPB + 4 * g];  // pass-start values
    v4u x = x0;
    int np = 0, nslow = 0;  // nslow: pivots taken from the listed rows
    for (int c = 0; c < bw && rank + np < m; ++c) {
        const int gc = c >> 2, ec = c & 3;
        const uint32_t xc = x[ec];
        const uint64_t b = __ballot(live && g == gc && xc != 0u);
        int q = -1;
        uint32_t dq = 0u;
        if (b != 0ull) {
            const int ql = (int)__builtin_ctzll(b), rq = ql >> 2;
            q = L.win[rq];
            dq = __builtin_amdgcn_readlane(xc, ql);
            v4u U;
#pragma unroll
            for (int e = 0; e < 4; ++e) U[e] = __shfl(x[e], 4 * rq + g);
            const uint32_t f = __shfl(xc, 4 * slot + gc);
            if (slot == rq) {
                *(v4u*)&L.upan[np * kPB + 4 * g] = x;
                *(v4u*)&L.mst[np * kPB + 4 * g] = x0;
                live = false;
            }
            if (live && f != 0u) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (4 * g + e > c)
                        x[e] = mul_sub_mod((double)dq, x[e], (double)f, (double)U[e], F);
            }
        } else if (nbeyond > nslow) {
            {
                for (int i0 = 0; i0 < nbeyond; i0 += 64) {
                    const int r = L.beyond[min(i0 + lane, nbeyond - 1)];
                    const bool cand = i0 + lane < nbeyond && L.piv[r] == 0;
                    const vpu y0 = *(const vpu*)&g_mult[r * kPB];  // pass-start values
                    vpu y = y0;
                    for (int sp = 0; sp < np; ++sp) {
                        const int ps = L.upc[sp];
                        const uint32_t f = y[ps];
                        if (f == 0u) continue;
                        const double ds = (double)L.ud[sp];
#pragma unroll
                        for (int cc = 0; cc < kPB; ++cc)
                            if (cc > ps)
                                y[cc] = mul_sub_mod(ds, y[cc], (double)f, (double)L.upan[sp * kPB + cc], F);
                    }
                    const uint64_t b2 = __ballot(cand && y[c] != 0u);
                    if (b2 != 0ull) {
                        const int ql = (int)__builtin_ctzll(b2);
                        q = __builtin_amdgcn_readlane(r, ql);
                        dq = __builtin_amdgcn_readlane(y[c], ql);
                        if (lane == ql) {
                            *(vpu*)&L.upan[np * kPB] = y;
                            *(vpu*)&L.mst[np * kPB] = y0;
                        }
                        ++nslow;
                        break;
                    }
                }
            }
        }
        if (q < 0) continue;  // free column
        if (lane == 0) {
            L.piv[q] = 2;
            L.pt[q] = (int8_t)np;
            L.pivrow[rank + np] = (int16_t)q;
            L.pivcol[rank + np] = (int16_t)(j0 + c);
            L.upc[np] = c;
            L.ud[np] = dq;
        }
        ++np;
    }
    return np;
}

__device__ void solve_one(const SysDesc& d, BatchLds& L) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = d.m, n = d.n, k = d.k, ncols = n + k, ldw = d.ldw;
    const FieldConst F = d.F;
    gu32* W = (gu32*)d.W;
    gu32* PN = W + (int64_t)m * ldw;  // the pass's reduced pivot rows
    gu32* X = (gu32*)d.X;
    // stage [A | B] (padding columns zero)
    if (n > 0) copy_block(W, ldw, (const gu32*)d.A, d.lda, m, n);
    if (k > 0) copy_block(W + n, ldw, (const gu32*)d.B, d.ldb, m, k);
    for (int r = tid; r < m; r += kThreads)
        for (int c = ncols; c < ldw; ++c) W[(int64_t)r * ldw + c] = 0u;
    for (int r = tid; r < m; r += kThreads) L.piv[r] = 0;
    __threadfence_block();
    __syncthreads();
    const int nri = (m + kThreads - 1) / kThreads;  // rows per thread: tid + kThreads u
    int rank = 0, npass = 0;
    for (int j0 = 0; j0 < n && rank < m; j0 += kPB) {
        const int bw = min(kPB, n - j0);
        // 1. the pass's pivots, found by wave 0, among the candidate rows that
        // are non-zero somewhere in the pass's columns.  The pass's columns of
        // every row are loaded once, into the multiplier array (the search
        // reads them there, and they become the multipliers in place).
        {
            vpu raw[kRowsPerThread];
            load_pass_cols(W, ldw, m, nri, j0, raw);
#pragma unroll
            for (int u = 0; u < kRowsPerThread; ++u) {
                const int r = tid + kThreads * u;
                if (u >= nri || r >= m) break;
                bool nz = false;
#pragma unroll
                for (int c = 0; c < kPB; ++c) nz |= c < bw && raw[u][c] != 0u;
                L.nz[r] = nz ? 1 : 0;
                *(vpu*)&g_mult[r * kPB] = raw[u];
            }
        }
        __syncthreads();
        if (wave == 0) {
            const int npw = search_pass(d, L, j0, bw, rank);
            if (lane == 0) L.npp[(j0 / kPB) & 1] = npw;
        }
        __syncthreads();
        const int np = L.npp[(j0 / kPB) & 1];
        if (np == 0) continue;
        if (tid == 0) L.pstart[npass] = (int16_t)rank;
        ++npass;
        // coefficients of the reduced pivot rows (wave 0), and the candidate
        // rows' multipliers: their pass-start values at the pass's pivot
        // columns (zero for every pivot row), picked in place from the pass
        // columns each thread stored for its own rows
        if (wave == 0) pivot_block_inverse(d, L, rank, np);
        {
            int pc[kPB];
#pragma unroll
            for (int t = 0; t < kPB; ++t)
                pc[t] = __builtin_amdgcn_readfirstlane(t < np ? L.pivcol[rank + t] - j0 : 0);
#pragma unroll
            for (int u = 0; u < kRowsPerThread; ++u) {
                const int r = tid + kThreads * u;
                if (u >= nri || r >= m) break;
                const bool live = L.piv[r] == 0;
                const vpu raw = *(const vpu*)&g_mult[r * kPB];
                vpu a;
#pragma unroll
                for (int t = 0; t < kPB; ++t) a[t] = live && t < np ? raw[pc[t]] : 0u;
                *(vpu*)&g_mult[r * kPB] = a;
            }
        }
        __syncthreads();
        // 2. PN_t = sum_s T[t][s] row_{q_s} over 4-column groups from c0.  Only
        // the columns after the pass are needed from here on (later passes
        // search there; the outputs read the right-hand sides), so steps 2 and
        // 3 start at the 32-aligned column at or before the first column after
        // the pass (rows are 128-byte aligned, so every strip of stores covers
        // whole cache lines).
        const int c0 = min(j0 + kPB, n) & ~31;
        const int ngroups = (ncols - c0 + 3) >> 2;
        // (the terms in halves of 8, every load of a half issued first: beyond
        // np the coefficients are zero and the row index is clamped to pivot 0)
        for (int i = tid; i < np * ngroups; i += kThreads) {
            const int t = i / ngroups, c = c0 + 4 * (i % ngroups);
            double s1[4] = {0.0, 0.0, 0.0, 0.0}, s0[4] = {0.0, 0.0, 0.0, 0.0};
            for (int s8 = 0; s8 < kPB; s8 += 8) {
                v4u wv[8];
#pragma unroll
                for (int h = 0; h < 8; ++h)
                    wv[h] = *(const gu4*)(W + (int64_t)L.pivrow[rank + (s8 + h < np ? s8 + h : 0)] * ldw + c);
#pragma unroll
                for (int h = 0; h < 8; ++h) {
                    const uint32_t tv = s8 + h < np ? L.T[t * kPB + s8 + h] : 0u;
                    const double hi = (double)(tv >> 16), lo = (double)(tv & 0xffffu);
                    const uint32_t w4[4] = {wv[h].x, wv[h].y, wv[h].z, wv[h].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        s1[e] = __fma_rn(hi, (double)w4[e], s1[e]);
                        s0[e] = __fma_rn(lo, (double)w4[e], s0[e]);
                    }
                }
            }
            uint32_t o[4];
            for (int e = 0; e < 4; ++e) o[e] = split_reduce(s1[e], s0[e], F);
            *(gu4*)(PN + (int64_t)t * ldw + c) = (v4u){o[0], o[1], o[2], o[3]};
        }
        __threadfence_block();
        __syncthreads();
        // 3. every candidate row with a non-zero multiplier updated, the
        // pass's pivot rows replaced by PN; the pivot rows of earlier passes
        // are left as they are (forward elimination, X by back-substitution)
        update_rows(d, L, PN, np, c0);
        __threadfence_block();
        __syncthreads();
        for (int r = tid; r < m; r += kThreads)
            if (L.piv[r] == 2) L.piv[r] = 1;
        rank += np;
        __syncthreads();
    }
    // outputs: rank, pivots (ascending by construction), consistency, X
    const int mn = min(m, n);
    if (tid == 0) *(gi32*)d.rank = rank;
    for (int s = tid; s < mn; s += kThreads) ((gi32*)d.pivots)[s] = s < rank ? L.pivcol[s] : -1;
    for (int t = tid; t < k; t += kThreads) L.cons[t] = 1;
    for (int64_t i = tid; i < (int64_t)n * k; i += kThreads) X[(i / k) * d.ldx + (i % k)] = 0u;
    __syncthreads();
    // a non-pivot row with a non-zero right-hand side entry makes its column
    // inconsistent (rows with loads in flight before the flags are written)
    for (int c0 = 0; c0 < k; c0 += 64) {
        const int t = c0 + lane, tc = min(t, k - 1);
        for (int r0 = wave; r0 < m; r0 += 4 * kStageRows) {
            uint32_t v[kStageRows];
#pragma unroll
            for (int u = 0; u < kStageRows; ++u)
                v[u] = W[(int64_t)min(r0 + 4 * u, m - 1) * ldw + n + tc];
#pragma unroll
            for (int u = 0; u < kStageRows; ++u) {
                const int r = r0 + 4 * u;
                if (r < m && t < k && L.piv[r] == 0 && v[u] != 0) L.cons[t] = 0;
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < k; t += kThreads) ((gu8*)d.consistent)[t] = L.cons[t];
    // X at the pivot columns, a pass at a time from the last.  A pivot row of
    // pass P holds P's reduced row (unit vectors at P's pivot columns, zeros at
    // earlier ones, never updated afterwards), so x_s = c_s - sum over the
    // later pivots s' of row_s[col_s'] x_s' (the back-substitution of the
    // echelon form, Sec. 5.2's solve).  G lanes of a wave share an output,
    // each summing every G-th later pivot in exact chunks of 8 split products
    // with the loads of a chunk in flight together.  Inconsistent columns of X
    // stay zero.
    if (tid == 0) L.pstart[npass] = (int16_t)rank;
    __syncthreads();
    for (int P = npass - 1; P >= 0; --P) {
        const int s0 = L.pstart[P], s1 = L.pstart[P + 1], later = rank - s1;
        const int nout = (s1 - s0) * k;
        int G = 64;
        while (G > 1 && nout * G > kThreads) G >>= 1;
        for (int o0 = 0; o0 < nout; o0 += kThreads / G) {
            const int o = o0 + tid / G, gi = tid % G;
            const int oc = min(o, nout - 1);
            const int s = s0 + oc / k, t = oc - (oc / k) * k;
            const gu32* urow = W + (int64_t)L.pivrow[s] * ldw;
            uint32_t acc = 0u;
            for (int i0 = gi; i0 < later; i0 += 8 * G) {
                uint32_t uv[8], xv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int col = L.pivcol[s1 + min(i0 + e * G, later - 1)];
                    uv[e] = urow[col];
                    xv[e] = X[(int64_t)col * d.ldx + t];
                }
                double h = 0.0, l = 0.0;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const double u = i0 + e * G < later ? (double)uv[e] : 0.0;
                    h = __fma_rn(u, (double)(xv[e] >> 16), h);
                    l = __fma_rn(u, (double)(xv[e] & 0xffffu), l);
                }
                acc = add_mod(acc, split_reduce(h, l, F), F.p);
            }
            for (int off = G >> 1; off > 0; off >>= 1) acc = add_mod(acc, __shfl_xor(acc, off), F.p);
            if (gi == 0 && o < nout)
                X[(int64_t)L.pivcol[s] * d.ldx + t] = L.cons[t] ? sub_mod(urow[n + t], acc, F.p) : 0u;
        }
        __threadfence_block();
        __syncthreads();
    }
}

// Persistent kernel: every workgroup takes the next system from the queue until
// the queue is exhausted (each workgroup exits once the counter passes count).
// Three waves per SIMD (at most 168 VGPRs; a few long-lived values spill
// outside the hot loops): with systems of up to 512 rows the LDS also allows
// three workgroups per CU, which hide each other's serial pivot chains.
__global__ __launch_bounds__(kThreads, 3) void batched_kernel(const SysDesc* sys, int32_t count,
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

// Words per workspace row: n + k rounded up to 32, so rows start on 128-byte
// boundaries.
static int64_t row_words(int64_t ncols) { return round_up(ncols > 0 ? ncols : 1, 32); }

bool batched_fits(int64_t m, int64_t n, int64_t k) {
    return m <= kMaxRows && n + k <= kMaxCols;
}

// Layout: [counter | descriptors | working regions]
size_t batched_workspace(const linac_system* sys, int32_t count) {
    size_t off = 256 + round_up((int64_t)count * sizeof(SysDesc), 256);
    for (int32_t i = 0; i < count; ++i) {
        const int64_t ldw = row_words(sys[i].n + sys[i].k);
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
        const int64_t ldw = row_words(sys[i].n + sys[i].k);
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
        d.ldw = (int32_t)row_words(s.n + s.k);
        d.pad = 0;
        d.F = make_field(s.p);
    }
}

int32_t batched_mult_rows(const linac_system* sys, int32_t count) {
    int32_t mx = 1;
    for (int32_t i = 0; i < count; ++i) mx = std::max(mx, sys[i].m);
    return (int32_t)round_up(mx, 64);
}

hipError_t batched_launch(void* ws, int32_t count, int32_t grid, int32_t mult_rows, hipStream_t s) {
    unsigned int* counter = (unsigned int*)ws;
    const SysDesc* desc = (const SysDesc*)((char*)ws + 256);
    const size_t dyn = (size_t)mult_rows * kPB * sizeof(uint32_t);
    hipError_t e = hipFuncSetAttribute((const void*)batched_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    hipLaunchKernelGGL(batched_kernel, dim3((unsigned)grid), dim3(kThreads), dyn, s, desc, count,
                       counter);
    return hipGetLastError();
}

void* batched_desc_ptr(void* ws) { return (char*)ws + 256; }

}  // namespace linac
