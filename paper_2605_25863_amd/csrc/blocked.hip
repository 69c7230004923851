// Blocked Gauss-Jordan elimination over F_p with an exact mod-p GEMM on MFMA.
//
// The paper finds its kernel bound by memory bandwidth and notes that larger
// gains need more arithmetic intensity (Sec. 3.4, Sec. 4.1.1).  Processing w
// pivot columns at a time turns the row update into a matrix product.
//
// Panel step for pivot columns [j0, j0 + w):
//  1. The panel columns of every row are copied to a side buffer PR next to a
//     w-column block E that starts at zero.
//  2. PR is reduced in leaves of 32 columns (leaf.hip): a pivot selection
//     picks the leaf's pivot rows and P^-1, and one MFMA product applies the
//     leaf to the rest of PR.  When row q becomes the pivot of local column s it
//     carries an implicit 1 in E[q][s], so the row operations applied to E
//     record, for every row r, the coefficients of its final value in terms of
//     the panel's pivot rows as they were at the panel start:
//        final_r = delta_r * row_r + E[r] . X_S,
//     with delta_r = 0 for the panel's pivot rows and 1 otherwise.  X_S holds
//     the pivot rows' trailing parts at the panel start (row s of X_S belongs
//     to the pivot of local column s; a free column gives a zero row).
//  3. The trailing columns of all rows are updated by that one product.
//
// Exactness of the product on int8 MFMA.  Every residue is first centred,
// x -> x - p when x > (p-1)/2, so |x| <= 2^30, then split into four signed
// base-256 digits in [-128, 127].  For y = X_S[k][c] the operand is
// pre-scaled: y_l = 256^l * y mod p for l = 0..3, each centred and split into
// digits b_{l,l'}.  With a_l the digits of E[r][k],
//    E[r][k] * y == sum_l a_l * y_l == sum_{l'} 256^{l'} sum_l a_l * b_{l,l'}  (mod p),
// so four int32 accumulators S_{l'} = sum_k sum_l a_l b_{l,l'} suffice (16
// int8 products per mod-p product).  |S_{l'}| <= 4 * K * 2^14 = K * 2^16 < 2^31
// for K < 2^15, and T = S_0 + 2^8 S_1 + 2^16 S_2 + 2^24 S_3 stays below 2^50 in
// magnitude for K <= 512, so it is exact in FP64 and one reduction mod p ends
// the panel.  For p < 2^21 the centred residues are below 2^20 and the product
// can instead run on FP64 MFMA directly: every partial sum is below K * 2^40,
// exact while K <= 8192.
#include "internal.h"

namespace linac {

namespace {

constexpr int kThreads = 256;
constexpr int kTileRows = 32;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int32_t centre(uint32_t v, uint32_t p) {
    return v > (p - 1) / 2 ? (int32_t)v - (int32_t)p : (int32_t)v;
}

// Four signed base-256 digits of x (|x| <= 2^30), least significant first.
__device__ __forceinline__ void digits4(int32_t x, int8_t d[4]) {
    for (int l = 0; l < 4; ++l) {
        int8_t lo = (int8_t)(x & 0xff);
        d[l] = lo;
        x = (x - lo) >> 8;
    }
}

// A row-major matrix view (device pointer and leading dimension).
struct Mat {
    uint32_t* M;
    int64_t ld;
};

// Copy columns [c0, c0 + width) of src into dst (all of dst's other columns,
// including the transform block, set to zero).
__global__ __launch_bounds__(kThreads) void panel_extract_kernel(int32_t m, Mat src, int64_t c0,
                                                                 Mat dst, int32_t width) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t d0 = (int64_t)blockIdx.y * 256 + lane * 4;
    const int row0 = blockIdx.x * kTileRows + wave * 8;
    for (int rr = 0; rr < 8; ++rr) {
        const int r = row0 + rr;
        if (r >= m || d0 >= dst.ld) continue;
        uint32_t v[4];
        for (int e = 0; e < 4; ++e) {
            const int64_t c = d0 + e;
            v[e] = c < width ? src.M[(int64_t)r * src.ld + c0 + c] : 0u;
        }
        *(uint4*)(dst.M + (int64_t)r * dst.ld + d0) = make_uint4(v[0], v[1], v[2], v[3]);
    }
}

// Row k of X_S: the pivot row of bookkeeping column gslot0 + k, columns
// [col0, col0 + N) of src, with the implicit 1 of an enclosing transform block
// at column inj0 + k (inj0 < 0: none); zero for a free column.
__device__ __forceinline__ uint32_t xs_value(const PlainArgs& w, Mat src, int32_t gslot0,
                                             int32_t wj, int64_t col0, int64_t N, int64_t inj0,
                                             int k, int64_t col) {
    if (k >= wj || col >= N) return 0u;
    const unsigned long long s = w.slots[gslot0 + k];
    if (s == kNoPivot) return 0u;
    if (inj0 >= 0 && col0 + col == inj0 + k) return 1u;
    return src.M[(int64_t)(s >> 32) * src.ld + col0 + col];
}

// B operand: X_S pre-scaled by 256^l and split into digits, stored in the lane
// order of the 32x32x32 int8 MFMA: fragment (cb, kb, plane = 4*l + l') is 64
// lanes x 16 bytes; lane L holds column cb*32 + L%32 and rows
// k = kb*32 + 16*(L/32) + i, i = 0..15.
__global__ void build_b_kernel(PlainArgs w, Mat src, int32_t gslot0, int32_t wj, int64_t col0,
                               int64_t N, int64_t inj0, int32_t KB, int64_t NB, int8_t* Bfrag,
                               uint4 scale) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= NB * KB * 64) return;
    const int L = (int)(gid & 63);
    const int64_t t = gid >> 6;
    const int kb = (int)(t % KB);
    const int64_t cb = t / KB;
    const int64_t col = cb * 32 + (L & 31);
    const uint32_t p = w.F.p;
    const uint32_t sc[4] = {scale.x, scale.y, scale.z, scale.w};
    int8_t out[16][16];  // [plane][i]
    for (int i = 0; i < 16; ++i) {
        const int k = kb * 32 + 16 * (L >> 5) + i;
        const uint32_t y = xs_value(w, src, gslot0, wj, col0, N, inj0, k, col);
        for (int l = 0; l < 4; ++l) {
            const uint32_t yl = l == 0 ? y : mul_mod(y, sc[l], w.F);
            int8_t d[4];
            digits4(centre(yl, p), d);
            for (int lp = 0; lp < 4; ++lp) out[4 * l + lp][i] = d[lp];
        }
    }
    int8_t* base = Bfrag + ((cb * KB + kb) * 16) * 1024 + L * 16;
    for (int pl = 0; pl < 16; ++pl) {
        v4i v;
        __builtin_memcpy(&v, out[pl], 16);
        *(v4i*)(base + pl * 1024) = v;
    }
}

// A operand: the transform block E = ebuf columns [ecol0, ecol0 + wj), split
// into digits, in MFMA lane order: fragment (rb, kb, l) is 64 lanes x 16 bytes;
// lane L holds row rb*32 + L%32 and k = kb*32 + 16*(L/32) + i.
__global__ void build_a_kernel(PlainArgs w, Mat ebuf, int64_t ecol0, int32_t wj, int32_t KB,
                               int64_t MB, int8_t* Afrag) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= MB * KB * 64) return;
    const int L = (int)(gid & 63);
    const int64_t t = gid >> 6;
    const int kb = (int)(t % KB);
    const int64_t rb = t / KB;
    const int64_t row = rb * 32 + (L & 31);
    const uint32_t p = w.F.p;
    int8_t out[4][16];
    for (int i = 0; i < 16; ++i) {
        const int k = kb * 32 + 16 * (L >> 5) + i;
        uint32_t e = (row < w.m && k < wj) ? ebuf.M[row * ebuf.ld + ecol0 + k] : 0u;
        int8_t d[4];
        digits4(centre(e, p), d);
        for (int l = 0; l < 4; ++l) out[l][i] = d[l];
    }
    int8_t* base = Afrag + ((rb * KB + kb) * 4) * 1024 + L * 16;
    for (int l = 0; l < 4; ++l) {
        v4i v;
        __builtin_memcpy(&v, out[l], 16);
        *(v4i*)(base + l * 1024) = v;
    }
}

// T = S0 + 2^8 S1 + 2^16 S2 + 2^24 S3 (exact in FP64) reduced mod p.
__device__ __forceinline__ uint32_t fold_mod(int32_t s0, int32_t s1, int32_t s2, int32_t s3,
                                             const FieldConst& F) {
    double T = __fma_rn(16777216.0, (double)s3,
                        __fma_rn(65536.0, (double)s2, __fma_rn(256.0, (double)s1, (double)s0)));
    double q = floor(T * F.pinv);
    double r = __fma_rn(-q, F.dp, T);
    if (r < 0.0) r += F.dp;
    if (r >= F.dp) r -= F.dp;
    if (r < 0.0) r += F.dp;
    return (uint32_t)r;
}

// Product update C = delta * C + E . X_S (mod p) on int8 MFMA (C = dst columns
// [col0, col0 + N); delta = 0 for the rows that became pivots of this panel).
// Block: 4 waves; wave v owns rows [(4*bx + v)*32, +32) and the block's 64
// columns (two 32-column blocks).  The B fragments of a k-block (2 x 16 planes
// x 1 KB) are shared through LDS, double-buffered: the next k-block is loaded
// into registers while MFMAs run on the current one, then written to the other
// buffer.  A fragments (each wave needs only its own rows) are prefetched into
// registers.
// With grid.x = row tiles and a multiple of 8 of them, all blocks of one row
// tile run on the same XCD, so each XCD's L2 holds one eighth of the A operand.
__global__ __launch_bounds__(kThreads, 2) void gemm_i8_kernel(PlainArgs w, Mat dst, int64_t col0,
                                                              int64_t N, const int8_t* Afrag,
                                                              const int8_t* Bfrag, int32_t KB,
                                                              int32_t fresh_lo, int32_t fresh_hi) {
    __shared__ v4i sB[2][2 * 16 * 64];  // 2 x 32 KB
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t rb = (int64_t)blockIdx.x * 4 + wave;
    const int64_t cb0 = (int64_t)blockIdx.y * 2;
    const int64_t NB = ceil_div(N, 32);
    // each wave moves 8 of the 32 B fragments of a k-block; column blocks past
    // the end read a valid block (their output columns are never written)
    const int8_t* bsrc[8];
    for (int i = 0; i < 8; ++i) {
        const int f = wave * 8 + i;
        int64_t cb = cb0 + f / 16;
        if (cb >= NB) cb = NB - 1;
        bsrc[i] = Bfrag + (cb * KB * 16 + (f % 16)) * 1024 + lane * 16;
    }
    const int8_t* asrc = Afrag + (rb * KB * 4) * 1024 + lane * 16;
    v16i acc[2][4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 4; ++b)
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;
    v4i stage[8], af[4], an[4];
    for (int i = 0; i < 8; ++i) stage[i] = *(const v4i*)bsrc[i];
    for (int l = 0; l < 4; ++l) af[l] = *(const v4i*)(asrc + l * 1024);
    for (int i = 0; i < 8; ++i) sB[0][(wave * 8 + i) * 64 + lane] = stage[i];
    __builtin_amdgcn_s_waitcnt(0);  // nothing in flight at the loop head
    __syncthreads();
    for (int kb = 0; kb < KB; ++kb) {
        const bool more = kb + 1 < KB;
        if (more) {  // next k-block in flight while this one computes
            for (int i = 0; i < 8; ++i)
                stage[i] = *(const v4i*)(bsrc[i] + (int64_t)(kb + 1) * 16 * 1024);
            for (int l = 0; l < 4; ++l)
                an[l] = *(const v4i*)(asrc + ((int64_t)(kb + 1) * 4 + l) * 1024);
        }
        const v4i* sb = sB[kb & 1];
        for (int cbi = 0; cbi < 2; ++cbi) {
            for (int l = 0; l < 4; ++l) {
                v4i bf[4];
                for (int lp = 0; lp < 4; ++lp) bf[lp] = sb[(cbi * 16 + 4 * l + lp) * 64 + lane];
                for (int lp = 0; lp < 4; ++lp)
                    acc[cbi][lp] =
                        __builtin_amdgcn_mfma_i32_32x32x32_i8(af[l], bf[lp], acc[cbi][lp], 0, 0, 0);
            }
        }
        if (more) {
            v4i* nb = sB[(kb + 1) & 1];
            for (int i = 0; i < 8; ++i) nb[(wave * 8 + i) * 64 + lane] = stage[i];
            for (int l = 0; l < 4; ++l) af[l] = an[l];
        }
        __syncthreads();
    }
    // epilogue: 32x32 accumulator layout: lane L holds column L%32 and rows
    // 8*(r/4) + 4*(L/32) + r%4 for r = 0..15.  All loads are issued before the
    // first store so their latencies overlap.
    bool fresh[16];
    for (int r = 0; r < 16; ++r) {
        const int64_t row = rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int rc = row < w.m ? w.rowcol[row] : -1;
        fresh[r] = rc >= fresh_lo && rc < fresh_hi;  // a pivot row of this panel
    }
    uint32_t cur[2][16];
    for (int cbi = 0; cbi < 2; ++cbi) {
        const int64_t col = (cb0 + cbi) * 32 + (lane & 31);
        for (int r = 0; r < 16; ++r) {
            const int64_t row = rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            cur[cbi][r] = (col < N && row < w.m && !fresh[r])
                              ? __builtin_nontemporal_load(dst.M + row * dst.ld + col0 + col)
                              : 0u;
        }
    }
    for (int cbi = 0; cbi < 2; ++cbi) {
        const int64_t col = (cb0 + cbi) * 32 + (lane & 31);
        if (col >= N) continue;
        for (int r = 0; r < 16; ++r) {
            const int64_t row = rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (row >= w.m) continue;
            const uint32_t t = fold_mod(acc[cbi][0][r], acc[cbi][1][r], acc[cbi][2][r],
                                        acc[cbi][3][r], w.F);
            dst.M[row * dst.ld + col0 + col] = fresh[r] ? t : add_mod(cur[cbi][r], t, w.F.p);
        }
    }
}

// FP64 operands for p < 2^21: centred residues as doubles in the lane order of
// the 16x16x4 FP64 MFMA.  A fragment (rb, kb): lane L holds E[rb*16 + L%16]
// [kb*4 + L/16]; B fragment (cb, kb): lane L holds X_S[kb*4 + L/16][cb*16 + L%16].
__global__ void build_a_f64_kernel(PlainArgs w, Mat ebuf, int64_t ecol0, int32_t wj, int32_t KB,
                                   int64_t MB, double* Afrag) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= MB * KB * 64) return;
    const int L = (int)(gid & 63);
    const int64_t t = gid >> 6;
    const int kb = (int)(t % KB);
    const int64_t rb = t / KB;
    const int64_t row = rb * 16 + (L & 15);
    const int k = kb * 4 + (L >> 4);
    const uint32_t e = (row < w.m && k < wj) ? ebuf.M[row * ebuf.ld + ecol0 + k] : 0u;
    Afrag[gid] = (double)centre(e, w.F.p);
}

__global__ void build_b_f64_kernel(PlainArgs w, Mat src, int32_t gslot0, int32_t wj, int64_t col0,
                                   int64_t N, int64_t inj0, int32_t KB, int64_t NB, double* Bfrag) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= NB * KB * 64) return;
    const int L = (int)(gid & 63);
    const int64_t t = gid >> 6;
    const int kb = (int)(t % KB);
    const int64_t cb = t / KB;
    const int64_t col = cb * 16 + (L & 15);
    const int k = kb * 4 + (L >> 4);
    const uint32_t y = xs_value(w, src, gslot0, wj, col0, N, inj0, k, col);
    Bfrag[gid] = (double)centre(y, w.F.p);
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Trailing update on FP64 MFMA: block = 4 waves over a 64 x 64 tile, each wave
// a 32 x 32 quarter (2 x 2 MFMA blocks of 16 x 16).  Accumulator layout of the
// 16x16x4 FP64 MFMA (checked on gfx950): lane L holds column L%16 and rows
// L/16 + 4*i, i = 0..3 (interleaved, unlike the int8 and FP32 shapes).
__global__ __launch_bounds__(kThreads) void gemm_f64_kernel(PlainArgs w, Mat dst, int64_t col0,
                                                            int64_t N, const double* Afrag,
                                                            const double* Bfrag, int32_t KB,
                                                            int64_t NB, int32_t fresh_lo,
                                                            int32_t fresh_hi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t rb0 = (int64_t)blockIdx.x * 4 + (wave >> 1) * 2;
    const int64_t cb0 = (int64_t)blockIdx.y * 4 + (wave & 1) * 2;
    v4d acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int kb = 0; kb < KB; ++kb) {
        double af[2], bf[2];
        for (int a = 0; a < 2; ++a) af[a] = Afrag[((rb0 + a) * KB + kb) * 64 + lane];
        for (int b = 0; b < 2; ++b)
            bf[b] = cb0 + b < NB ? Bfrag[((cb0 + b) * KB + kb) * 64 + lane] : 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    uint32_t cur[2][2][4];
    bool fresh[2][4];
    for (int a = 0; a < 2; ++a)
        for (int i = 0; i < 4; ++i) {
            const int64_t row = (rb0 + a) * 16 + (lane >> 4) + 4 * i;
            const int rc = row < w.m ? w.rowcol[row] : -1;
            fresh[a][i] = rc >= fresh_lo && rc < fresh_hi;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int64_t col = (cb0 + b) * 16 + (lane & 15);
            for (int i = 0; i < 4; ++i) {
                const int64_t row = (rb0 + a) * 16 + (lane >> 4) + 4 * i;
                cur[a][b][i] = (col < N && row < w.m && !fresh[a][i])
                                   ? dst.M[row * dst.ld + col0 + col]
                                   : 0u;
            }
        }
    for (int a = 0; a < 2; ++a) {
        for (int b = 0; b < 2; ++b) {
            const int64_t col = (cb0 + b) * 16 + (lane & 15);
            if (col >= N) continue;
            for (int i = 0; i < 4; ++i) {
                const int64_t row = (rb0 + a) * 16 + (lane >> 4) + 4 * i;
                if (row >= w.m) continue;
                const double T = acc[a][b][i];  // exact: |T| < K * 2^40
                double q = floor(T * w.F.pinv);
                double r = __fma_rn(-q, w.F.dp, T);
                if (r < 0.0) r += w.F.dp;
                if (r >= w.F.dp) r -= w.F.dp;
                const uint32_t t = (uint32_t)r;
                dst.M[row * dst.ld + col0 + col] =
                    fresh[a][i] ? t : add_mod(cur[a][b][i], t, w.F.p);
            }
        }
    }
}

// Write columns [0, width) of src into dst columns [d0, d0 + width); pivot
// columns (bookkeeping columns gcol0 + js) become unit vectors.
__global__ void panel_writeback_kernel(PlainArgs w, Mat src, Mat dst, int64_t d0, int32_t width,
                                       int32_t gcol0) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)w.m * width) return;
    const int64_t r = gid / width;
    const int js = (int)(gid % width);
    const int s = w.colpiv[gcol0 + js];
    uint32_t v;
    if (s >= 0) v = (w.pivrow[s] == r) ? 1u : 0u;
    else v = src.M[r * src.ld + js];
    dst.M[r * dst.ld + d0 + js] = v;
}

constexpr int32_t kLeaf = 32;  // inner panel width of the two-level reduction

struct Blocked {
    PlainArgs w;  // the working matrix and the bookkeeping (shared with the plain path)
    Mat PR;       // outer panel [panel | E]
    int8_t* Afrag;
    int8_t* Bfrag;
    LeafState leaf;
    int32_t panel;
};

// Workspace after the plain layout: PR (m x ldpr), the operand fragments (sized
// for the larger of the int8 layouts, A 4 B and B 16 B per element, and the
// FP64 ones, 8 B each, for both the trailing product and the leaf products) and
// the leaf selection state.
size_t carve_blocked(void* ws, int64_t m, int64_t n, int64_t k, int32_t panel, Blocked* b) {
    const size_t base = plain_workspace(m, n, k);
    Carver c(ws ? (char*)ws + base : nullptr);
    const int64_t ldpr = round_up(2 * (int64_t)panel, 64);
    const int64_t Kp = round_up(panel, 32);
    const int64_t Mp = round_up(m > 0 ? m : 1, 128);
    const int64_t Np = round_up(n + k > 0 ? n + k : 1, 64);
    const int64_t Nl = round_up(2 * (int64_t)panel + kLeaf, 64);  // leaf product columns
    const int64_t abytes = Mp * (Kp > kLeaf ? Kp : kLeaf) * 8;
    const int64_t bbytes = (Np * Kp > Nl * kLeaf ? Np * Kp : Nl * kLeaf) * 16;
    uint32_t* PR = c.take<uint32_t>(m * ldpr);
    int8_t* A = c.take<int8_t>(abytes);
    int8_t* B = c.take<int8_t>(bbytes);
    LeafState ls;
    leaf_carve(c, m, &ls);
    if (b) {
        plain_carve(ws, m, n, k, b->w);
        b->PR = Mat{PR, ldpr};
        b->Afrag = A;
        b->Bfrag = B;
        b->leaf = ls;
        b->panel = panel;
    }
    return base + c.off + 256;
}

// The product kernel: dst columns [col0, col0 + N) of every row become
// delta * C + A . B from the prepared fragments (K = 32 KB for int8, 4 KB for
// FP64); delta = 0 for the rows whose pivot column lies in [fresh_lo, fresh_hi).
hipError_t run_product(const Blocked& b, const PlainArgs& w, bool fp64, Mat dst, int64_t col0,
                       int64_t N, int32_t KB, int32_t fresh_lo, int32_t fresh_hi, hipStream_t s,
                       LaunchTimer& lt, int kind) {
    const int64_t m = w.m;
    lt.before(kind);
    if (fp64) {
        hipLaunchKernelGGL(gemm_f64_kernel, dim3((unsigned)ceil_div(m, 64), (unsigned)ceil_div(N, 64)),
                           dim3(kThreads), 0, s, w, dst, col0, N, (const double*)b.Afrag,
                           (const double*)b.Bfrag, KB, ceil_div(N, 16), fresh_lo, fresh_hi);
    } else {
        hipLaunchKernelGGL(gemm_i8_kernel, dim3((unsigned)ceil_div(m, 128), (unsigned)ceil_div(N, 64)),
                           dim3(kThreads), 0, s, w, dst, col0, N, b.Afrag, b.Bfrag, KB, fresh_lo,
                           fresh_hi);
    }
    lt.after();
    return hipGetLastError();
}

// Trailing update: dst columns [col0, col0 + N) of every row become
// delta * C + E . X_S, where E is PR's transform block (columns [wj, 2 wj)) and
// X_S the pivot rows of bookkeeping columns [j0, j0 + wj) read from dst (before
// the update), with delta = 0 for the panel's pivot rows.
hipError_t trailing_product(const Blocked& b, const PlainArgs& w, bool fp64, Mat dst, int32_t j0,
                            int32_t wj, int64_t col0, int64_t N, hipStream_t s, LaunchTimer& lt) {
    const int64_t m = w.m;
    if (N <= 0) return hipSuccess;
    lt.before(LINAC_KERNEL_OPERANDS);
    int32_t KB;
    if (fp64) {
        KB = (int32_t)ceil_div(wj, 4);
        const int64_t NB = ceil_div(N, 16);
        const int64_t MB = ceil_div(m, 64) * 4;
        hipLaunchKernelGGL(build_b_f64_kernel, dim3((unsigned)ceil_div(NB * KB * 64, 256)), dim3(256),
                           0, s, w, dst, j0, wj, col0, N, (int64_t)-1, KB, NB, (double*)b.Bfrag);
        hipLaunchKernelGGL(build_a_f64_kernel, dim3((unsigned)ceil_div(MB * KB * 64, 256)), dim3(256),
                           0, s, w, b.PR, (int64_t)wj, wj, KB, MB, (double*)b.Afrag);
    } else {
        KB = (int32_t)ceil_div(wj, 32);
        const int64_t NB = ceil_div(N, 32);
        const int64_t MB = ceil_div(m, 128) * 4;
        uint32_t sc[4] = {1, 0, 0, 0};
        for (int l = 1; l < 4; ++l) sc[l] = (uint32_t)(((uint64_t)sc[l - 1] * 256u) % w.F.p);
        const uint4 scale = make_uint4(sc[0], sc[1], sc[2], sc[3]);
        hipLaunchKernelGGL(build_b_kernel, dim3((unsigned)ceil_div(NB * KB * 64, 256)), dim3(256), 0,
                           s, w, dst, j0, wj, col0, N, (int64_t)-1, KB, NB, b.Bfrag, scale);
        hipLaunchKernelGGL(build_a_kernel, dim3((unsigned)ceil_div(MB * KB * 64, 256)), dim3(256), 0,
                           s, w, b.PR, (int64_t)wj, wj, KB, MB, b.Afrag);
    }
    lt.after();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return run_product(b, w, fp64, dst, col0, N, KB, j0, j0 + wj, s, lt,
                       LINAC_KERNEL_TRAIL_PRODUCT);
}

}  // namespace

size_t blocked_workspace(int64_t m, int64_t n, int64_t k, int32_t panel) {
    return carve_blocked(nullptr, m, n, k, panel, nullptr);
}

// Two-level blocked Gauss-Jordan.  Outer panels of `panel` columns; inside a
// panel, leaves of kLeaf columns: a pivot selection (leaf.hip) and one MFMA
// product with K = kLeaf that applies the leaf to the rest of the panel buffer
// PR (the leaf's own columns, the panel columns after it and the outer
// transform block, where the leaf's pivots carry their implicit 1).  After the
// last leaf, PR holds the reduced panel and the panel transform, and one MFMA
// product with K = panel updates all trailing columns of W.
hipError_t blocked_eliminate(void* ws, int64_t m, int64_t n, int64_t k, int32_t panel, bool fp64,
                             PlainArgs& out, const linac_opts* opts, hipStream_t s) {
    Blocked b;
    carve_blocked(ws, m, n, k, panel, &b);
    b.w.F = out.F;
    b.w.resolved = 1;
    out = b.w;
    const PlainArgs& w = b.w;
    if (m == 0) return hipSuccess;
    const int64_t ncols = n + k;
    const unsigned tiles = (unsigned)ceil_div(m, kTileRows);
    const Mat Wm{w.W, w.ld};
    int64_t outer_products = 0;
    LaunchTimer lt(opts, s);
    hipError_t e = leaf_init(b.leaf, (int32_t)m, s);
    int32_t leaf_index = 0;
    for (int32_t j0 = 0; j0 < n && e == hipSuccess; j0 += panel) {
        const int32_t wj = (int32_t)(n - j0 < panel ? n - j0 : panel);
        hipLaunchKernelGGL(panel_extract_kernel, dim3(tiles, (unsigned)ceil_div(b.PR.ld, 256)),
                           dim3(kThreads), 0, s, w.m, Wm, (int64_t)j0, b.PR, wj);
        for (int32_t l0 = 0; l0 < wj && e == hipSuccess; l0 += kLeaf) {
            const int32_t wl = wj - l0 < kLeaf ? wj - l0 : kLeaf;
            const int32_t parity = leaf_index & 1;
            // the leaf's own columns, the panel columns after it and the transform
            // block up to this leaf's pivots (beyond it every row is still zero)
            const int64_t N = (int64_t)wj + wl;
            lt.before(LINAC_KERNEL_SELECT);
            e = leaf_select(w, b.leaf, b.PR.M, b.PR.ld, l0, wl, j0 + l0, parity, s);
            lt.after();
            if (e != hipSuccess) break;
            lt.before(LINAC_KERNEL_OPERANDS);
            e = leaf_operands(w, b.leaf, b.PR.M, b.PR.ld, l0, wl, wj, j0 + l0, N, parity, fp64,
                              b.Afrag, b.Bfrag, s);
            lt.after();
            if (e != hipSuccess) break;
            e = run_product(b, w, fp64, b.PR, (int64_t)l0, N, fp64 ? kLeaf / 4 : 1, j0 + l0,
                            j0 + l0 + wl, s, lt, LINAC_KERNEL_LEAF_PRODUCT);
            ++leaf_index;
        }
        if (e != hipSuccess) break;
        const int64_t N = ncols - (j0 + wj);
        if (N > 0) {
            if (opts && opts->ev_begin && outer_products == 0) (void)hipEventRecord(opts->ev_begin, s);
            e = trailing_product(b, w, fp64, Wm, j0, wj, (int64_t)j0 + wj, N, s, lt);
            ++outer_products;
        }
        hipLaunchKernelGGL(panel_writeback_kernel, dim3((unsigned)ceil_div(m * wj, 256)), dim3(256),
                           0, s, w, b.PR, Wm, (int64_t)j0, wj, j0);
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (opts && opts->ev_end && outer_products > 0) (void)hipEventRecord(opts->ev_end, s);
    if (opts && opts->dominant_launches) *opts->dominant_launches = outer_products;
    return e;
}

}  // namespace linac
