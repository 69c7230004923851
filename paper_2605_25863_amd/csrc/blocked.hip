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
// base-256 digits in [-128, 127]: x = sum_l 256^l x_l.  For an A entry a and
// a B entry b,
//    a * b = sum_{s=0..6} 256^s sum_{l + l' = s} a_l * b_l',
// so seven int32 accumulators S_s = sum_k sum_{l+l'=s} a_l b_l' (16 int8 MFMA
// products per mod-p product, at most four per group) give the product sum.
// |S_s| <= 4 * K * 2^14 < 2^31 for K < 2^15.  T_lo = S_0 + 2^8 S_1 + 2^16 S_2
// + 2^24 S_3 and T_hi = S_4 + 2^8 S_5 + 2^16 S_6 stay below 2^50 and 2^40 in
// magnitude for K <= 512, so both are exact in FP64, and the result is
// T_lo + (2^32 mod p) T_hi reduced mod p.  Both operands keep four digit
// planes, so the B operand (read by every block of a column) is no larger
// than A.  For p < 2^21 the centred residues are below 2^20 and the product
// can instead run on FP64 MFMA directly: every partial sum is below K * 2^40,
// exact while K <= 8192.
#include <type_traits>

#include "internal.h"
#include "leafprod.h"

namespace linac {

namespace {

constexpr int kThreads = 256;
constexpr int kTileRows = 32;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

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
    // all eight rows' loads first (128-bit where the four columns are inside
    // the panel: c0 and d0 are multiples of 4), then the stores
    uint4 v[8];
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
        const int64_t r = row0 + rr < m ? row0 + rr : m - 1;
        const uint32_t* srow = src.M + r * src.ld + c0;
        if (d0 + 3 < width) {
            v[rr] = *(const uint4*)(srow + d0);
        } else {
            uint32_t x[4];
            for (int e = 0; e < 4; ++e) x[e] = d0 + e < width ? srow[d0 + e] : 0u;
            v[rr] = make_uint4(x[0], x[1], x[2], x[3]);
        }
    }
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
        const int r = row0 + rr;
        if (r < m && d0 < dst.ld) *(uint4*)(dst.M + (int64_t)r * dst.ld + d0) = v[rr];
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

// B operand: X_S split into digits, stored in the lane order of the 32x32x32
// int8 MFMA: fragment (cb, kb, l') is 64 lanes x 16 bytes; lane L holds digit
// l' of column cb*32 + L%32 and rows k = kb*32 + 16*(L/32) + i, i = 0..15.
template <bool kNeg = false>  // (kNeg: fragments of -X_S)
__device__ __forceinline__ void build_b_at(const PlainArgs& w, Mat src, int32_t gslot0, int32_t wj, int64_t col0,
                                           int64_t N, int64_t inj0, int32_t KB, int64_t NB, int8_t* Bfrag,
                                           int64_t gid) {
    if (gid >= NB * KB * 64) return;
    const int L = (int)(gid & 63);
    const int64_t t = gid >> 6;
    const int kb = (int)(t % KB);
    const int64_t cb = t / KB;
    const int64_t col = cb * 32 + (L & 31);
    const uint32_t p = w.F.p;
    int8_t out[4][16];  // [digit][i]
    for (int i = 0; i < 16; ++i) {
        const int k = kb * 32 + 16 * (L >> 5) + i;
        int8_t d[4];
        const int32_t c = centre(xs_value(w, src, gslot0, wj, col0, N, inj0, k, col), p);
        digits4(kNeg ? -c : c, d);
        for (int l = 0; l < 4; ++l) out[l][i] = d[l];
    }
    int8_t* base = Bfrag + ((cb * KB + kb) * 4) * 1024 + L * 16;
    for (int l = 0; l < 4; ++l) {
        v4i v;
        __builtin_memcpy(&v, out[l], 16);
        *(v4i*)(base + l * 1024) = v;
    }
}

// A operand: the transform block E = ebuf columns [ecol0, ecol0 + wj), split
// into digits, in MFMA lane order: fragment (rb, kb, l) is 64 lanes x 16 bytes;
// lane L holds row rb*32 + L%32 and k = kb*32 + 16*(L/32) + i.
__device__ __forceinline__ void build_a_at(const PlainArgs& w, Mat ebuf, int64_t ecol0, int32_t wj, int32_t KB,
                                           int64_t MB, int8_t* Afrag, int64_t gid) {
    if (gid >= MB * KB * 64) return;
    const int L = (int)(gid & 63);
    const int64_t t = gid >> 6;
    const int kb = (int)(t % KB);
    const int64_t rb = t / KB;
    const int64_t row = rb * 32 + (L & 31);
    const uint32_t p = w.F.p;
    const int k0 = kb * 32 + 16 * (L >> 5);
    uint32_t ev[16];
    if (row < w.m && k0 + 15 < wj && (ecol0 & 3) == 0) {  // 128-bit loads (row starts and k0 are multiples of 4)
        const uint4* src = (const uint4*)(ebuf.M + row * ebuf.ld + ecol0 + k0);
        for (int q = 0; q < 4; ++q) {
            const uint4 x = src[q];
            ev[4 * q] = x.x;
            ev[4 * q + 1] = x.y;
            ev[4 * q + 2] = x.z;
            ev[4 * q + 3] = x.w;
        }
    } else {
        for (int i = 0; i < 16; ++i)
            ev[i] = (row < w.m && k0 + i < wj) ? ebuf.M[row * ebuf.ld + ecol0 + k0 + i] : 0u;
    }
    int8_t out[4][16];
    for (int i = 0; i < 16; ++i) {
        int8_t d[4];
        digits4(centre(ev[i], p), d);
        for (int l = 0; l < 4; ++l) out[l][i] = d[l];
    }
    int8_t* base = Afrag + ((rb * KB + kb) * 4) * 1024 + L * 16;
    for (int l = 0; l < 4; ++l) {
        v4i v;
        __builtin_memcpy(&v, out[l], 16);
        *(v4i*)(base + l * 1024) = v;
    }
}

// k-blocks of 32 in one trailing product: panels are at most 512 columns wide
// (the fold is exact up to K = 512)
constexpr int kMaxKB = 16;

__device__ __forceinline__ uint32_t fold7(const v16i* acc, int r, uint32_t add, double c32,
                                          const FieldConst& F) {
    return fold7s(acc[0][r], acc[1][r], acc[2][r], acc[3][r], acc[4][r], acc[5][r], acc[6][r], add,
                  c32, F);
}

// One fragment row of 64 lanes x 16 bytes straight from global memory into
// LDS (lane i's 16 bytes land at lds + 16 i); the wave's vector-memory count
// covers it like a load.
__device__ __forceinline__ void lds_dma16(const int8_t* g, v4i* lds) {
    __builtin_amdgcn_global_load_lds((const void*)g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// s_waitcnt with only the vector-memory count (expcnt and lgkmcnt at their
// no-wait maxima): wait until at most n of this wave's vector-memory
// operations are outstanding.
template <int n>
__device__ __forceinline__ void wait_vm() {
    static_assert(n >= 0 && n < 64, "six-bit vmcnt");
    __builtin_amdgcn_s_waitcnt((n & 15) | (0x7 << 4) | (0xF << 8) | ((n >> 4) << 14));
}

// A workgroup barrier that orders the compiler's memory accesses but adds no
// wait of its own (the k loop waits for its LDS copies explicitly).
__device__ __forceinline__ void bare_barrier() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
}

// Product update C = delta * C + A . B (mod p) on int8 MFMA (C = dst columns
// [col0, col0 + N); delta = 0 for the rows whose pivot column lies in
// [fresh_lo, fresh_hi)).  Block: 4 waves over a 64 x 64 tile; wave v owns the
// 32 x 32 block (row block v & 1, column block v >> 1) with the seven group
// accumulators of one 32x32 MFMA block.  A k-block's operands (two row blocks
// and two column blocks, 4 digit planes x 1 KB each, 16 KB) go through LDS,
// each fragment read by the two waves that share its rows or columns: per
// output, half the A traffic of a 32-column tile.  They are copied from global
// memory straight into a ring of four LDS stages, three k-blocks ahead of the
// MFMAs that use them, so that an L2 or HBM round trip overlaps three k-blocks
// of MFMA work without holding registers.  A tile's C entries are loaded
// after its first k-block, behind the copies, so that the first step waits
// for operands only, and a workgroup retires without waiting for its stores
// to complete.  Tiles are taken by the workgroups
// in turn, row tiles fastest, so that concurrent workgroups share their B
// slices in L2; with a multiple of 8 row tiles all tiles of one row range run
// on the same XCD, whose L2 then holds one eighth of the A operand.  The grid
// is one workgroup per tile, or fewer that loop, which leaves compute units
// free for other work on the device.  With out.M set the results go to out
// (columns from 0) instead of dst, and out's columns [ezero, ezero + N) of
// the same rows are set to zero: the next panel's columns written straight
// into the panel buffer, with its transform block cleared.
// Rows a product leaves alone: in the trailing update the pivot rows of earlier
// panels (forward elimination; skip_below = the panel's first column, else 0),
// in the back-substitution update every row but those.
template <bool kBack>
__device__ __forceinline__ bool row_left(int32_t rowcol, int32_t skip_below) {
    return kBack ? !(rowcol >= 0 && rowcol < skip_below) : earlier_pivot(rowcol, skip_below);
}

template <bool kBack>
__device__ __forceinline__ void gemm_i8_body(const PlainArgs& w, Mat dst, int64_t col0, int64_t N,
                                             const int8_t* Afrag, const int8_t* Bfrag, int32_t KB,
                                             int32_t fresh_lo, int32_t fresh_hi, double c32,
                                             int32_t skip_below, Mat out, int32_t ezero) {
    // four stages, each [A row block 0, 1 | B column block 0, 1][digit plane][lane]
    // (separate arrays, so that the compiler sees a stage's reads apart from
    // the copies in flight into the others)
    __shared__ v4i st0[4][4][64], st1[4][4][64], st2[4][4][64], st3[4][4][64];  // 4 x 16 KB
    typedef v4i Stage[4][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rg = wave & 1, cg = wave >> 1;
    const int64_t mtiles = ceil_div(w.m, 64);
    const int64_t nb = ceil_div(N, 32);  // column blocks with built B fragments
    const int64_t ntiles = mtiles * ceil_div(N, 64);
    const int last = KB - 1;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t rt = tile % mtiles, ct = tile / mtiles;
        // The stores of the previous tile (if this workgroup had one) first:
        // the k steps below count the loads in flight, and stores need not
        // complete in order with loads.  (The barriers below also wait for
        // every wave to be done with its stages.)
        wait_vm<0>();
        if (skip_below > 0) {  // forward elimination: a tile of earlier pivot rows only is skipped
            const int64_t row = rt * 64 + (threadIdx.x >> 2);
            int keep = 0;
            if ((threadIdx.x & 3) == 0 && row < w.m) keep = !row_left<kBack>(w.rowcol[row], skip_below);
            if (__syncthreads_or(keep) == 0) continue;
        } else {
            __syncthreads();
        }
        // The tile's C entries and its rows' bookkeeping first (the k loop's
        // first wait then covers them).  32x32 accumulator layout: lane L holds
        // column L%32 and rows 8*(r/4) + 4*(L/32) + r%4 for r = 0..15.
        // Addresses are clamped into the matrix so that every load is issued
        // unconditionally; out-of-range values are discarded in the epilogue.
        const int64_t rb = rt * 2 + rg;
        const int64_t col = (ct * 2 + cg) * 32 + (lane & 31);
        const int64_t colc = col < N ? col : N - 1;
        // Lane rows row0 + 8 (r / 4) + r % 4: four group bases 8 rows apart and
        // offsets of 0..3 rows give every address with additions only (no
        // 64-bit multiply per entry).
        const int64_t row0 = rb * 32 + 4 * (lane >> 5);
        const int64_t ld = dst.ld, ld2 = ld + ld, ld3 = ld2 + ld, ld8 = ld << 3;
        const int64_t roff[4] = {0, ld, ld2, ld3};
        const bool full = rb * 32 + 32 <= w.m;  // (uniform) every row of the block is inside the matrix
        int rcv[16];
        if (full) {
            const int32_t* rc = w.rowcol + row0;
            for (int q = 0; q < 4; ++q, rc += 8)
                for (int e = 0; e < 4; ++e) rcv[4 * q + e] = rc[e];
        } else {
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + 8 * (r >> 2) + (r & 3);
                rcv[r] = w.rowcol[row < w.m ? row : w.m - 1];
            }
        }
        // this wave copies digit planes 2 cg, 2 cg + 1 of row block rg of A and
        // of column block rg of B (a column block past the built ones reads
        // the last one: its products fall on columns >= N and are dropped)
        const int64_t cbl = ct * 2 + rg < nb ? ct * 2 + rg : nb - 1;
        const int8_t* asrc = Afrag + ((rt * 2 + rg) * KB * 4 + 2 * cg) * 1024 + lane * 16;
        const int8_t* bsrc = Bfrag + (cbl * KB * 4 + 2 * cg) * 1024 + lane * 16;
        // Four copies per wave and k-block.  Every step copies one k-block,
        // the last one again once the tile has no more (into a stage that is
        // not read again), so that before each step exactly the copies of the
        // two k-blocks after it may still be in flight.
        auto copy = [&](Stage& st, int kb) {
            const int64_t o = (int64_t)min(kb, last) * 4 * 1024;
            lds_dma16(asrc + o, &st[rg][2 * cg][0]);
            lds_dma16(asrc + o + 1024, &st[rg][2 * cg + 1][0]);
            lds_dma16(bsrc + o, &st[2 + rg][2 * cg][0]);
            lds_dma16(bsrc + o + 1024, &st[2 + rg][2 * cg + 1][0]);
        };
        copy(st0, 0);
        copy(st1, 1);
        copy(st2, 2);
        v16i acc[7];
        for (int g = 0; g < 7; ++g)
            for (int r = 0; r < 16; ++r) acc[g][r] = 0;
        // step kb: wait for this wave's copies of k-block kb (at most those of
        // kb + 1 and kb + 2 outstanding), barrier (every wave's copies of kb
        // have landed, and every wave is done with stage kb - 1), copy k-block
        // kb + 3 into stage kb - 1, multiply k-block kb
        auto step = [&](auto vm, const Stage& cur_st, Stage& next_st, int kb) {
            wait_vm<decltype(vm)::value>();
            bare_barrier();
            copy(next_st, kb + 3);
            v4i af[4], bf[4];
            for (int l = 0; l < 4; ++l) af[l] = cur_st[rg][l][lane];
            for (int l = 0; l < 4; ++l) bf[l] = cur_st[2 + cg][l][lane];
            for (int l = 0; l < 4; ++l)
                for (int lp = 0; lp < 4; ++lp)
                    acc[l + lp] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[l], bf[lp], acc[l + lp], 0, 0, 0);
        };
        typedef std::integral_constant<int, 8> Ahead;
        typedef std::integral_constant<int, 24> AheadC;
        uint32_t cur[16];
        step(Ahead{}, st0, st3, 0);
        // The tile's C entries, issued after the copies of k-block 3: exactly
        // 16 loads per lane, which the next three steps' waits allow to be
        // outstanding beside the copies of the two k-blocks ahead.
        __asm__ volatile("" ::: "memory");
        if (full) {
            const uint32_t* g = dst.M + row0 * ld + col0 + colc;
            for (int q = 0; q < 4; ++q, g += ld8)
                for (int e = 0; e < 4; ++e) cur[4 * q + e] = __builtin_nontemporal_load(g + roff[e]);
        } else {
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + 8 * (r >> 2) + (r & 3);
                cur[r] = __builtin_nontemporal_load(dst.M + (row < w.m ? row : w.m - 1) * ld + col0 + colc);
            }
        }
        do {
            if (KB <= 1) break;
            step(AheadC{}, st1, st0, 1);
            if (KB <= 2) break;
            step(AheadC{}, st2, st1, 2);
            if (KB <= 3) break;
            step(AheadC{}, st3, st2, 3);
#pragma unroll
            for (int kb = 4; kb < kMaxKB; kb += 4) {
                if (kb >= KB) break;
                step(Ahead{}, st0, st3, kb);
                if (kb + 1 >= KB) break;
                step(Ahead{}, st1, st0, kb + 1);
                if (kb + 2 >= KB) break;
                step(Ahead{}, st2, st1, kb + 2);
                if (kb + 3 >= KB) break;
                step(Ahead{}, st3, st2, kb + 3);
            }
        } while (false);
        // The C loads and the copies of the last steps (a k-block copied
        // again into stages no longer read) have landed: the workgroup's LDS
        // can be handed on once its stores are issued.  (The empty asm hands
        // the values over as new definitions: the compiler's own wait
        // analysis loses the count of the C loads at the joins of the k steps
        // and would otherwise wait for every store before each fold.)
        wait_vm<0>();
        for (int r = 0; r < 16; ++r) __asm__ volatile("" : "+v"(cur[r]));
        if (col < N && !out.M) {
            uint32_t* g = dst.M + row0 * ld + col0 + col;
            for (int q = 0; q < 4; ++q, g += ld8)
                for (int e = 0; e < 4; ++e) {
                    const int r = 4 * q + e;
                    if (row0 + 8 * q + e >= w.m || row_left<kBack>(rcv[r], skip_below)) continue;
                    const bool fresh = rcv[r] >= fresh_lo && rcv[r] < fresh_hi;  // a pivot row of this panel
                    // (streamed past L2, where the A and B fragments stay)
                    __builtin_nontemporal_store(fold7(acc, r, fresh ? 0u : cur[r], c32, w.F), g + roff[e]);
                }
        } else if (col < N) {
            // (a pivot row of this panel also keeps its entries in dst: in
            // forward elimination it takes no part in the next panel, whose
            // write-back then skips it, and back-substitution reads them there)
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + 8 * (r >> 2) + (r & 3);
                if (row >= w.m) continue;
                uint32_t* o = out.M + row * out.ld;
                o[ezero + col] = 0u;
                if (row_left<kBack>(rcv[r], skip_below)) continue;
                const bool fresh = rcv[r] >= fresh_lo && rcv[r] < fresh_hi;  // a pivot row of this panel
                const uint32_t v = fold7(acc, r, fresh ? 0u : cur[r], c32, w.F);
                o[col] = v;
                if (fresh) dst.M[row * ld + col0 + col] = v;
            }
        }
    }
}

__global__ __launch_bounds__(kThreads, 2) void gemm_i8_kernel(PlainArgs w, Mat dst, int64_t col0,
                                                              int64_t N, const int8_t* Afrag,
                                                              const int8_t* Bfrag, int32_t KB,
                                                              int32_t fresh_lo, int32_t fresh_hi,
                                                              double c32, int32_t skip_below, Mat out,
                                                              int32_t ezero) {
    gemm_i8_body<false>(w, dst, col0, N, Afrag, Bfrag, KB, fresh_lo, fresh_hi, c32, skip_below, out,
                        ezero);
}

// The back-substitution update of one panel (see back_substitute): the
// right-hand sides (dst columns [col0, col0 + N)) of the pivot rows of earlier
// panels (rowcol below j0) become C + A . B, A = their entries in the panel's
// columns, B = -x of the panel's columns.
__global__ __launch_bounds__(kThreads, 2) void bs_product_kernel(PlainArgs w, Mat dst, int64_t col0,
                                                                 int64_t N, const int8_t* Afrag,
                                                                 const int8_t* Bfrag, int32_t KB,
                                                                 double c32, int32_t j0) {
    gemm_i8_body<true>(w, dst, col0, N, Afrag, Bfrag, KB, 0, 0, c32, j0, Mat{nullptr, 0}, 0);
}

// The int8 leaf product (leafprod.h) over a grid of 64-row blocks (x) and
// column groups (y).
template <int kLeafBlocks, int kMode>
__global__ __launch_bounds__(kThreads, 4) void leaf_product_i8_kernel(LeafProdArgs a) {
    leaf_product_block<kLeafBlocks, kMode, 4>(a, blockIdx.x, blockIdx.y,
                                              (int64_t)blockIdx.y * gridDim.x + blockIdx.x);
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
    // clamped addresses: every load is issued unconditionally
    uint32_t cur[2][2][4];
    bool fresh[2][4];
    for (int a = 0; a < 2; ++a)
        for (int i = 0; i < 4; ++i) {
            const int64_t row = (rb0 + a) * 16 + (lane >> 4) + 4 * i;
            const int rc = w.rowcol[row < w.m ? row : w.m - 1];
            fresh[a][i] = rc >= fresh_lo && rc < fresh_hi;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int64_t col = (cb0 + b) * 16 + (lane & 15);
            const int64_t colc = col < N ? col : N - 1;
            for (int i = 0; i < 4; ++i) {
                const int64_t row = (rb0 + a) * 16 + (lane >> 4) + 4 * i;
                cur[a][b][i] = dst.M[(row < w.m ? row : w.m - 1) * dst.ld + col0 + colc];
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
__device__ __forceinline__ void writeback_at(const PlainArgs& w, Mat src, Mat dst, int64_t d0, int32_t width,
                                             int32_t gcol0, int32_t skip_below, int64_t gid) {
    if (gid >= (int64_t)w.m * width) return;
    const int64_t r = gid / width;
    if (earlier_pivot(w.rowcol[r], skip_below)) return;
    const int js = (int)(gid % width);
    const int s = w.colpiv[gcol0 + js];
    uint32_t v;
    if (s >= 0) v = (w.pivrow[s] == r) ? 1u : 0u;
    else v = src.M[r * src.ld + js];
    dst.M[r * dst.ld + d0 + js] = v;
}

__global__ void panel_writeback_kernel(PlainArgs w, Mat src, Mat dst, int64_t d0, int32_t width,
                                       int32_t gcol0, int32_t skip_below) {
    writeback_at(w, src, dst, d0, width, gcol0, skip_below, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// The int8 trailing product's operands and the panel's write-back in one
// launch: workgroups [0, gb) build B, [gb, gb + ga) build A, the rest write the
// reduced panel back into W.  The three touch disjoint data (B reads the pivot
// rows right of the panel, A the transform block of PR, the write-back the
// panel block of PR and the panel's columns of W, which neither product
// reads), so they run side by side instead of as three dependent launches.
__global__ void panel_operands_kernel(PlainArgs w, Mat W, Mat PR, int32_t j0, int32_t wj, int64_t col0,
                                      int64_t N, int32_t KB, int64_t NB, int64_t MB, int8_t* Afrag,
                                      int8_t* Bfrag, int32_t skip_below, int32_t gb, int32_t ga) {
    const int64_t b = blockIdx.x;
    if (b < gb) {
        build_b_at(w, W, j0, wj, col0, N, (int64_t)-1, KB, NB, Bfrag, b * blockDim.x + threadIdx.x);
    } else if (b < gb + ga) {
        build_a_at(w, PR, (int64_t)wj, wj, KB, MB, Afrag, (b - gb) * blockDim.x + threadIdx.x);
    } else {
        writeback_at(w, PR, W, (int64_t)j0, wj, j0, skip_below,
                     (b - gb - ga) * blockDim.x + threadIdx.x);
    }
}

// Back-substitution after forward elimination (the solve).  The pivot row q of
// a column c in panel [j0, j0 + wj) is 1 at c and 0 at every other pivot column
// of its panel and of the panels before it; right of its panel it keeps
// entries U[q][c'].  So x(c, t) = W[q][n + t] once the terms of every later
// column have been taken off: panel by panel from the last, the right-hand
// sides of the pivot rows of the earlier panels become
//    W[q'][n + t] - sum over c in the panel of U[q'][c] x(c, t),
// with x(c, t) = W[pivot row of c][n + t] (0 for a free column): one int8 MFMA
// product per panel with K = the panel width (A = those rows' entries in the
// panel's columns, B = -x), reduced exactly as the trailing update is.
// bs_operands_kernel builds its fragments: the first gb blocks B, the rest A.
__global__ void bs_operands_kernel(PlainArgs w, Mat W, int32_t j0, int32_t wj, int64_t col0, int64_t N,
                                   int32_t KB, int64_t NB, int64_t MB, int8_t* Afrag, int8_t* Bfrag,
                                   int32_t gb) {
    const int64_t b = blockIdx.x;
    if (b < gb)
        build_b_at<true>(w, W, j0, wj, col0, N, (int64_t)-1, KB, NB, Bfrag, b * blockDim.x + threadIdx.x);
    else
        build_a_at(w, W, (int64_t)j0, wj, KB, MB, Afrag, (b - gb) * blockDim.x + threadIdx.x);
}

constexpr int32_t kLeaf = 32;  // inner panel width of the two-level reduction

struct Blocked {
    PlainArgs w;  // the working matrix and the bookkeeping (shared with the plain path)
    Mat PR;       // outer panel [panel | E]
    int8_t* Afrag;
    int8_t* Bfrag;
    int64_t abytes, bbytes;  // sizes of the two fragment buffers
    int8_t* Yfrag;  // the int8 leaf products' right operand (kept apart from the trailing one)
    LeafState leaf;
    int32_t panel;
};

// Workspace after the plain layout: PR (m x ldpr), the operand fragments (sized
// for the larger of the int8 layouts, 4 B per element, and the FP64 ones, 8 B,
// for both the trailing product and the leaf products), the leaf products' Y
// fragments and the leaf selection state.
size_t carve_blocked(void* ws, int64_t m, int64_t n, int64_t k, int32_t panel, Blocked* b) {
    const size_t base = plain_workspace(m, n, k);
    Carver c(ws ? (char*)ws + base : nullptr);
    const int64_t ldpr = round_up(2 * (int64_t)panel, 64);
    const int64_t Kp = round_up(panel, 32);
    const int64_t Mp = round_up(m > 0 ? m : 1, 128);
    const int64_t Np = round_up(n + k > 0 ? n + k : 1, 64);
    const int64_t Nl = round_up(2 * (int64_t)panel + kLeaf, 64);  // leaf product columns
    const int64_t abytes = Mp * (Kp > kLeaf ? Kp : kLeaf) * 8;
    const int64_t bbytes = (Np * Kp > Nl * kLeaf ? Np * Kp : Nl * kLeaf) * 8;
    uint32_t* PR = c.take<uint32_t>(m * ldpr);
    int8_t* A = c.take<int8_t>(abytes);
    int8_t* B = c.take<int8_t>(bbytes);
    int8_t* Y = c.take<int8_t>(Nl * kLeaf * 4);
    LeafState ls;
    leaf_carve(c, m, Nl, &ls);
    if (b) {
        plain_carve(ws, m, n, k, b->w);
        b->PR = Mat{PR, ldpr};
        b->Afrag = A;
        b->Bfrag = B;
        b->abytes = abytes;
        b->bbytes = bbytes;
        b->Yfrag = Y;
        b->leaf = ls;
        b->panel = panel;
    }
    return base + c.off + 256;
}

// The product kernel: dst columns [col0, col0 + N) of every row become
// delta * C + A . B from the prepared fragments (K = 32 KB for int8, 4 KB for
// FP64; B's first fragment belongs to column col0); delta = 0 for the rows
// whose pivot column lies in [fresh_lo, fresh_hi).
hipError_t run_product(const PlainArgs& w, bool fp64, const int8_t* Af, const int8_t* Bf, Mat dst,
                       int64_t col0, int64_t N, int32_t KB, int32_t fresh_lo, int32_t fresh_hi,
                       hipStream_t s, LaunchTimer& lt, int kind, int64_t max_wgs = 0,
                       int32_t skip_below = 0, Mat out = Mat{nullptr, 0}, int32_t ezero = 0) {
    const int64_t m = w.m;
    lt.before(kind, s);
    if (fp64) {
        hipLaunchKernelGGL(gemm_f64_kernel, dim3((unsigned)ceil_div(m, 64), (unsigned)ceil_div(N, 64)),
                           dim3(kThreads), 0, s, w, dst, col0, N, (const double*)Af,
                           (const double*)Bf, KB, ceil_div(N, 16), fresh_lo, fresh_hi);
    } else {
        if (KB < 1 || KB > kMaxKB) return hipErrorInvalidValue;
        const double c32 = (double)((((uint64_t)1) << 32) % w.F.p);
        const int64_t tiles = ceil_div(m, 64) * ceil_div(N, 64);
        const int64_t grid = max_wgs > 0 && max_wgs < tiles ? max_wgs : tiles;
        hipLaunchKernelGGL(gemm_i8_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, w, dst, col0, N,
                           Af, Bf, KB, fresh_lo, fresh_hi, c32, skip_below, out, ezero);
    }
    lt.after();
    return hipGetLastError();
}

// Operands of the trailing update of panel [j0, j0 + wj) over dst columns
// [col0, col0 + N): A = PR's transform block (columns [wj, 2 wj)), B = X_S,
// the pivot rows of bookkeeping columns [j0, j0 + wj) read from dst.  On the
// int8 path the same launch also writes the reduced panel back into dst.
// Returns the number of k-blocks.
int32_t trailing_operands(const Blocked& b, const PlainArgs& w, bool fp64, Mat dst, int32_t j0,
                          int32_t wj, int64_t col0, int64_t N, int32_t skip_below, hipStream_t s,
                          LaunchTimer& lt, int8_t* Af, int8_t* Bf, int64_t nb_cols) {
    const int64_t m = w.m;
    lt.before(LINAC_KERNEL_OPERANDS);
    int32_t KB;
    if (fp64) {
        KB = (int32_t)ceil_div(wj, 4);
        const int64_t NB = ceil_div(N, 16);
        const int64_t MB = ceil_div(m, 64) * 4;
        hipLaunchKernelGGL(build_b_f64_kernel, dim3((unsigned)ceil_div(NB * KB * 64, 256)), dim3(256),
                           0, s, w, dst, j0, wj, col0, N, (int64_t)-1, KB, NB, (double*)Bf);
        hipLaunchKernelGGL(build_a_f64_kernel, dim3((unsigned)ceil_div(MB * KB * 64, 256)), dim3(256),
                           0, s, w, b.PR, (int64_t)wj, wj, KB, MB, (double*)Af);
    } else {
        KB = (int32_t)ceil_div(wj, 32);
        const int64_t NB = ceil_div(nb_cols, 32);
        const int64_t MB = ceil_div(m, 128) * 4;
        const int32_t gb = (int32_t)ceil_div(NB * KB * 64, 256), ga = (int32_t)ceil_div(MB * KB * 64, 256);
        const int32_t gw = (int32_t)ceil_div(m * wj, 256);
        hipLaunchKernelGGL(panel_operands_kernel, dim3((unsigned)(gb + ga + gw)), dim3(256), 0, s, w, dst,
                           b.PR, j0, wj, col0, nb_cols, KB, NB, MB, Af, Bf, skip_below, gb, ga);
    }
    lt.after();
    return KB;
}

// The B fragments of trailing columns [col0, col0 + N) alone (int8 path; Bf is
// the fragment of column col0), for the part of a split trailing product that
// runs on the side stream.
hipError_t trailing_b_rest(const Blocked& b, const PlainArgs& w, Mat dst, int32_t j0, int32_t wj,
                           int64_t col0, int64_t N, int32_t KB, int8_t* Bf, hipStream_t s,
                           LaunchTimer& lt) {
    const int64_t NB = ceil_div(N, 32);
    const int32_t gb = (int32_t)ceil_div(NB * KB * 64, 256);
    lt.before(LINAC_KERNEL_OPERANDS, s);
    hipLaunchKernelGGL(panel_operands_kernel, dim3((unsigned)gb), dim3(256), 0, s, w, dst, b.PR, j0, wj,
                       col0, N, KB, NB, (int64_t)0, (int8_t*)nullptr, Bf, 0, gb, 0);
    lt.after();
    return hipGetLastError();
}

// Panels from the last to the first (see bs_operands_kernel); the first panel
// has no earlier pivot rows to update.
hipError_t back_substitute(const Blocked& b, int64_t n, int64_t k, int32_t panel, hipStream_t s) {
    const PlainArgs& w = b.w;
    const int64_t m = w.m;
    const Mat Wm{w.W, w.ld};
    const double c32 = (double)((((uint64_t)1) << 32) % w.F.p);
    const int64_t last = (n - 1) / panel * panel;
    for (int64_t j0 = last; j0 > 0; j0 -= panel) {
        const int32_t wj = (int32_t)(n - j0 < panel ? n - j0 : panel);
        const int32_t KB = (int32_t)ceil_div(wj, 32);
        if (KB > kMaxKB) return hipErrorInvalidValue;
        const int64_t NB = ceil_div(k, 32), MB = ceil_div(m, 128) * 4;
        const int32_t gb = (int32_t)ceil_div(NB * KB * 64, 256), ga = (int32_t)ceil_div(MB * KB * 64, 256);
        hipLaunchKernelGGL(bs_operands_kernel, dim3((unsigned)(gb + ga)), dim3(256), 0, s, w, Wm,
                           (int32_t)j0, wj, n, k, KB, NB, MB, b.Afrag, b.Bfrag, gb);
        hipLaunchKernelGGL(bs_product_kernel, dim3((unsigned)(ceil_div(m, 64) * ceil_div(k, 64))),
                           dim3(kThreads), 0, s, w, Wm, n, k, (const int8_t*)b.Afrag,
                           (const int8_t*)b.Bfrag, KB, c32, (int32_t)j0);
    }
    return hipGetLastError();
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
//
// Look-ahead (int8 path): the trailing update of panel k is split into the
// next panel's columns (on the caller's stream, before that panel starts) and
// the remaining columns, which run on a side stream while the next panel's
// leaves (latency bound, on few compute units) proceed.  The next panel's
// trailing operands wait for that remainder: it writes the columns they read.
// The leaves touch only PR, the leaf state and the pivot bookkeeping; of those
// the remainder reads only rowcol, to spot the previous panel's pivot rows,
// which new pivot rows (from -1 to a later column) never are either way.
hipError_t blocked_eliminate(void* ws, int64_t m, int64_t n, int64_t k, int32_t panel, bool fp64,
                             bool overlap, bool forward, int32_t leaf_blocks, bool leaf_pipeline,
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
    hipStream_t side = nullptr;
    hipEvent_t ev_t1 = nullptr, ev_t2 = nullptr, ev_t3 = nullptr;
    const bool lookahead = overlap && !fp64 && n > panel;
    forward = forward && !fp64 && k > 0;  // the int8 path with right-hand sides to solve for
    // Y built by the selection's second launch when the first one decided the
    // leaf (faster than a rebuild in every product workgroup)
    const bool select_y = true;
    hipError_t e = hipSuccess;
    // (a remainder capped at one workgroup per compute unit ran longer and
    // slowed the leaves as much: the contention is in the memory system)
    const int64_t side_wgs = 0;
    if (lookahead) {
        e = side_stream(&side);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_t1, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_t2, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_t3, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (ev_t1) (void)hipEventDestroy(ev_t1);
            if (ev_t2) (void)hipEventDestroy(ev_t2);
            return e;
        }
    }
    // Leaf pipeline (int8 path): each leaf's product in two halves, the next
    // leaf's first chunk alone, then the other rows in the same launch as the
    // next leaf's first selection, which overlaps them.
    const bool pipeline = !fp64 && leaf_pipeline;
    bool t2_pending = false;
    bool t3_pending = false;  // the side stream's first part of a split remainder is in flight
    bool pr_ready = false;  // the next panel's columns are in PR already
    int32_t opset = 0;      // operand fragment set of the current panel (two alternate, int8 path)
    if (e == hipSuccess) e = leaf_init(b.leaf, (int32_t)m, s);
    int32_t leaf_index = 0;
    for (int32_t j0 = 0; j0 < n && e == hipSuccess; j0 += panel) {
        const int32_t wj = (int32_t)(n - j0 < panel ? n - j0 : panel);
        const int32_t skip_below = forward ? j0 : 0;
        if (!pr_ready)  // (else the previous trailing product wrote this panel into PR)
            hipLaunchKernelGGL(panel_extract_kernel, dim3(tiles, (unsigned)ceil_div(b.PR.ld, 256)),
                               dim3(kThreads), 0, s, w.m, Wm, (int64_t)j0, b.PR, wj);
        pr_ready = false;
        bool first_done = false;  // this leaf's first selection already ran (pipelined)
        for (int32_t l0 = 0; l0 < wj && e == hipSuccess; l0 += kLeaf) {
            const int32_t wl = wj - l0 < kLeaf ? wj - l0 : kLeaf;
            const int32_t parity = leaf_index & 1;
            // the leaf's own columns, the panel columns after it and the transform
            // block up to this leaf's pivots (beyond it every row is still zero)
            const int64_t N = (int64_t)wj + wl;
            int8_t* yf = fp64 || !select_y ? nullptr : b.Yfrag;
            const bool piped = pipeline && l0 + kLeaf < wj;  // (see the product below)
            lt.before(LINAC_KERNEL_SELECT);
            e = leaf_select(w, b.leaf, b.PR.M, b.PR.ld, l0, wl, wj, j0 + l0, parity, N, yf, !fp64, s,
                            first_done ? kSelectRest : kSelectFirst | kSelectRest);
            lt.after();
            first_done = false;
            if (e != hipSuccess) break;
            if (fp64) {
                lt.before(LINAC_KERNEL_OPERANDS);
                e = leaf_operands(w, b.leaf, b.PR.M, b.PR.ld, l0, wl, wj, j0 + l0, N, parity, fp64,
                                  b.Afrag, b.Bfrag, s);
                lt.after();
                if (e != hipSuccess) break;
                e = run_product(w, fp64, b.Afrag, b.Bfrag, b.PR, (int64_t)l0, N, kLeaf / 4, j0 + l0,
                                j0 + l0 + wl, s, lt, LINAC_KERNEL_LEAF_PRODUCT);
            } else {
                const double c32 = (double)((((uint64_t)1) << 32) % w.F.p);
                LeafProdArgs pa;
                pa.w = w;
                pa.PR = b.PR.M;
                pa.ldpr = b.PR.ld;
                pa.l0 = l0;
                pa.wl = wl;
                pa.wj = wj;
                pa.gcol0 = j0 + l0;
                pa.N = N;
                pa.out = b.leaf.out[parity];
                pa.rsave = b.leaf.rsave;
                pa.ldr = b.leaf.ldr;
                pa.c32 = c32;
                pa.cand = b.leaf.cand[parity];
                pa.cand_next = b.leaf.cand[parity ^ 1];
                pa.count = b.leaf.count + parity;
                pa.count_next = b.leaf.count + (parity ^ 1);
                pa.yfrag = b.Yfrag;
                pa.skip_below = skip_below;
                pa.chunk = b.leaf.chunk;
                pa.ymode = piped ? 1 : 0;  // (a chunk launch stores the Y it forms)
                pa.ystore = b.Yfrag;
#define LEAF_PRODUCT(LB, MODE)                                                                      \
    hipLaunchKernelGGL((leaf_product_i8_kernel<LB, MODE>),                                          \
                       dim3((unsigned)(MODE == kLeafChunk ? 1 : ceil_div(m, 64)),                   \
                            (unsigned)ceil_div(N, 16 * (LB))),                                      \
                       dim3(kThreads), 0, s, pa)
                const int32_t l1 = l0 + kLeaf;  // the next leaf of this panel, if any
                if (piped) {
                    // The next leaf's first chunk is updated first; then one launch
                    // runs the next leaf's first selection (on that chunk) beside the
                    // update of the other rows.
                    const int32_t wl1 = wj - l1 < kLeaf ? wj - l1 : kLeaf;
                    lt.before(LINAC_KERNEL_LEAF_PRODUCT);
                    LEAF_PRODUCT(2, kLeafChunk);
                    lt.after();
                    e = hipGetLastError();
                    if (e != hipSuccess) break;
                    LeafProdArgs pr = pa;
                    pr.ymode = 2;  // Y built by the selection or stored by the chunk launch
                    lt.before(LINAC_KERNEL_LEAF_FUSED);
                    e = leaf_fused(w, b.leaf, b.PR.M, b.PR.ld, l1, wl1, wj, j0 + l1, parity ^ 1,
                                   (int64_t)wj + wl1, yf, pr, leaf_blocks, s);
                    lt.after();
                    first_done = true;
                } else {
                    lt.before(LINAC_KERNEL_LEAF_PRODUCT);
                    if (leaf_blocks >= 9) LEAF_PRODUCT(9, kLeafAll);
                    else if (leaf_blocks >= 6) LEAF_PRODUCT(6, kLeafAll);
                    else if (leaf_blocks >= 3) LEAF_PRODUCT(3, kLeafAll);
                    else LEAF_PRODUCT(2, kLeafAll);
                    lt.after();
                    e = hipGetLastError();
                }
#undef LEAF_PRODUCT
            }
            ++leaf_index;
        }
        if (e != hipSuccess) break;
        const int64_t N = ncols - (j0 + wj);
        const int64_t col0 = (int64_t)j0 + wj;
        // The next panel's columns now, the rest on the side stream.  On the
        // int8 path the next panel's columns go straight into PR (with its
        // transform block cleared), so that panel needs no copy; that takes a
        // width that keeps the remaining B fragments 32-aligned.
        const int64_t wnext = n - (j0 + wj) < panel ? n - (j0 + wj) : panel;
        const bool direct = !fp64 && wnext > 0 && wnext % 32 == 0;
        const int64_t n1 = direct ? wnext : (lookahead && N > panel ? panel : N);
        // Split remainder (int8 look-ahead, forward elimination): the columns of
        // the panel after next first, in a launch of their own, so that the next
        // panel waits for those only; the B fragments of the columns after them
        // are built on the side stream, behind the previous remainder, whose
        // later columns they read.  Two fragment sets alternate between panels,
        // since the side stream may still read this panel's set while the next
        // panel's operands are built.  (Under Gauss-Jordan the remainder hides
        // behind the leaves and the extra launches only add to them.)
        const int64_t after = n - (j0 + wj) - wnext;
        const int64_t w2 = after < panel ? after : panel;
        const bool split = N > 0 && lookahead && forward && direct && w2 > 0 && w2 % 32 == 0 &&
                           n1 + w2 < N;
        // The previous remainder writes the columns read next: its first part
        // covers this panel's next-panel columns, all that a split panel reads on
        // this stream; any other panel builds B over every trailing column and
        // waits for all of it.
        if (split && t3_pending) {
            e = hipStreamWaitEvent(s, ev_t3, 0);
        } else if (t2_pending) {
            e = hipStreamWaitEvent(s, ev_t2, 0);
            t2_pending = false;
        }
        t3_pending = false;
        if (e != hipSuccess) break;
        if (N > 0) {
            if (opts && opts->ev_begin && outer_products == 0) (void)hipEventRecord(opts->ev_begin, s);
            int8_t* Af = b.Afrag;
            int8_t* Bf = b.Bfrag;
            if (lookahead && !fp64) {  // (the int8 fragments take half of each buffer)
                Af += (size_t)opset * (b.abytes / 2);
                Bf += (size_t)opset * (b.bbytes / 2);
                opset ^= 1;
            }
            const int32_t KB = trailing_operands(b, w, fp64, Wm, j0, wj, col0, N, skip_below, s, lt, Af,
                                                 Bf, split ? n1 : N);
            e = hipGetLastError();
            if (e == hipSuccess)
                e = run_product(w, fp64, Af, Bf, Wm, col0, n1, KB, j0, j0 + wj, s, lt,
                                LINAC_KERNEL_TRAIL_PRODUCT, 0, skip_below,
                                direct ? b.PR : Mat{nullptr, 0}, (int32_t)wnext);
            pr_ready = direct && e == hipSuccess;
            int8_t* Bf1 = Bf + (n1 / 32) * KB * 4 * 1024;
            if (e == hipSuccess && n1 < N && !lookahead) {  // the rest on this stream
                e = run_product(w, fp64, Af, Bf1, Wm, col0 + n1, N - n1, KB, j0, j0 + wj, s, lt,
                                LINAC_KERNEL_TRAIL_PRODUCT, 0, skip_below);
            } else if (e == hipSuccess && n1 < N) {
                e = hipEventRecord(ev_t1, s);
                if (e == hipSuccess) e = hipStreamWaitEvent(side, ev_t1, 0);
                if (e == hipSuccess && split) {
                    e = trailing_b_rest(b, w, Wm, j0, wj, col0 + n1, N - n1, KB, Bf1, side, lt);
                    if (e == hipSuccess)
                        e = run_product(w, fp64, Af, Bf1, Wm, col0 + n1, w2, KB, j0, j0 + wj, side, lt,
                                        LINAC_KERNEL_TRAIL_PRODUCT, side_wgs, skip_below);
                    if (e == hipSuccess) e = hipEventRecord(ev_t3, side);
                    t3_pending = e == hipSuccess;
                    if (e == hipSuccess)
                        e = run_product(w, fp64, Af, Bf1 + (w2 / 32) * KB * 4 * 1024, Wm, col0 + n1 + w2,
                                        N - n1 - w2, KB, j0, j0 + wj, side, lt,
                                        LINAC_KERNEL_TRAIL_PRODUCT, side_wgs, skip_below);
                } else if (e == hipSuccess) {
                    e = run_product(w, fp64, Af, Bf1, Wm, col0 + n1, N - n1, KB, j0, j0 + wj, side, lt,
                                    LINAC_KERNEL_TRAIL_PRODUCT, side_wgs, skip_below);
                }
                if (e == hipSuccess) e = hipEventRecord(ev_t2, side);
                t2_pending = e == hipSuccess;
            }
            ++outer_products;
        }
        if (fp64 || N <= 0) {  // (the int8 operand launch above wrote the panel back already)
            hipLaunchKernelGGL(panel_writeback_kernel, dim3((unsigned)ceil_div(m * wj, 256)), dim3(256),
                               0, s, w, b.PR, Wm, (int64_t)j0, wj, j0, skip_below);
            if (e == hipSuccess) e = hipGetLastError();
        }
    }
    if (t2_pending) {
        const hipError_t e2 = hipStreamWaitEvent(s, ev_t2, 0);
        if (e == hipSuccess) e = e2;
    }
    if (forward && e == hipSuccess) e = back_substitute(b, n, k, panel, s);
    if (ev_t1) (void)hipEventDestroy(ev_t1);
    if (ev_t2) (void)hipEventDestroy(ev_t2);
    if (ev_t3) (void)hipEventDestroy(ev_t3);
    if (opts && opts->ev_end && outer_products > 0) (void)hipEventRecord(opts->ev_end, s);
    if (opts && opts->dominant_launches) *opts->dominant_launches = outer_products;
    return e;
}

}  // namespace linac
