// Pivot selection for a leaf of at most 32 pivot columns, and the operands of
// the leaf's product update (the blocked path's inner level).
//
// Over a field every non-zero entry is an acceptable pivot (Sec. 3.2,
// "Pivoting"), and the reduced row-echelon form does not depend on which rows
// serve as pivots.  The pivot columns of a leaf are fixed by the span of its
// eligible rows (rows that are not pivots yet): column c is a pivot column iff
// it raises the rank of the columns before it.  So any row basis of the leaf
// gives its pivot columns, and the leaf is reduced as one block:
//
//   select    the candidate rows (eligible rows in row order) are cut into
//             chunks of 32.  One workgroup per chunk runs Gauss-Jordan on its
//             rows' leaf values (registers + LDS) and keeps a basis of at most
//             32 rows.  Bases merge pairwise up a binary tree (a merge
//             eliminates the two bases' up to 64 rows); the second of two
//             siblings to finish does the merge.  A node that covers a prefix of
//             the candidates and has full rank, or the root, is final.  With
//             dense data the first chunk already has full rank, so a first
//             launch runs that chunk alone and publishes it when it decides the
//             leaf; the second launch then builds Y instead of the tree.
//   operands  Y = P^-1 R, where P is the pivot rows' values at the pivot
//             columns and R those rows over the columns to update (with the
//             implicit 1 of each new pivot in the panel's transform block), and
//             the multipliers -L[i, C] of every other row, both in the MFMA
//             operand layouts; the candidate list drops the new pivot rows.
//   product   C <- C + A Y for the other rows, C <- Y for the pivot rows (the
//             blocked path's MFMA product).
//
// The selection's Gauss-Jordan is fraction free (row_i <- d row_i - f_i row_q,
// no inverse on the critical path) and also tracks, for every row, the
// coefficients T of its current value in terms of the original pivot rows.  At
// the end pivot row s equals D_s e_s on the pivot columns, so
// P^-1 = diag(D)^-1 T.  D_s is the product of the pivot values d from step s
// on (each later step scales row s by its d), so with c_s the product before
// step s, D_s^-1 = c_s / (product of all d): one inverse per leaf.  Residues are held lazily in FP64, in (-3p, 3p): a product
// a b - floor(fl(ab)/p) p is exact by FMA and lies in [-p, 2p).
#include "internal.h"
#include "leafprod.h"

namespace linac {

namespace {

constexpr int kSelWaves = 4;   // the tree launch
constexpr int kSelThreads = 64 * kSelWaves;
// The first-chunk launch: eight waves, two per SIMD (one wave's FP64 issue rate
// is the limit, so a second wave per SIMD nearly doubles the throughput).  The
// layouts also support 16 waves, measured no faster.
constexpr int kFirstWaves = 8;
constexpr int kFirstThreads = 64 * kFirstWaves;
constexpr int kChunk = 32;     // candidate rows per first-level tree node
constexpr int kNodeInts = 64;  // per node: basis size, then its list positions

typedef int v4i __attribute__((ext_vector_type(4)));

struct Lazy {
    double p, pinv;
};

// a b - q p, q = floor(fl(a b) / p): exact and in [-p, 2p) for |a|, |b| < 2^33.
__device__ __forceinline__ double lz_mul(double a, double b, const Lazy& L) {
    const double h = a * b;
    const double l = __fma_rn(a, b, -h);
    const double q = floor(h * L.pinv);
    return __fma_rn(-q, L.p, h) + l;
}

// d v - f u, in (-3p, 3p).
__device__ __forceinline__ double lz_ff(double d, double v, double f, double u, const Lazy& L) {
    return lz_mul(d, v, L) - lz_mul(f, u, L);
}

// lz_ff over registers K0..K1-1 with shared d and f, written stage by stage so
// that the 2 (K1 - K0) independent products are interleaved in the instruction
// stream: with one wave per SIMD nothing else hides the latency of a dependent
// chain.  Same operations, same results as lz_ff per register.
template <int K0, int K1>
__device__ __forceinline__ void lz_ff_n(double y[4], double d, const double x[4], double f,
                                        const double u[4], const Lazy& L) {
    double h1[4], h2[4], l1[4], l2[4], q1[4], q2[4];
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        h1[k] = d * x[k];
        h2[k] = f * u[k];
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        q1[k] = h1[k] * L.pinv;
        q2[k] = h2[k] * L.pinv;
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        l1[k] = __fma_rn(d, x[k], -h1[k]);
        l2[k] = __fma_rn(f, u[k], -h2[k]);
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        q1[k] = floor(q1[k]);
        q2[k] = floor(q2[k]);
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        h1[k] = __fma_rn(-q1[k], L.p, h1[k]);
        h2[k] = __fma_rn(-q2[k], L.p, h2[k]);
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) y[k] = (h1[k] + l1[k]) - (h2[k] + l2[k]);
}

// The residue in [0, p) of an integer x with |x| < 2^34.
__device__ __forceinline__ double lz_canon(double x, const Lazy& L) {
    const double q = floor(x * L.pinv);
    double r = __fma_rn(-q, L.p, x);
    if (r < 0.0) r += L.p;
    if (r >= L.p) r -= L.p;
    return r;
}

// The residue in [0, p) of an integer x with |x| < 2^53 (for tiny p the first
// quotient may be off by more than one; the second pass starts below 3p).
__device__ __forceinline__ double lz_canon_wide(double x, const Lazy& L) {
    const double q = floor(x * L.pinv);
    return lz_canon(__fma_rn(-q, L.p, x), L);
}

// a^-1 = a^(p-2) for a canonical non-zero a (lane-parallel square-and-multiply).
__device__ double lz_inverse(double a, uint32_t p, const Lazy& L) {
    double r = 1.0, x = a;
    for (uint32_t e = p - 2; e != 0; e >>= 1) {
        if (e & 1) r = lz_mul(r, x, L);
        x = lz_mul(x, x, L);
    }
    return lz_canon(r, L);
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

struct SelArgs {
    PlainArgs w;
    const uint32_t* PR;
    int64_t ldpr;
    int32_t l0;     // leaf start column in PR
    int32_t wl;     // leaf width (1..32)
    int32_t gcol0;  // global column of leaf column 0
    int32_t gmax;   // level-0 nodes the grid covers
    int32_t ncnt;   // arrival counters per launch
    const int32_t* cand;
    const int32_t* count;
    int32_t* cnt_cur;
    int32_t* cnt_next;
    int32_t* res;
    LeafOut* out;
    uint32_t* rsave;
    int64_t ldr;
    int64_t ncopy;
    int32_t wj;      // panel width (the transform block starts at PR column wj)
    int8_t* yfrag;   // int8 B fragments of Y, or NULL
    int32_t save_rows;  // keep a copy of the pivot rows for the product to rebuild Y from
};

// Shared memory of the selection kernel.
struct Sel {
    double f[2][64];              // the current pivot column (double-buffered by step)
    double d[2];                  // its pivot value
    int32_t q[2];                 // its pivot row within the node, -1 for a free column
    double f2[2][32];             // pair steps: the second column after the first pivot
    double d2[2];
    int32_t q2[2];
    double cp[32];                // product of the pivot values before pivot s
    int32_t pos[64];              // list positions of this node's rows (lane order)
    int32_t basis[32];            // list positions of the node's basis rows (pivot order)
    int32_t rows[32];             // their row ids (final node)
    int32_t rowid[64];            // row id of each of the node's rows (lane order)
    int32_t sidx[64];             // lane -> pivot index, -1
    int32_t pl[32];               // pivot index -> lane
    int32_t pc[32];               // pivot index -> leaf column
    int32_t cpv[32];              // leaf column -> pivot index, -1 (in-place elimination)
    double total;                 // product of all pivot values
    int32_t nrows;
    int32_t t;
    int32_t bcast;
    int32_t wcount[16];           // per-wave counts of a candidate scan
};

__device__ int node_id(int level, int k, int gmax) {
    int base = 0, n = gmax;
    for (int l = 0; l < level; ++l) {
        base += n;
        n = (n + 1) >> 1;
    }
    return base + k;
}

// Register layout of the selection's Gauss-Jordan (4 waves, one per SIMD).
// R = 32 rows: lane = 32 h + row; register k of wave v holds column 8k + 4h + v
// (k < 4).  R = 64 rows: lane = row; register k holds column 4k + v (k < 8).
// Leaf columns live in v[], transform columns in T[], with the same layout.
template <int R>
struct Lay {
    static constexpr int kRegs = R == 32 ? 4 : 8;
    __device__ static int col(int wave, int h, int k) { return R == 32 ? 8 * k + 4 * h + wave : 4 * k + wave; }
    __device__ static int owner_wave(int j) { return j & 3; }
    __device__ static int owner_half(int j) { return R == 32 ? (j >> 2) & 1 : 0; }
    __device__ static int owner_reg(int j) { return R == 32 ? j >> 3 : j >> 2; }
};

// Gauss-Jordan over the leaf columns of the node's rows.  Per step the owner
// wave of column j finds the first eligible row with a non-zero entry and
// posts it with the column and the pivot value to LDS.
template <int R>
__device__ __forceinline__ void node_gj(const SelArgs& a, Sel& S, double v[8], double T[8],
                                        const Lazy& L) {
    typedef Lay<R> Y;
    const int lane = threadIdx.x & 63, wave = uniform(threadIdx.x >> 6);
    const int h = R == 32 ? lane >> 5 : 0;
    const int r = R == 32 ? lane & 31 : lane;  // this lane's row within the node
    const int nrows = S.nrows;
    const int32_t row = r < nrows ? a.cand[S.pos[r]] : -1;
    if (threadIdx.x < R) S.rowid[r] = row;
#pragma unroll
    for (int k = 0; k < Y::kRegs; ++k) {
        const int c = Y::col(wave, h, k);
        v[k] = (row >= 0 && c < a.wl) ? (double)a.PR[(int64_t)row * a.ldpr + a.l0 + c] : 0.0;
        T[k] = 0.0;
    }
    if (threadIdx.x < 64) S.sidx[threadIdx.x] = -1;
    const unsigned long long valid = nrows >= 64 ? ~0ull : ((1ull << nrows) - 1ull);
    unsigned long long chosen = 0;
    int t = 0;
    double cprod = 1.0;  // common scale of the non-pivot rows' own coefficient
    // A lazy value x in (-3p, 3p) is zero mod p iff |x| is 0, p or 2p.
    auto detect = [&](int j) {
        const int hj = Y::owner_half(j), kj = Y::owner_reg(j);
        // x = v[kj] as arithmetic (exact: one term is the value, the rest are 0),
        // which keeps the registers out of indexed scratch memory
        double x = 0.0;
#pragma unroll
        for (int k = 0; k < Y::kRegs; ++k) x = __fma_rn(v[k], k == kj ? 1.0 : 0.0, x);
        const double ax = fabs(x);
        const unsigned long long nz = __ballot(!(ax == 0.0 || ax == L.p || ax == 2.0 * L.p));
        const unsigned long long m =
            (R == 32 ? (nz >> (32 * hj)) & 0xffffffffull : nz) & valid & ~chosen;
        const int mlo = uniform((int)(uint32_t)m), mhi = uniform((int)(uint32_t)(m >> 32));
        const int q = mlo != 0 ? __builtin_ctz((uint32_t)mlo)
                               : (mhi != 0 ? 32 + __builtin_ctz((uint32_t)mhi) : -1);
        const int buf = j & 1;
        if (R == 64 || h == hj) S.f[buf][r] = x;
        const double d = q >= 0 ? readlane_d(x, R == 32 ? 32 * hj + q : q) : 0.0;
        if (lane == 0) {
            S.q[buf] = q;
            S.d[buf] = d;
        }
    };
    // this lane's copy of the pivot row's entry in register k
    auto prow = [&](double x, int q) {
        if (R == 64) return readlane_d(x, q);
        const double u0 = readlane_d(x, q), u1 = readlane_d(x, 32 + q);
        return h ? u1 : u0;
    };
    __syncthreads();
    if (wave == Y::owner_wave(0) && a.wl > 0) detect(0);
    for (int j = 0; j < a.wl; ++j) {
        __syncthreads();  // step j posted; every wave is done with step j - 1's post
        const int buf = j & 1;
        const int qv = S.q[buf];
        const double fi = S.f[buf][r];
        const double d = S.d[buf];
        const int q = uniform(qv);
        const int s = t;
        if (q >= 0) {
            if (threadIdx.x == 0) {
                S.pl[s] = q;
                S.pc[s] = j;
                S.sidx[q] = s;
                S.cp[s] = cprod;
            }
            // leaf columns first: the next column's owner posts right after
#pragma unroll
            for (int k = 0; k < Y::kRegs; ++k) {
                const int cmax = R == 32 ? 8 * k + 4 + wave : 4 * k + wave;
                if (cmax > j) {
                    const double u = prow(v[k], q);
                    const int c = Y::col(wave, h, k);
                    if (c > j && c < a.wl && r != q) v[k] = lz_ff(d, v[k], fi, u, L);
                }
            }
            chosen |= 1ull << q;
        }
        if (j + 1 < a.wl && wave == Y::owner_wave(j + 1)) detect(j + 1);
        if (q >= 0) {
#pragma unroll
            for (int k = 0; k < Y::kRegs; ++k) {
                const int cmin = R == 32 ? 8 * k + wave : 4 * k + wave;
                if (cmin <= s) {
                    const double u = prow(T[k], q);
                    const int c = Y::col(wave, h, k);
                    if (c < s) {
                        if (r != q) T[k] = lz_ff(d, T[k], fi, u, L);
                    } else if (c == s) {
                        T[k] = r == q ? cprod : -lz_mul(fi, cprod, L);
                    }
                }
            }
            cprod = lz_mul(cprod, d, L);
            t = s + 1;
        }
    }
    if (threadIdx.x == 0) {
        S.t = t;
        S.total = cprod;
    }
    __syncthreads();
    if (threadIdx.x < t) {
        S.basis[threadIdx.x] = S.pos[S.pl[threadIdx.x]];
        S.rows[threadIdx.x] = S.rowid[S.pl[threadIdx.x]];
    }
    __syncthreads();
}

// The pair layout of the 32-row elimination (two columns per step: 16
// synchronisations per leaf instead of 32).  Lane = 32 h + row; with W waves,
// register 2k + e of wave v holds column 2P + e of pair P = 2Wk + Wh + v (k, e
// in {0, 1}).
template <int W>
__device__ __forceinline__ int pair_col(int k, int h, int wave) {
    return 2 * (2 * W * (k >> 1) + W * h + wave) + (k & 1);
}

// The pivot row's entry in this lane's column of a pair-layout register: the
// value lane 32 h + q holds, fetched through the LDS crossbar (bpaddr = 4 (32 h
// + q), see pair_bpaddr), two permutes and no vector-ALU work.
__device__ __forceinline__ double pair_row(double x, int bpaddr) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_ds_bpermute(bpaddr, (int)b);
    const int hi = __builtin_amdgcn_ds_bpermute(bpaddr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}

__device__ __forceinline__ int pair_bpaddr(int q) { return (int)(((threadIdx.x & 32) + q) << 2); }

// The 32-row elimination in place: the slot of a leaf column holds that
// column until it becomes the pivot column of pivot s, and from then on column
// s of the transform T (the in-place form of Gauss-Jordan inversion).  Every
// slot is then live at every step, so a lane updates its 16 / W slots per pivot
// instead of the live part of 16 / W leaf and 16 / W transform registers.  The
// slots follow the pair layout (slot k = register k of pair_col<W>): the
// owner wave of pair P first brings the pair's two slots up to date, posts
// both pivots, then updates its other slots.  A pivot (row q, value d, column
// j, column values f) maps every slot of every row but q to d x - f x_q, and
// slot j to cprod on row q and -f cprod elsewhere (the new pivot's transform
// column).  Slots of free columns hold values that nothing reads.  The owner
// wave of pair P finds the first column's pivot, applies it to the second
// column itself, finds the second pivot and posts both; every wave then applies
// the two pivots in order, which gives the results of one column per step.
// S.cpv maps a column to its pivot.
template <int W>
__device__ __forceinline__ void node_gj_inplace(const SelArgs& a, Sel& S, double x[], const Lazy& L) {
    static_assert(W == 4 || W == 8, "four or eight waves");
    constexpr int NR = 16 / W;  // slots per lane
    const int lane = threadIdx.x & 63, wave = uniform(threadIdx.x >> 6);
    const int h = lane >> 5, r = lane & 31;
    const int nrows = S.nrows;
    const int32_t row = r < nrows ? a.cand[S.pos[r]] : -1;
    if (threadIdx.x < 32) S.rowid[r] = row;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int c = pair_col<W>(k, h, wave);
        x[k] = (row >= 0 && c < a.wl) ? (double)a.PR[(int64_t)row * a.ldpr + a.l0 + c] : 0.0;
    }
    if (threadIdx.x < 64) S.sidx[threadIdx.x] = -1;
    if (threadIdx.x < 32) S.cpv[threadIdx.x] = -1;
    const unsigned long long valid = nrows >= 32 ? 0xffffffffull : ((1ull << nrows) - 1ull);
    unsigned long long chosen = 0;  // rows of this node (bits 0..31)
    int t = 0;
    double cprod = 1.0;
    auto first_nz = [&](double v, int hh, unsigned long long excl) {
        const double av = fabs(v);  // lazy value in (-3p, 3p): zero iff |v| is 0, p or 2p
        const unsigned long long nz = __ballot(!(av == 0.0 || av == L.p || av == 2.0 * L.p));
        const unsigned long long m = ((nz >> (32 * hh)) & 0xffffffffull) & valid & ~excl;
        const int mlo = uniform((int)(uint32_t)m);
        return mlo != 0 ? __builtin_ctz((uint32_t)mlo) : -1;
    };
    const int npairs = (a.wl + 1) >> 1;
    // owner of pair P (wave P % W, half (P / W) & 1, slots 2 kp and 2 kp + 1
    // with kp = P / 2W): both pivots of the pair, posted
    auto detect = [&](int P) {
        const int hp = (P / W) & 1, kp = P / (2 * W);
        double xa = x[0];
        double xb = x[1];
        if constexpr (NR == 4) {
            if (kp != 0) {  // (uniform)
                xa = x[2];
                xb = x[3];
            }
        }
        const int q1 = first_nz(xa, hp, chosen);
        const double d1 = q1 >= 0 ? readlane_d(xa, 32 * hp + q1) : 0.0;
        if (q1 >= 0) {
            const double ub = readlane_d(xb, 32 * hp + q1);
            if (r != q1) xb = lz_ff(d1, xb, xa, ub, L);
        }
        int q2 = -1;
        double d2 = 0.0;
        if (2 * P + 1 < a.wl) {
            q2 = first_nz(xb, hp, chosen | (q1 >= 0 ? 1ull << q1 : 0ull));
            d2 = q2 >= 0 ? readlane_d(xb, 32 * hp + q2) : 0.0;
        }
        const int buf = P & 1;
        if (h == hp) {
            S.f[buf][r] = xa;
            S.f2[buf][r] = xb;
        }
        if (lane == 0) {
            S.q[buf] = q1;
            S.d[buf] = d1;
            S.q2[buf] = q2;
            S.d2[buf] = d2;
        }
    };
    // one pivot on slots K0..K1-1: d x - f x_q off the pivot row, inj (the
    // transform column's start) in the pivot column's slot
    auto apply = [&](auto k0, auto k1, int q, double d, double f, int j, double inj) {
        constexpr int K0 = decltype(k0)::value, K1 = decltype(k1)::value;
        const int bp = pair_bpaddr(q);
        double u[4], y[4];
#pragma unroll
        for (int k = K0; k < K1; ++k) u[k] = pair_row(x[k], bp);
        lz_ff_n<K0, K1>(y, d, x, f, u, L);
#pragma unroll
        for (int k = K0; k < K1; ++k)
            x[k] = pair_col<W>(k, h, wave) == j ? inj : (r != q ? y[k] : x[k]);
    };
    using I0 = std::integral_constant<int, 0>;
    using I2 = std::integral_constant<int, 2>;
    using IN = std::integral_constant<int, NR>;
    __syncthreads();
    if (wave == 0 && a.wl > 0) detect(0);
    for (int P = 0; P < npairs; ++P) {
        __syncthreads();  // pair P posted; every wave is done with pair P - 1's post
        const int buf = P & 1;
        const int q1v = S.q[buf], q2v = S.q2[buf];
        const double f1 = S.f[buf][r], f2 = S.f2[buf][r];
        const double d1 = S.d[buf], d2 = S.d2[buf];
        const int q1 = uniform(q1v), q2 = uniform(q2v);
        const int j = 2 * P;
        const int s1 = t, s2 = t + (q1 >= 0);
        const double cp2 = q1 >= 0 ? lz_mul(cprod, d1, L) : cprod;  // cprod after pivot 1
        if (threadIdx.x == 0) {
            if (q1 >= 0) {
                S.pl[s1] = q1;
                S.pc[s1] = j;
                S.cpv[j] = s1;
                S.sidx[q1] = s1;
                S.cp[s1] = cprod;
            }
            if (q2 >= 0) {
                S.pl[s2] = q2;
                S.pc[s2] = j + 1;
                S.cpv[j + 1] = s2;
                S.sidx[q2] = s2;
                S.cp[s2] = cp2;
            }
        }
        const double inj1 = r == q1 ? cprod : -lz_mul(f1, cprod, L);
        const double inj2 = r == q2 ? cp2 : -lz_mul(f2, cp2, L);
        const bool owner = P + 1 < npairs && wave == (P + 1) % W;
        if (NR == 4 && owner) {
            // the next pair's owner: that pair's two slots, its post, the rest
            if ((P + 1) / (2 * W) == 0) {
                if (q1 >= 0) apply(I0{}, I2{}, q1, d1, f1, j, inj1);
                if (q2 >= 0) apply(I0{}, I2{}, q2, d2, f2, j + 1, inj2);
            } else {
                if (q1 >= 0) apply(I2{}, IN{}, q1, d1, f1, j, inj1);
                if (q2 >= 0) apply(I2{}, IN{}, q2, d2, f2, j + 1, inj2);
            }
            if (q1 >= 0) chosen |= 1ull << q1;
            if (q2 >= 0) chosen |= 1ull << q2;
            detect(P + 1);
            if ((P + 1) / (2 * W) == 0) {
                if (q1 >= 0) apply(I2{}, IN{}, q1, d1, f1, j, inj1);
                if (q2 >= 0) apply(I2{}, IN{}, q2, d2, f2, j + 1, inj2);
            } else {
                if (q1 >= 0) apply(I0{}, I2{}, q1, d1, f1, j, inj1);
                if (q2 >= 0) apply(I0{}, I2{}, q2, d2, f2, j + 1, inj2);
            }
        } else {
            if (q1 >= 0) apply(I0{}, IN{}, q1, d1, f1, j, inj1);
            if (q2 >= 0) apply(I0{}, IN{}, q2, d2, f2, j + 1, inj2);
            if (q1 >= 0) chosen |= 1ull << q1;
            if (q2 >= 0) chosen |= 1ull << q2;
            if (owner) detect(P + 1);
        }
        cprod = q2 >= 0 ? lz_mul(cp2, d2, L) : cp2;
        t = s2 + (q2 >= 0);
    }
    if (threadIdx.x == 0) {
        S.t = t;
        S.total = cprod;
    }
    __syncthreads();
    if (threadIdx.x < t) {
        S.basis[threadIdx.x] = S.pos[S.pl[threadIdx.x]];
        S.rows[threadIdx.x] = S.rowid[S.pl[threadIdx.x]];
    }
    __syncthreads();
}

// The first kChunk candidates (in list order) that are non-zero somewhere in
// the leaf, into S.pos and S.nrows, by a workgroup of NW waves scanning the
// list in order.
template <int NW>
__device__ void pick_nonzero_rows(const SelArgs& a, Sel& S, int E) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int found = 0;
    for (int base = 0; base < E && found < kChunk; base += 64 * NW) {
        const int i = base + threadIdx.x;
        bool nz = false;
        if (i < E) {  // the leaf's columns of a row: one 128-byte aligned segment
            const uint32_t* rp = a.PR + (int64_t)a.cand[i] * a.ldpr + a.l0;
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const v4i q = *(const v4i*)(rp + 4 * h);
#pragma unroll
                for (int e = 0; e < 4; ++e) nz |= 4 * h + e < a.wl && q[e] != 0;
            }
        }
        const unsigned long long b = __ballot(nz);
        if (lane == 0) S.wcount[wave] = (int)__popcll(b);
        __syncthreads();
        int before = found, total = 0;
        for (int w = 0; w < NW; ++w) {
            before += w < wave ? S.wcount[w] : 0;
            total += S.wcount[w];
        }
        const int rank = before + (int)__popcll(b & ((1ull << lane) - 1ull));
        if (nz && rank < kChunk) S.pos[rank] = i;
        found += total;
        __syncthreads();  // the counts are rewritten by the next round
    }
    if (threadIdx.x == 0) S.nrows = min(found, kChunk);
    __syncthreads();
}

// Final node: P^-1, the leaf result, the pivot bookkeeping, and a copy of the
// pivot rows over the columns the leaf updates (the product overwrites them).
// R = 32: the pair layout of node_gj_inplace; R = 64: the layout of node_gj<64>.
// kInPlace: T comes from node_gj_inplace (slot of leaf column c = transform
// column S.cpv[c]).
template <int R, int W, bool kInPlace = false>
__device__ __forceinline__ void publish(const SelArgs& a, Sel& S, const double T[8], bool save_rows,
                                        const Lazy& L) {
    static_assert(!kInPlace || (R == 32 && (W == 4 || W == 8)), "the in-place layout has four or eight waves");
    static_assert(R == 32 || W == 4, "the 64-row layout has four waves");
    constexpr int NR = R == 32 ? 16 / W : 8;  // transform registers per lane
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = R == 32 ? lane >> 5 : 0;
    const int r = R == 32 ? lane & 31 : lane;
    auto colof = [&](int k) {
        return R == 32 ? pair_col<W>(k, h, wave) : Lay<64>::col(wave, 0, k);
    };
    const int t = S.t;  // (S.rows was set by the elimination that precedes every publish)
    if (threadIdx.x == 0) {
        __hip_atomic_store(a.cnt_cur + (a.ncnt - 1), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S.bcast = a.w.state[0];
        if (t > 0) S.total = lz_inverse(lz_canon(S.total, L), a.w.F.p, L);
    } else if (threadIdx.x >= 64 && t > 0 && save_rows) {  // meanwhile the other waves save the rows
        for (int64_t c = threadIdx.x - 64; c < a.ncopy; c += 64 * W - 64) {
            // eight loads in flight before their stores; pivots k >= t reuse pivot
            // 0's row (S.rows[0] is set because t > 0)
            for (int k0 = 0; k0 < 32; k0 += 8) {
                uint32_t x[8];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    x[k] = a.PR[(int64_t)S.rows[k0 + k < t ? k0 + k : 0] * a.ldpr + a.l0 + c];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k0 + k < t) a.rsave[(k0 + k) * a.ldr + c] = x[k];
            }
        }
    }
    __syncthreads();
    const int s = r < S.nrows ? S.sidx[r] : -1;
    if (s >= 0) {
        const double dinv = lz_mul(S.cp[s], S.total, L);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int c = kInPlace ? S.cpv[colof(k)] : colof(k);
            if (kInPlace ? c >= 0 : c < t)
                a.out->pinv[s * 32 + c] = (uint32_t)lz_canon(lz_mul(dinv, T[k], L), L);
        }
    }
    const int r0 = S.bcast;
    if (threadIdx.x < t) {
        const int i = threadIdx.x;
        const int row = S.rows[i];
        const int gcol = a.gcol0 + S.pc[i];
        a.out->pos[i] = S.basis[i];
        a.out->row[i] = row;
        a.out->col[i] = S.pc[i];
        a.w.pivrow[r0 + i] = row;
        a.w.pivcol[r0 + i] = gcol;
        a.w.colpiv[gcol] = r0 + i;
        a.w.rowcol[row] = gcol;
        a.w.is_piv[row] = 1u;
        a.w.slots[gcol] = ((unsigned long long)row << 32) | 1ull;
    }
    if (threadIdx.x == 0) {
        a.out->t = t;
        a.out->yready = 0;
        a.w.state[0] = r0 + t;
    }
}

// One 32-column block of Y = P^-1 R (R = the pivot rows over the leaf's update
// columns, with each new pivot's implicit 1 in the transform block) as int8 B
// fragments: thread (s, c) forms Y[s][c] with exact 16-bit-split FP64 sums and
// writes its four digits into the fragment's byte layout (digit plane l, lane
// c + 32 (s / 16), byte s % 16).
__device__ void build_y_block(const SelArgs& a, int g, const Lazy& L) {
    __shared__ uint32_t sP[32][33];
    __shared__ uint32_t sR[32][33];
    // the two 16-column blocks of this 32-column slice, in the B lanes of the
    // 16x16x32 int8 MFMA: Y(s, c) in lane c + 16 (s / 8), byte s % 8
    __shared__ __attribute__((aligned(16))) int8_t sB[2][4][64][8];
    const int tid = threadIdx.x;
    const int t = a.out->t;
    for (int i = tid; i < 32 * 32; i += kSelThreads) {  // stage R[k][c] and Pinv[k][c]
        const int k = i >> 5, c = i & 31;
        const int64_t col = (int64_t)g * 32 + c;
        const int krow = a.out->row[k < t ? k : 0];
        const int kcol = a.out->col[k];
        const int64_t colc = col < a.ncopy ? col : a.ncopy - 1;
        const uint32_t rv = a.PR[(int64_t)(t > 0 ? krow : 0) * a.ldpr + a.l0 + colc];
        const uint32_t pv = a.out->pinv[k * 32 + c];
        sR[k][c] = (k < t && col < a.ncopy) ? (col == (int64_t)a.wj + kcol ? 1u : rv) : 0u;
        sP[k][c] = (k < t && c < t) ? pv : 0u;
    }
    __syncthreads();
    const uint32_t p = a.w.F.p;
    for (int i = tid; i < 32 * 32; i += kSelThreads) {
        const int s = i >> 5, c = i & 31;
        double s1 = 0.0, s0 = 0.0;
        for (int k = 0; k < t; ++k) {
            const uint32_t pv = sP[s][k];
            const double r = (double)sR[k][c];
            s1 = __fma_rn((double)(pv >> 16), r, s1);
            s0 = __fma_rn((double)(pv & 0xffffu), r, s0);
        }
        // s1 < 2^51, s0 < 2^52: exact; (s1 mod p) 2^16 + s0 < 2^53
        const uint32_t yv = (uint32_t)lz_canon_wide(__fma_rn(lz_canon_wide(s1, L), 65536.0, s0), L);
        int32_t x = yv > (p - 1) / 2 ? (int32_t)yv - (int32_t)p : (int32_t)yv;
        for (int l = 0; l < 4; ++l) {
            const int8_t dg = (int8_t)(x & 0xff);
            sB[c >> 4][l][(c & 15) + 16 * (s >> 3)][s & 7] = dg;
            x = (x - dg) >> 8;
        }
    }
    __syncthreads();
    {  // plane l of 16-column block b at (4 b + l) * 512 bytes; 16 bytes (two lanes) per thread
        const int half = tid >> 7, l = (tid >> 5) & 3, L2 = (tid & 31) * 2;
        *(v4i*)(a.yfrag + ((int64_t)(2 * g + half) * 4 + l) * 512 + L2 * 8) =
            *(const v4i*)&sB[half][l][L2][0];
    }
}

// The first chunk of candidates alone, by one workgroup of kFirstThreads:
// publishes when that chunk already has full rank in the leaf (as with dense
// data) or holds every candidate.
__device__ void select_first_block(const SelArgs& a) {
    __shared__ Sel S;
    const Lazy L{(double)a.w.F.p, a.w.F.pinv};
    const int E = *a.count;
    if (E == 0) {
        if (threadIdx.x == 0) {
            __hip_atomic_store(a.cnt_cur + (a.ncnt - 1), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            a.out->t = 0;
            a.out->yready = 0;
        }
        return;
    }
    if (threadIdx.x < 64) S.pos[threadIdx.x] = threadIdx.x;
    if (threadIdx.x == 0) S.nrows = min(kChunk, E);
    __syncthreads();
    static_assert(kFirstWaves == 8, "the in-place elimination has eight waves");
    double x[8];
    node_gj_inplace<kFirstWaves>(a, S, x, L);
    if (S.t == a.wl || E <= kChunk) publish<32, kFirstWaves, true>(a, S, x, a.save_rows && !a.yfrag, L);
}

// The last arrival counter of each set is the "published" flag: once the final
// node is known, workgroups still merging stop at their next tree level.
//
// Two launches per leaf: `first` runs the first chunk alone (one workgroup, no
// other work on the device; select_first_block) and publishes when that chunk
// already has full rank, as with dense data; the full tree launch then finds
// the result published and ends at once, or selects over all candidates.
template <bool first>
__global__ __launch_bounds__(first ? kFirstThreads : kSelThreads, first ? 2 : 1) void leaf_select_kernel(
    SelArgs a) {
    if (first) {
        select_first_block(a);
        return;
    }
    __shared__ Sel S;
    const Lazy L{(double)a.w.F.p, a.w.F.pinv};
    int32_t* published = a.cnt_cur + (a.ncnt - 1);
    for (int i = blockIdx.x * kSelThreads + threadIdx.x; i < a.ncnt; i += gridDim.x * kSelThreads)
        a.cnt_next[i] = 0;
    const int E = *a.count;
    const int G = (E + kChunk - 1) / kChunk;
    const int g = blockIdx.x;
    if (threadIdx.x == 0)
        S.bcast = __hip_atomic_load(published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (S.bcast != 0) {  // decided by the first launch: build Y instead
        if (a.yfrag && (int64_t)g * 32 < a.ncopy) build_y_block(a, g, L);
        if (a.yfrag && g == 0 && threadIdx.x == 0) a.out->yready = 1;
        return;
    }
    if (E == 0 || g >= G) return;  // (E = 0 was published by the first launch)
    if (threadIdx.x < 64) S.pos[threadIdx.x] = g * kChunk + threadIdx.x;
    if (threadIdx.x == 0) S.nrows = min(kChunk, E - g * kChunk);
    __syncthreads();
    int level = 0, k = g, nodes = G;
    double v[8], T[8];
    // Chunk 0 of the tree takes the first kChunk candidates that are non-zero
    // in the leaf: rows that are combinations of earlier pivot rows stay
    // candidates and gather at the front of the list, zero in every later
    // leaf, and are what keeps the first chunk short of full rank.  A zero row
    // adds nothing to the leaf's span, so node (level, 0) still spans what the
    // candidates before its range span, and the tree's finality rule holds.
    if (g == 0) pick_nonzero_rows<kSelWaves>(a, S, E);
    node_gj_inplace<kSelWaves>(a, S, T, L);
    int regs = 32;  // T holds the in-place Gauss-Jordan of the node's basis rows (64: v, T of node_gj<64>; 0: none)
    while (true) {
        const int t = S.t;
        if ((k == 0 && t == a.wl) || nodes == 1) {
            if (regs == 0) {  // a basis passed up without elimination: reduce it now
                if (threadIdx.x < t) S.pos[threadIdx.x] = S.basis[threadIdx.x];
                if (threadIdx.x == 0) S.nrows = t;
                __syncthreads();
                node_gj_inplace<kSelWaves>(a, S, T, L);
                regs = 32;
            }
            // the tree launch leaves Y to the product, which needs the rows as selected
            const bool save_rows = a.save_rows != 0;
            if (regs == 32) publish<32, kSelWaves, true>(a, S, T, save_rows, L);
            else publish<64, kSelWaves>(a, S, T, save_rows, L);
            return;
        }
        const int up = (nodes + 1) >> 1;
        if ((k ^ 1) >= nodes) {  // no sibling: the node passes up unchanged
            ++level;
            k >>= 1;
            nodes = up;
            continue;
        }
        int32_t* mine = a.res + (int64_t)node_id(level, k, a.gmax) * kNodeInts;
        if (threadIdx.x < t) mine[1 + threadIdx.x] = S.basis[threadIdx.x];
        if (threadIdx.x == 0) mine[0] = t;
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            const int old = atomicAdd(&a.cnt_cur[node_id(level + 1, k >> 1, a.gmax)], 1);
            S.bcast = old == 0 ? 1
                               : __hip_atomic_load(published, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        // first of the two siblings (the other merges later), or already published
        if (S.bcast != 0) return;
        __threadfence();
        const int32_t* lres = a.res + (int64_t)node_id(level, k & ~1, a.gmax) * kNodeInts;
        const int32_t* rres = a.res + (int64_t)node_id(level, k | 1, a.gmax) * kNodeInts;
        const int tl = __hip_atomic_load(lres, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int tr = __hip_atomic_load(rres, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();  // every thread has read S.t before it changes
        // a full left basis spans everything; an empty side adds nothing: no
        // elimination needed, the other side's basis is the merged one
        const bool lazy = tl == a.wl || tl == 0 || tr == 0;
        const int32_t* one = tl == a.wl || tr == 0 ? lres : rres;
        const int tone = tl == a.wl || tr == 0 ? tl : tr;
        if (lazy) {
            if (threadIdx.x < tone)
                S.basis[threadIdx.x] = __hip_atomic_load(one + 1 + threadIdx.x, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            if (threadIdx.x == 0) S.t = tone;
        } else {
            if (threadIdx.x < tl)
                S.pos[threadIdx.x] = __hip_atomic_load(lres + 1 + threadIdx.x, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            else if (threadIdx.x < tl + tr)
                S.pos[threadIdx.x] = __hip_atomic_load(rres + 1 + threadIdx.x - tl,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (threadIdx.x == 0) S.nrows = tl + tr;
        }
        __syncthreads();
        if (lazy) {
            regs = 0;
        } else {
            node_gj<64>(a, S, v, T, L);
            regs = 64;
        }
        ++level;
        k >>= 1;
        nodes = up;
    }
}

// Leaf l's product on every row but leaf l + 1's first chunk (workgroups 1..,
// kFirstWaves x 16 rows each, rbx row blocks per column group) and leaf l + 1's
// first selection on that chunk (workgroup 0) in one launch.  The two touch
// disjoint data: the selection reads the chunk rows (updated by the chunk half
// before this launch) and writes leaf l + 1's result and the bookkeeping of its
// pivot rows; the product reads leaf l's result and writes the other rows and
// the next candidate list.
template <int kLeafBlocks>
// (at most 128 VGPRs, so that two workgroups fit on a compute unit: with the
// tuned six column blocks the product half needs 132 otherwise)
__global__ __attribute__((amdgpu_flat_work_group_size(kFirstThreads, kFirstThreads),
                          amdgpu_waves_per_eu(4, 8))) void leaf_fused_kernel(SelArgs sa, LeafProdArgs pa,
                                                                     int32_t rbx) {
    if (blockIdx.x == 0) {
        select_first_block(sa);
        return;
    }
    const int64_t b = (int64_t)blockIdx.x - 1;
    leaf_product_block<kLeafBlocks, kLeafRest, kFirstWaves>(pa, b % rbx, b / rbx, b);
}

__global__ void leaf_init_kernel(int32_t* cand, int32_t* count, int32_t* cnt, int32_t ncnt2,
                                 int32_t m) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < m; i += stride) cand[i] = (int32_t)i;
    for (int64_t i = tid; i < ncnt2; i += stride) cnt[i] = 0;
    if (tid == 0) count[0] = m;
}

struct OpArgs {
    PlainArgs w;
    const uint32_t* PR;
    int64_t ldpr;
    int32_t l0, wl, wj, gcol0;
    int64_t N;  // PR columns [l0, l0 + N) are updated
    const LeafOut* out;
    const int32_t* cand;
    int32_t* cand_next;
    const int32_t* count;
    int32_t* count_next;
    void* Afrag;
    void* Bfrag;
    int32_t nyb, nab;  // blocks of the Y and A parts (the rest compact the list)
    int32_t fp64;
};

// Y part: one block per 32 update columns.  Y[s][c] = sum_s' Pinv[s][s'] R[s'][c]
// with Pinv split into 15- and 16-bit halves, so both partial sums stay below
// 2^53 and accumulate exactly in FP64.
__device__ void operands_y(const OpArgs& a, int b) {
    __shared__ uint32_t sR[32][33];
    __shared__ uint32_t sP[32][33];
    __shared__ uint32_t sY[32][33];
    const int tid = threadIdx.x;
    const int t = a.out->t;
    const FieldConst& F = a.w.F;
    const int64_t c0 = (int64_t)b * 32;
    for (int i = tid; i < 32 * 32; i += 256) {
        const int s = i >> 5, c = i & 31;
        uint32_t r = 0, pv = 0;
        if (s < t) {
            const int64_t col = c0 + c;
            if (col < a.N) {
                r = a.PR[(int64_t)a.out->row[s] * a.ldpr + a.l0 + col];
                if (col == (int64_t)a.wj + a.out->col[s]) r = 1u;  // the new pivot's implicit 1
            }
            if (c < t) pv = a.out->pinv[s * 32 + c];
        }
        sR[s][c] = r;
        sP[s][c] = pv;
    }
    __syncthreads();
    {
        const int s = tid >> 3, cb = (tid & 7) * 4;
        double s1[4] = {0.0, 0.0, 0.0, 0.0}, s0[4] = {0.0, 0.0, 0.0, 0.0};
        if (s < t) {
            for (int k = 0; k < t; ++k) {
                const uint32_t pv = sP[s][k];
                const double hi = (double)(pv >> 16), lo = (double)(pv & 0xffffu);
                for (int e = 0; e < 4; ++e) {
                    const double r = (double)sR[k][cb + e];
                    s1[e] = __fma_rn(hi, r, s1[e]);
                    s0[e] = __fma_rn(lo, r, s0[e]);
                }
            }
        }
        const Lazy L{F.dp, F.pinv};
        for (int e = 0; e < 4; ++e) {
            const double h = lz_canon_wide(s1[e], L);
            sY[s][cb + e] = (uint32_t)lz_canon_wide(__fma_rn(h, 65536.0, s0[e]), L);
        }
    }
    __syncthreads();
    if (!a.fp64) {
        // int8 B fragment (cb = b, one k-block): digit plane l', lane L holds
        // column L % 32 and rows 16 (L / 32) + i
        if (tid < 64) {
            const int L = tid;
            int8_t outb[4][16];
            for (int i = 0; i < 16; ++i) {
                int8_t d[4];
                digits4(centre(sY[16 * (L >> 5) + i][L & 31], F.p), d);
                for (int lp = 0; lp < 4; ++lp) outb[lp][i] = d[lp];
            }
            int8_t* base = (int8_t*)a.Bfrag + (int64_t)b * 4 * 1024 + L * 16;
            for (int lp = 0; lp < 4; ++lp) {
                v4i vv;
                __builtin_memcpy(&vv, outb[lp], 16);
                *(v4i*)(base + lp * 1024) = vv;
            }
        }
    } else {
        // FP64 B fragments (cb16 = 2b, 2b + 1; 8 k-blocks of 4): lane L holds
        // row 4 kb + L / 16, column 16 cb16 + L % 16
        double* Bd = (double*)a.Bfrag;
        for (int i = tid; i < 2 * 8 * 64; i += 256) {
            const int half = i >> 9, kb = (i >> 6) & 7, L = i & 63;
            const uint32_t y = sY[kb * 4 + (L >> 4)][half * 16 + (L & 15)];
            Bd[(((int64_t)(2 * b + half)) * 8 + kb) * 64 + L] = (double)centre(y, F.p);
        }
    }
}

// Multiplier of row `row` for leaf pivot k: -L[row, C_k], or the unit vector e_s
// for the leaf's own pivot row s.
__device__ __forceinline__ uint32_t a_value(const OpArgs& a, int64_t row, int k, int t, int sel,
                                            const int32_t* cols) {
    if (row >= a.w.m || k >= t) return 0u;
    if (sel >= 0) return k == sel ? 1u : 0u;
    const uint32_t x = a.PR[row * a.ldpr + a.l0 + cols[k]];
    return x == 0 ? 0u : a.w.F.p - x;
}

__device__ __forceinline__ int leaf_sel(const OpArgs& a, int64_t row, const int32_t* cols, int t) {
    if (row >= a.w.m) return -1;
    const int rc = a.w.rowcol[row] - a.gcol0;
    if (rc < 0 || rc >= a.wl) return -1;
    for (int s = 0; s < t; ++s)
        if (cols[s] == rc) return s;
    return -1;
}

__device__ void operands_a(const OpArgs& a, int b) {
    __shared__ int32_t cols[32];
    const int tid = threadIdx.x;
    const int t = a.out->t;
    if (tid < 32) cols[tid] = tid < t ? a.out->col[tid] : 0;
    __syncthreads();
    const uint32_t p = a.w.F.p;
    if (!a.fp64) {
        // int8 A fragment (rb, one k-block, limb l): lane L holds row 32 rb + L % 32
        // and k = 16 (L / 32) + i
        const int L = tid & 63;
        const int64_t rb = (int64_t)b * 4 + (tid >> 6);
        const int64_t row = rb * 32 + (L & 31);
        const int sel = leaf_sel(a, row, cols, t);
        int8_t outb[4][16];
        for (int i = 0; i < 16; ++i) {
            const int k = 16 * (L >> 5) + i;
            int8_t d[4];
            digits4(centre(a_value(a, row, k, t, sel, cols), p), d);
            for (int l = 0; l < 4; ++l) outb[l][i] = d[l];
        }
        int8_t* base = (int8_t*)a.Afrag + rb * 4 * 1024 + L * 16;
        for (int l = 0; l < 4; ++l) {
            v4i vv;
            __builtin_memcpy(&vv, outb[l], 16);
            *(v4i*)(base + l * 1024) = vv;
        }
    } else {
        // FP64 A fragment (rb of 16 rows, kb of 4): lane L holds row 16 rb + L % 16,
        // k = 4 kb + L / 16; a block covers 2 row blocks x 8 k-blocks x 64 lanes
        double* Ad = (double*)a.Afrag;
        for (int i = tid; i < 2 * 8 * 64; i += 256) {
            const int64_t rb = (int64_t)b * 2 + (i >> 9);
            const int kb = (i >> 6) & 7, L = i & 63;
            const int64_t row = rb * 16 + (L & 15);
            const int sel = leaf_sel(a, row, cols, t);
            Ad[(rb * 8 + kb) * 64 + L] =
                (double)centre(a_value(a, row, kb * 4 + (L >> 4), t, sel, cols), p);
        }
    }
}

__global__ __launch_bounds__(256) void leaf_operands_kernel(OpArgs a) {
    const int b = blockIdx.x;
    if (b < a.nyb) {
        operands_y(a, b);
    } else if (b < a.nyb + a.nab) {
        operands_a(a, b - a.nyb);
    } else {
        const int64_t i = (int64_t)(b - a.nyb - a.nab) * 256 + threadIdx.x;
        const int t = a.out->t, E = *a.count;
        if (i == 0) *a.count_next = E - t;
        leaf_compact_entry(a.out, t, a.cand, a.cand_next, E, i);
    }
}

}  // namespace

int32_t leaf_nodes(int64_t m) {
    int64_t n = ceil_div(m > 0 ? m : 1, kChunk), tot = 0;
    while (true) {
        tot += n;
        if (n == 1) break;
        n = (n + 1) / 2;
    }
    return (int32_t)(tot + 1);
}

void leaf_carve(Carver& c, int64_t m, int64_t ldr, LeafState* ls) {
    const int32_t nodes = leaf_nodes(m);
    int32_t* cand0 = c.take<int32_t>(m > 0 ? m : 1);
    int32_t* cand1 = c.take<int32_t>(m > 0 ? m : 1);
    int32_t* count = c.take<int32_t>(64);
    int32_t* cnt = c.take<int32_t>(2 * (int64_t)nodes);
    int32_t* res = c.take<int32_t>((int64_t)nodes * kNodeInts);
    LeafOut* out = c.take<LeafOut>(2);
    int32_t* chunk = c.take<int32_t>(64);
    uint32_t* rsave = c.take<uint32_t>(32 * ldr);
    if (ls) {
        ls->rsave = rsave;
        ls->chunk = chunk;
        ls->ldr = ldr;
        ls->cand[0] = cand0;
        ls->cand[1] = cand1;
        ls->count = count;
        ls->cnt[0] = cnt;
        ls->cnt[1] = cnt + nodes;
        ls->res = res;
        ls->out[0] = out;
        ls->out[1] = out + 1;
        ls->nodes = nodes;
        ls->gmax = (int32_t)ceil_div(m > 0 ? m : 1, kChunk);
    }
}

hipError_t leaf_init(const LeafState& ls, int32_t m, hipStream_t s) {
    const int64_t work = m > 2 * ls.nodes ? m : 2 * ls.nodes;
    const unsigned blocks = (unsigned)(ceil_div(work, 256) < 1024 ? ceil_div(work, 256) : 1024);
    hipLaunchKernelGGL(leaf_init_kernel, dim3(blocks), dim3(256), 0, s, ls.cand[0], ls.count,
                       ls.cnt[0], 2 * ls.nodes, m);
    return hipGetLastError();
}

namespace {

SelArgs sel_args(const PlainArgs& w, const LeafState& ls, const uint32_t* PR, int64_t ldpr,
                 int32_t l0, int32_t wl, int32_t wj, int32_t gcol0, int32_t parity, int64_t ncopy,
                 int8_t* yfrag, bool save_rows) {
    SelArgs a;
    a.w = w;
    a.PR = PR;
    a.ldpr = ldpr;
    a.l0 = l0;
    a.wl = wl;
    a.gcol0 = gcol0;
    a.gmax = ls.gmax;
    a.ncnt = ls.nodes;
    a.cand = ls.cand[parity];
    a.count = ls.count + parity;
    a.cnt_cur = ls.cnt[parity];
    a.cnt_next = ls.cnt[parity ^ 1];
    a.res = ls.res;
    a.out = ls.out[parity];
    a.rsave = ls.rsave;
    a.ldr = ls.ldr;
    a.ncopy = ncopy;
    a.wj = wj;
    a.yfrag = yfrag;
    a.save_rows = save_rows ? 1 : 0;
    return a;
}

}  // namespace

hipError_t leaf_select(const PlainArgs& w, const LeafState& ls, const uint32_t* PR, int64_t ldpr,
                       int32_t l0, int32_t wl, int32_t wj, int32_t gcol0, int32_t parity,
                       int64_t ncopy, int8_t* yfrag, bool save_rows, hipStream_t s, int stages,
                       bool from_chunk) {
    const SelArgs a = sel_args(w, ls, PR, ldpr, l0, wl, wj, gcol0, parity, ncopy, yfrag, save_rows);
    const int64_t nyb = ceil_div(ncopy, 32);
    const unsigned grid = (unsigned)(ls.gmax > nyb ? ls.gmax : nyb);
    if (stages & kSelectFirst) {
        SelArgs f = a;
        if (from_chunk) {  // positions 0..31 of the new list are the chunk's entries
            f.cand = ls.chunk;
            f.count = ls.chunk + 32;
        }
        hipLaunchKernelGGL(leaf_select_kernel<true>, dim3(1), dim3(kFirstThreads), 0, s, f);
    }
    if (stages & kSelectRest)
        hipLaunchKernelGGL(leaf_select_kernel<false>, dim3(grid), dim3(kSelThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t leaf_fused(const PlainArgs& w, const LeafState& ls, const uint32_t* PR, int64_t ldpr,
                      int32_t l0, int32_t wl, int32_t wj, int32_t gcol0, int32_t parity,
                      int64_t ncopy, int8_t* yfrag, const LeafProdArgs& pa, int32_t leaf_blocks,
                      hipStream_t s) {
    SelArgs a = sel_args(w, ls, PR, ldpr, l0, wl, wj, gcol0, parity, ncopy, yfrag, true);
    a.cand = ls.chunk;  // positions 0..31 of the new list are the chunk's entries
    a.count = ls.chunk + 32;
    const int64_t rbx = ceil_div(w.m > 0 ? w.m : 1, 16 * kFirstWaves);
#define LEAF_FUSED(LB)                                                                            \
    hipLaunchKernelGGL(leaf_fused_kernel<LB>,                                                     \
                       dim3((unsigned)(1 + rbx * ceil_div(pa.N, 16 * (LB)))), dim3(kFirstThreads), \
                       0, s, a, pa, (int32_t)rbx)
    if (leaf_blocks >= 9) LEAF_FUSED(9);
    else if (leaf_blocks >= 6) LEAF_FUSED(6);
    else if (leaf_blocks >= 3) LEAF_FUSED(3);
    else LEAF_FUSED(2);
#undef LEAF_FUSED
    return hipGetLastError();
}

hipError_t leaf_operands(const PlainArgs& w, const LeafState& ls, const uint32_t* PR, int64_t ldpr,
                         int32_t l0, int32_t wl, int32_t wj, int32_t gcol0, int64_t N,
                         int32_t parity, bool fp64, void* Afrag, void* Bfrag, hipStream_t s) {
    OpArgs a;
    a.w = w;
    a.PR = PR;
    a.ldpr = ldpr;
    a.l0 = l0;
    a.wl = wl;
    a.wj = wj;
    a.gcol0 = gcol0;
    a.N = N;
    a.out = ls.out[parity];
    a.cand = ls.cand[parity];
    a.cand_next = ls.cand[parity ^ 1];
    a.count = ls.count + parity;
    a.count_next = ls.count + (parity ^ 1);
    a.Afrag = Afrag;
    a.Bfrag = Bfrag;
    a.fp64 = fp64 ? 1 : 0;
    a.nyb = (int32_t)ceil_div(N, 32);
    // A fragments for every row block the product kernel reads: int8 128-row
    // tiles of four 32-row blocks (4 per operand block); FP64 64-row tiles of
    // four 16-row blocks (2 per operand block)
    a.nab = fp64 ? (int32_t)(ceil_div(w.m, 64) * 2) : (int32_t)ceil_div(w.m, 128);
    const int64_t ncb = ceil_div(w.m > 0 ? w.m : 1, 256);
    hipLaunchKernelGGL(leaf_operands_kernel, dim3((unsigned)(a.nyb + a.nab + ncb)), dim3(256), 0,
                       s, a);
    return hipGetLastError();
}

}  // namespace linac
