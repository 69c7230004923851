// Internal interfaces between the C-ABI front end (api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "field.h"
#include "../../include/linac.h"

namespace linac {

// Sentinel of a per-column pivot slot: no pivot found (yet).
static constexpr unsigned long long kNoPivot = ~0ull;

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
__host__ __device__ inline int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }

// Carve regions out of a caller-owned workspace, each starting at a 256-byte
// aligned ADDRESS (64-bit atomics and 128-bit accesses need their natural
// alignment, and a region may start at an arbitrary offset of the caller's
// buffer).  With base == NULL it only measures, aligning offsets; a real carve
// then uses at most 255 bytes more, which the 256 bytes every workspace query
// adds at the end cover.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T>
    T* take(int64_t count) {
        if (base) {
            const uintptr_t at = (uintptr_t)(base + off);
            off += (size_t)(((at + 255) & ~(uintptr_t)255) - at);
        } else {
            off = (size_t)round_up((int64_t)off, 256);
        }
        T* p = base ? (T*)(base + off) : nullptr;
        off += (size_t)count * sizeof(T);
        return p;
    }
};

// Working state of the plain Gauss-Jordan path for one system, all in the
// workspace.  W is the m x ld working copy of [A | B] (ld a multiple of 64, the
// padding columns zero).  Rows are never moved: the s-th pivot row is the
// physical row pivrow[s] (a virtual row swap), and the final gather writes the
// rows in pivot order.
struct PlainArgs {
    uint32_t* W;
    int64_t ld;
    int32_t m;
    int32_t ncols;    // n + k (columns that exist in W)
    int32_t nsearch;  // n: pivots are searched in columns [0, nsearch)
    int32_t coloff;   // global column of local column 0 (bookkeeping arrays are global)
    int32_t einject;  // >= 0: local column where the transform block E starts; the pivot
                      // row of local column j carries an implicit 1 at einject + j
    int32_t resolved; // 1: no deferred normalisation is left in W at the end
    uint32_t* fcol[2];           // column j as of step j (ping-pong); bit 31 marks pivot rows
    uint32_t* is_piv;            // 1 for rows already chosen as pivots
    unsigned long long* slots;   // per column: (pivot row << 32) | inverse of its head
    int32_t* pivrow;             // s-th pivot row
    int32_t* pivcol;             // s-th pivot column
    int32_t* colpiv;             // per column: s, or -1 for a free column
    int32_t* rowcol;             // per row: its pivot column, or -1
    int32_t* state;              // [0] = rank so far
    uint32_t* incons;            // per right-hand side: 1 once a residual is non-zero
    FieldConst F;
};

size_t plain_workspace(int64_t m, int64_t n, int64_t k);
void plain_carve(void* ws, int64_t m, int64_t n, int64_t k, PlainArgs& a);

// Optional per-launch timing through linac_opts (see include/linac.h).
struct LaunchTimer {
    const linac_opts* o;
    hipStream_t s;
    int32_t used = 0;
    LaunchTimer(const linac_opts* opts, hipStream_t st) : o(opts), s(st) {}
    bool on() const { return o && o->launch_events && o->launch_cap > 0 && used < o->launch_cap; }
    hipStream_t cur = nullptr;  // the stream of the launch being bracketed
    void before(int kind, hipStream_t on_stream = nullptr) {
        if (!on()) return;
        cur = on_stream ? on_stream : s;
        (void)hipEventRecord(o->launch_events[2 * used], cur);
        if (o->launch_kinds) o->launch_kinds[used] = kind;
    }
    void after() {
        if (!on()) return;
        (void)hipEventRecord(o->launch_events[2 * used + 1], cur);
        ++used;
        if (o->launch_used) *o->launch_used = used;
    }
};

// A second stream per device (created on first use, default priority) for work
// that may overlap the caller's stream within one call; the call joins it back
// to the caller's stream before returning.
hipError_t side_stream(hipStream_t* out);

// One Gauss-Jordan step for local pivot column j over local columns [.., ncols_eff).
hipError_t launch_gj_step(const PlainArgs& a, int32_t j, int32_t ncols_eff, hipStream_t s);

// Launch sequences (stream-ordered, no host synchronisation).
hipError_t plain_prepare(const PlainArgs& a, const uint32_t* A, int64_t lda, const uint32_t* B,
                         int64_t ldb, int32_t n, int32_t k, hipStream_t s);
hipError_t plain_eliminate(const PlainArgs& a, const linac_opts* opts, hipStream_t s);
hipError_t plain_finish_solve(const PlainArgs& a, int32_t n, int32_t k, uint32_t* X, int64_t ldx,
                              int32_t* rank, int32_t* pivots, uint8_t* consistent, hipStream_t s);
hipError_t plain_finish_rref(const PlainArgs& a, uint32_t* A, int64_t lda, int32_t* rank,
                             int32_t* pivots, hipStream_t s);

// Leaf pivot selection and leaf operands (leaf.hip).  The selection's result
// for the current leaf: t pivots, their candidate-list positions, row ids and
// leaf-local columns (ascending), and P^-1 for P = the pivot rows' values at
// the pivot columns (row-major, stride 32).
struct LeafOut {
    int32_t t;
    int32_t yready;  // 1: the selection also built Y = P^-1 R as int8 B fragments
    int32_t pad[62];
    int32_t pos[32];
    int32_t row[32];
    int32_t col[32];
    uint32_t pinv[32 * 32];
};

// Candidate lists (rows that are not pivots yet, ascending; ping-pong by leaf
// parity), their lengths, the selection tree's arrival counters (one set per
// parity), node results and the leaf results (one per parity, so that a leaf's
// product can still read its result while the next leaf's first selection
// publishes).  chunk: the next leaf's first kChunk candidates and, at [32], the
// length of its candidate list, for a first selection that runs before the
// compacted list exists.
struct LeafState {
    int32_t* cand[2];
    int32_t* count;  // count[parity]
    int32_t* cnt[2];
    int32_t* res;
    LeafOut* out[2];
    int32_t* chunk;
    uint32_t* rsave;  // the pivot rows over the columns the leaf updates, as selected
    int64_t ldr;
    int32_t nodes;
    int32_t gmax;
};

// The next leaf's candidate list: entry i of the current one (E entries) moves
// down by the number of this leaf's pivot positions below it, unless it is one
// of them (order kept).
__device__ __forceinline__ void leaf_compact_entry(const LeafOut* out, int32_t t,
                                                   const int32_t* cand, int32_t* cand_next,
                                                   int32_t E, int64_t i) {
    if (i >= E) return;
    int pos[32];  // all loads first (the array always has 32 entries)
#pragma unroll
    for (int k = 0; k < 32; ++k) pos[k] = out->pos[k];
    const int32_t row = cand[i];
    int shift = 0;
    bool gone = false;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const bool in = k < t;
        shift += in && pos[k] < i;
        gone |= in && pos[k] == i;
    }
    if (!gone) cand_next[i - shift] = row;
}

// The first 32 entries of the next candidate list: the first entries of
// `cand` (E entries) that are not this leaf's pivot positions.  At most t <= 32
// of the first 64 entries are pivot positions, so one wave looking at those 64
// finds them all.  Called by a whole wave (lane = its lane); lane i keeps entry
// i when it survives, at `rank` in the new list.  Returns min(32, E - t).
__device__ __forceinline__ int next_chunk_entry(const LeafOut* out, int32_t t, const int32_t* cand,
                                                int32_t E, int lane, int32_t* row, int* rank) {
    int pos[32];  // all loads first (the array always has 32 entries)
#pragma unroll
    for (int k = 0; k < 32; ++k) pos[k] = out->pos[k];
    bool gone = false;
#pragma unroll
    for (int k = 0; k < 32; ++k) gone |= k < t && pos[k] == lane;
    const bool keep = lane < E && !gone;
    const unsigned long long b = __ballot(keep);
    *rank = keep ? (int)__popcll(b & ((1ull << lane) - 1ull)) : 64;
    *row = keep ? cand[lane] : -1;
    const int n = (int)__popcll(b);
    return n < 32 ? n : 32;
}

// The int8 leaf product's operands and outputs: PR columns [l0, l0 + N) (ldpr apart),
// the leaf's result `out`, the saved pivot rows, c32 = 2^32 mod p, the
// candidate lists of this leaf and the next one, the Y fragments, the panel
// start for forward elimination (0: Gauss-Jordan) and the chunk buffer.
struct LeafProdArgs {
    PlainArgs w;
    uint32_t* PR;
    int64_t ldpr;
    int32_t l0, wl, wj, gcol0;
    int64_t N;
    const LeafOut* out;
    const uint32_t* rsave;
    int64_t ldr;
    double c32;
    const int32_t* cand;
    int32_t* cand_next;
    const int32_t* count;
    int32_t* count_next;
    const int8_t* yfrag;
    int32_t skip_below;
    int32_t* chunk;
    // Y's source: 0 = yfrag when the selection built it (out->yready), else
    // every workgroup forms its own slices from the saved pivot rows; 1 (the
    // chunk launch of a pipelined leaf, one workgroup per column group) = as 0,
    // and slices formed here are also stored in ystore (= yfrag); 2 (the
    // launch of the other rows after that chunk launch) = yfrag, built by the
    // selection or stored by the chunk launch
    int32_t ymode;
    int8_t* ystore;
};

int32_t leaf_nodes(int64_t m);
void leaf_carve(Carver& c, int64_t m, int64_t ldr, LeafState* ls);
hipError_t leaf_init(const LeafState& ls, int32_t m, hipStream_t s);
// The selection of a leaf over PR columns [l0, l0 + wl).  ncopy = the number
// of PR columns the leaf updates (from l0), wj = the panel width.  With yfrag
// non-NULL it also builds Y = P^-1 R over those columns as int8 B fragments
// (one k-block, 4 digit planes per 32 columns) when the first chunk of
// candidates already decides the leaf, setting out->yready.  With save_rows,
// every result that leaves Y to the product (out->yready = 0) also saves the
// pivot rows over those columns in ls.rsave (row s = pivot s).
// stages: kSelectFirst (the first chunk alone), kSelectRest (the tree, or the
// build of Y when the first chunk decided), or both.  from_chunk: the first
// stage reads its candidates from ls.chunk (written by the previous leaf's
// chunk product) instead of the compacted list.
constexpr int kSelectFirst = 1, kSelectRest = 2;
hipError_t leaf_select(const PlainArgs& w, const LeafState& ls, const uint32_t* PR, int64_t ldpr,
                       int32_t l0, int32_t wl, int32_t wj, int32_t gcol0, int32_t parity,
                       int64_t ncopy, int8_t* yfrag, bool save_rows, hipStream_t s,
                       int stages = kSelectFirst | kSelectRest, bool from_chunk = false);
// The larger half of leaf l's int8 product (every row but the next leaf's first
// chunk; pa as for the product kernel) in one launch with the first selection
// of leaf l + 1 (columns [l0, l0 + wl) of PR, parity its leaf parity, reading
// its candidates from ls.chunk).  Needs the chunk half of leaf l's product
// done first (same stream).
hipError_t leaf_fused(const PlainArgs& w, const LeafState& ls, const uint32_t* PR, int64_t ldpr,
                      int32_t l0, int32_t wl, int32_t wj, int32_t gcol0, int32_t parity,
                      int64_t ncopy, int8_t* yfrag, const LeafProdArgs& pa, int32_t leaf_blocks,
                      hipStream_t s);
// Operands of the FP64 leaf product over PR columns [l0, l0 + N): the B operand
// Y = P^-1 R and the A operand (multipliers) in the layout of the FP64 product
// kernel (16 x 16 blocks with 8 k-blocks of 4); also compacts the candidate
// list.
hipError_t leaf_operands(const PlainArgs& w, const LeafState& ls, const uint32_t* PR, int64_t ldpr,
                         int32_t l0, int32_t wl, int32_t wj, int32_t gcol0, int64_t N,
                         int32_t parity, bool fp64, void* Afrag, void* Bfrag, hipStream_t s);

// Blocked path (blocked.hip): workspace = the plain layout followed by the panel
// buffer and the MFMA operand fragments.  `a` carries the field in and the
// carved bookkeeping out (for the shared extraction kernels).
size_t blocked_workspace(int64_t m, int64_t n, int64_t k, int32_t panel);
// forward = true (solves with right-hand sides, int8 path): forward elimination
// then back-substitution into the pivot rows' right-hand sides, instead of
// Gauss-Jordan (the reduced matrix is then not an RREF; only X is read).
// leaf_blocks: 16-column blocks per workgroup of the int8 leaf product (2, 3,
// 6 or 9; a tuned shape, results identical).  leaf_pipeline (int8 path): each
// leaf's product in two launches, the larger half beside the next leaf's first
// selection (results identical).
hipError_t blocked_eliminate(void* ws, int64_t m, int64_t n, int64_t k, int32_t panel, bool fp64,
                             bool lookahead, bool forward, int32_t leaf_blocks, bool leaf_pipeline,
                             PlainArgs& a, const linac_opts* opts, hipStream_t s);

// Batched path (batched.hip): workspace = [queue counter | descriptors | one
// working region per system].
bool batched_fits(int64_t m, int64_t n, int64_t k);
size_t batched_desc_bytes();
size_t batched_workspace(const linac_system* sys, int32_t count);
void batched_describe(const linac_system* sys, int32_t count, void* ws, void* host_desc,
                      int32_t* order);
void* batched_desc_ptr(void* ws);
// Rows of the multiplier array in dynamic LDS: the largest m, rounded up to 64.
int32_t batched_mult_rows(const linac_system* sys, int32_t count);
hipError_t batched_launch(void* ws, int32_t count, int32_t grid, int32_t mult_rows, hipStream_t s);

// Around the elimination (apps.hip): the system construction from monomials,
// the canonical null-space basis of an RREF and the pivot columns of A.
hipError_t launch_load_matrix(const uint32_t* bases, int64_t nrows, int64_t nb, int64_t ldbases,
                              const int32_t* lind, int64_t ncols, int64_t d, int64_t ldl,
                              const FieldConst& F, uint32_t* A, int64_t lda, hipStream_t s);
hipError_t launch_nullspace(const uint32_t* R, int64_t m, int64_t n, int64_t ldr, const int32_t* rank,
                            const int32_t* pivots, uint32_t p, uint32_t* K, int64_t kcols, int64_t ldk,
                            int32_t* free_cols, hipStream_t s);
hipError_t launch_column_basis(const uint32_t* A, int64_t m, int64_t n, int64_t lda, const int32_t* rank,
                               const int32_t* pivots, uint32_t* C, int64_t ccols, int64_t ldc,
                               hipStream_t s);

// Column-step engine (colstep.hip): Gauss-Jordan for 64-bit primes and the
// LUP factorisation, one search and one update launch per pivot column.
size_t colstep_workspace(int64_t m, int64_t n, int64_t k, bool wide);
template <typename W>
hipError_t colstep_range(const W* M, int64_t rows, int64_t cols, int64_t ld, W p, uint32_t* flag,
                         hipStream_t s);
template <typename W>
hipError_t colstep_rref(W* A, int64_t m, int64_t n, int64_t lda, W p, int32_t* rank, int32_t* pivots,
                        void* ws, hipStream_t s);
template <typename W>
hipError_t colstep_solve(const W* A, int64_t m, int64_t n, int64_t lda, const W* B, int64_t k,
                         int64_t ldb, W p, W* X, int64_t ldx, int32_t* rank, int32_t* pivots,
                         uint8_t* consistent, void* ws, hipStream_t s);
template <typename W>
hipError_t colstep_lup(W* A, int64_t m, int64_t n, int64_t lda, W p, int32_t* perm, int32_t* rank,
                       int32_t* pivots, void* ws, hipStream_t s);

// linac_solve split in two (api.hip): the host checks (on success *path and
// *need, the workspace bytes, are set), and the launches on a workspace of at
// least that size.  allow_overlap = false keeps the blocked int8 path on `s`
// (no side stream, no events created).  hip_status records a HIP error for
// linac_last_hip_error and maps it to a status.
linac_status solve_check(const uint32_t* A, int64_t m, int64_t n, int64_t lda, const uint32_t* B,
                         int64_t k, int64_t ldb, uint32_t p, const uint32_t* X, int64_t ldx,
                         const int32_t* rank, const int32_t* pivots, const uint8_t* consistent,
                         const linac_opts* opts, int* path, size_t* need);
linac_status solve_launch(const uint32_t* A, int64_t m, int64_t n, int64_t lda, const uint32_t* B,
                          int64_t k, int64_t ldb, uint32_t p, uint32_t* X, int64_t ldx,
                          int32_t* rank, int32_t* pivots, uint8_t* consistent, void* ws, int path,
                          const linac_opts* opts, hipStream_t s, bool allow_overlap,
                          const char* name);
linac_status hip_status(hipError_t e);

// Range check of residues: sets *flag to 1 when an entry is >= p.
hipError_t launch_range_check(const uint32_t* M, int64_t rows, int64_t cols, int64_t ld, uint32_t p,
                              uint32_t* flag, hipStream_t s);

}  // namespace linac
