// Persistent lock-step decoding engine for dense transition models (gfx950).
//
// One cooperative launch runs every step of every decoding task of a batch:
// vanilla passes (Sec. III-A), FLASH root passes and FLASH subtasks
// (Alg. 1 / Alg. 2).  A "row" is one task in flight; at every global step each
// row advances one time step.  Compute blocks execute the rows of the current
// step; the last block is the scheduler, which meanwhile builds the next
// step's row lists (task creation, slot reuse) and then acts as the master of
// the step barrier.
//
// MI355X layout: the 256 CUs sit in 8 XCDs, each with its own L2.  Row
// buffer slot s belongs to XCD s % 8 and only blocks running on that XCD
// (read from the XCC_ID hardware register) compute or read its rows, so a
// row's state moves between steps through one L2: publishing it needs only
// "my stores are done" and reading it only an L1 invalidate.  The small
// state shared across XCDs (row lists, counts, path entries, anchors, status)
// is read and written with coherent (sc1) accesses.  No L2 write-back or
// invalidate is issued per step (except with wide rows, whose row data does
// cross XCDs), and log A stays resident in every L2.
//
// Dense step of a row at time t (Sec. III-A recurrence, log domain):
//     c(j)   = max_i delta_{t-1}(i) + log A(i, j)     (one float32 add per candidate)
//     psi(j) = the lowest i attaining c(j)
//     delta_t(j) = c(j) + log B_t(j)
// Tile = 64 rows (one per lane) x 16 destination columns; the 4 waves split
// the predecessors i.  log A(i, j0..j0+15) is wave-uniform and arrives through
// scalar loads as SGPR operands, so each candidate costs one v_add_f32 and
// half a v_max3_f32.  The arg max is tracked per group of 16 predecessors
// (strictly greater group maximum wins, so the earliest group keeps ties) and
// refined once per output inside the winning group, recomputing the exact
// candidates; the stored value is that winning candidate.
#include "fv_internal.h"

namespace fv {

static_assert(sizeof(Row) == 64, "Row is moved as 8 coherent 64-bit words");

// The engine reads its arguments from a copy in the workspace through the
// constant address space: field loads are scalar loads in every function.
typedef __attribute__((address_space(4))) const EngineArgs cargs_t;
// the argument block is the same for every lane: keep its address scalar
__device__ __forceinline__ cargs_t& uniform_args(cargs_t& a) {
    const uint64_t v = reinterpret_cast<uint64_t>(&a);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return *reinterpret_cast<cargs_t*>(((uint64_t)hi << 32) | lo);
}

// The engine runs one 1024-thread block per CU: 16 waves = 4 tile groups of
// 4 waves (one wave per SIMD each), which keeps 4 waves per SIMD for latency
// hiding while the step barrier has one participant per CU.
constexpr int kEngBlock = 1024;
constexpr int kEngWaves = kEngBlock / 64;

// ---------------------------------------------------------------- access helpers
template <typename T>
__device__ __forceinline__ T ld_c(const T* p) {  // coherent across XCDs
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_c(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// st_c on a pointer known to address global memory: a global (not flat)
// store, so waiting for LDS results does not also wait for it
template <typename T>
__device__ __forceinline__ void st_cg(T* p, T v) {
    typedef __attribute__((address_space(1))) T gT;
    __hip_atomic_store(reinterpret_cast<gT*>(reinterpret_cast<uint64_t>(p)), v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_cf(const float* p) {
    return __uint_as_float(ld_c(reinterpret_cast<const uint32_t*>(p)));
}
__device__ __forceinline__ void st_cf(float* p, float v) {
    st_c(reinterpret_cast<uint32_t*>(p), __float_as_uint(v));
}
__device__ __forceinline__ Row ld_row(const Row* p) {
    const uint64_t* q = reinterpret_cast<const uint64_t*>(p);
    uint64_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = ld_c(q + k);
    Row r;
    __builtin_memcpy(&r, w, sizeof r);
    return r;
}
__device__ __forceinline__ void st_row(Row* p, const Row& r) {
    uint64_t w[8];
    __builtin_memcpy(w, &r, sizeof r);
    uint64_t* q = reinterpret_cast<uint64_t*>(p);
#pragma unroll
    for (int k = 0; k < 8; ++k) st_c(q + k, w[k]);
}
__device__ __forceinline__ int32_t clampi(int32_t v, int32_t hi) { return v < 0 ? 0 : (v >= hi ? hi - 1 : v); }
// A value known to be the same in every lane, moved to a scalar register (so
// that the addresses and loops it controls are scalar too).
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Explicit address spaces for the hot loops, which live in non-inlined
// functions (where pointers are generic): log A is never written during a
// decode, so a wave-uniform pointer to it may be read through the constant
// address space (scalar loads); per-lane data goes through the global one.
typedef __attribute__((address_space(4))) const float cfloat_t;
typedef __attribute__((address_space(1))) const float gfloat_t;
__device__ __forceinline__ cfloat_t* uniform_const(const float* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<cfloat_t*>(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ gfloat_t* as_global(const float* p) {
    return reinterpret_cast<gfloat_t*>(reinterpret_cast<uint64_t>(p));
}
// coherent (agent-scope) load through the global address space
__device__ __forceinline__ float ld_cg(const float* p) {
    typedef __attribute__((address_space(1))) const uint32_t gu32_t;
    gu32_t* q = reinterpret_cast<gu32_t*>(reinterpret_cast<uint64_t>(p));
    return __uint_as_float(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Final arg-max keys are combined by tiles and read by the finalize step
// with coherent loads, so the max is performed at the memory side (sc1).
__device__ __forceinline__ void key_max(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ uint32_t my_xcd() {
    return __builtin_amdgcn_s_getreg((15 << 11) | (0 << 6) | 20) & (kXcd - 1);  // HW_REG_XCC_ID
}

__device__ __forceinline__ unsigned long long order_key(float v, int32_t j) {
    if (v == 0.0f) v = 0.0f;  // -0 and +0 compare equal; the lower index must win
    uint32_t b = __float_as_uint(v);
    uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((unsigned long long)o << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
}

// Emission score of the Gaussian point model: state j's point xy[j] against
// observation t's point obs[t], in float64 with each operation rounded once
// (no contraction into fused multiply-adds), then rounded to float32:
// (float)(c2 * ((x - u)^2 + (y - v)^2) - c0).
__device__ __forceinline__ float gauss2d_score(const double* __restrict__ xy, const double* __restrict__ obs,
                                               double c2, double c0, int32_t t, int32_t j) {
#pragma clang fp contract(off)
    const double dx = xy[2 * (int64_t)j] - obs[2 * (int64_t)t];
    const double dy = xy[2 * (int64_t)j + 1] - obs[2 * (int64_t)t + 1];
    const double sx = dx * dx;
    const double sy = dy * dy;
    const double d2 = sx + sy;
    const double e = c2 * d2;
    return (float)(e - c0);
}

// log B_t(j) of a sequence whose emission data starts at lb: its table's
// entry lb[t * ld + j], or the Gaussian point model's score with lb
// addressing the observations (float64 [T][2]).  emit_kind is uniform.
__device__ __forceinline__ float emission_of(int32_t kind, const double* xy, double c2, double c0,
                                             const float* __restrict__ lb, int64_t ld, int32_t t, int32_t j) {
    if (kind == FV_EMIT_TABLE) return as_global(lb)[(int64_t)t * ld + j];
    return gauss2d_score(xy, reinterpret_cast<const double*>(lb), c2, c0, t, j);
}
__device__ __forceinline__ float emission(cargs_t& a, const float* lb, int64_t ld, int32_t t, int32_t j) {
    return emission_of(a.emit_kind, a.emit_xy, a.emit_c2, a.emit_c0, lb, ld, t, j);
}

__device__ __forceinline__ float* slot_delta(cargs_t& a, int32_t slot, int32_t parity) {
    return a.slot_base + (int64_t)slot * a.slot_floats + (int64_t)parity * a.Kp;
}
__device__ __forceinline__ int32_t* slot_anc(cargs_t& a, int32_t slot, int32_t parity) {
    return reinterpret_cast<int32_t*>(a.slot_base + (int64_t)slot * a.slot_floats +
                                      (int64_t)(2 + parity) * a.Kp);
}
__device__ __forceinline__ float* slot_snap(cargs_t& a, int32_t slot) {
    return a.slot_base + (int64_t)slot * a.slot_floats + (int64_t)4 * a.Kp;
}
__device__ __forceinline__ uint16_t* slot_leaf(cargs_t& a, int32_t slot) {
    return reinterpret_cast<uint16_t*>(a.slot_base + (int64_t)slot * a.slot_floats + a.leaf_off);
}
// A dense subtask short enough to be a leaf (never an exact re-decode of a
// beam subtask: those keep the beam procedure's structure).
__device__ __forceinline__ bool is_leaf(cargs_t& a, int32_t kind, int32_t m, int32_t n) {
    return kind == KIND_SUB && a.leaf_len > 0 && n - m + 1 <= a.leaf_len;
}
// Division copies of a w-way subtask in its slot: delta at e_k (k < kWSplit - 1),
// then the chain links at e_k (k >= 1: the state at e_{k-1} on the best path
// into each state at e_k).
__device__ __forceinline__ float* slot_div_d(cargs_t& a, int32_t slot, int32_t k) {
    return a.slot_base + (int64_t)slot * a.slot_floats + a.div_off + (int64_t)k * a.Kp;
}
__device__ __forceinline__ int32_t* slot_div_l(cargs_t& a, int32_t slot, int32_t k) {
    return reinterpret_cast<int32_t*>(a.slot_base + (int64_t)slot * a.slot_floats + a.div_off +
                                      (int64_t)(kWSplit - 2 + k) * a.Kp);
}
__device__ __forceinline__ float* root_dsnap(cargs_t& a, int64_t root_off, int32_t d) {
    return a.root_copy + (root_off + d) * (int64_t)a.Kp;
}
__device__ __forceinline__ int32_t* root_link(cargs_t& a, int64_t root_off, int32_t pp, int32_t d) {
    return reinterpret_cast<int32_t*>(a.root_copy + (root_off + (pp - 1) + d) * (int64_t)a.Kp);
}
__device__ __forceinline__ Row* list_full(cargs_t& a, int parity, int x) {
    return a.rows_full + ((int64_t)parity * kXcd + x) * a.pool;
}
__device__ __forceinline__ Row* list_light(cargs_t& a, int parity, int x) {
    return a.rows_light + ((int64_t)parity * kXcd + x) * a.pool;
}
__device__ __forceinline__ Row* list_beam(cargs_t& a, int parity, int x) {
    return a.rows_beam + ((int64_t)parity * kXcd + x) * a.pool;
}

// ---------------------------------------------------------------- LDS
// The engine's shared memory, at file scope so that every function of the
// engine addresses it as LDS (a reference passed to a non-inlined function
// would become a generic pointer).
struct TileLds {
    float m[kEngWaves][kTileCols][kTileRows];
    int32_t g[kEngWaves][kTileCols][kTileRows];
    uint64_t stash[4][kTileRows][4];   // per tile group: row words 0, 3, 4, 5 of each lane's row
    uint32_t gsync[4];                  // per tile group: barrier arrivals
    int32_t gitem[4];                   // per tile group: the work item it claimed
};

constexpr int32_t kWideRows = 16;
constexpr int32_t kWideCols = 64;
constexpr int32_t kWideStage = 64;   // predecessors staged per LDS refill (4 groups)
constexpr int32_t kLocalColRows = 160;  // an XCD with at most this many dense rows uses column items

struct WideLds {
    float area[kEngWaves][2 * kWideRows * kWideCols];   // per wave: staged scores, later (max, group)
    Row rows[kWideRows];
};

// Two-column items (Kp <= kColMaxKp): 8 rows x 128 destinations, the rows'
// previous scores staged whole, partial results merged through 64-bit keys.
constexpr int32_t kColRows = 8;
constexpr int32_t kColCols = 128;
constexpr int32_t kColItemFixed = 2;     // an item's fixed cost, in rows of work
struct ColLds {
    float d[kColRows * kColMaxKp];
    unsigned long long key[kColRows * kColCols];
    Row rows[kColRows];
};
static_assert(kColRows * kColCols == kEngBlock, "one refine output per thread");

constexpr int32_t kBeamPartMax = 4096;   // destinations per part
constexpr int32_t kBeamCandMax = 8192;   // W * B: candidates of a rebuild

struct BeamLds {
    int32_t cs[kBeamCandMax];   // candidates of a rebuild: states, scores, anchors
    float cv[kBeamCandMax];
    int32_t ca[kBeamCandMax];
    float sc[kBeamPartMax];     // scores and anchors of a part's destinations
    int32_t an[kBeamPartMax];
    int32_t bs[kBeamMaxB];      // the rebuilt beam, in state order
    float bv[kBeamMaxB];
    int32_t ba[kBeamMaxB];
    uint32_t hist[256];
    int32_t wsum[kEngWaves];
    unsigned long long wkey[kEngWaves];
    int32_t pofs[33];
    int32_t misc[8];
};

// A sparse beam step (push over the beam states' out-edges) works in the
// candidate area of BeamLds; the rebuilt beam (bs/bv/ba) stays in place.
struct SpBeamLds {
    uint64_t key[kSpCandMax];    // (destination << 32) | candidate position, sorted
    float cval[kSpCandMax];      // candidate score by position
    int32_t ds[kSpCandMax];      // distinct destinations (state order), their
    float dv[kSpCandMax];        // scores and anchors
    int32_t da[kSpCandMax];
    int32_t offs[kBeamMaxB + 1]; // first candidate position of each beam entry
    int32_t estart[kBeamMaxB];   // first out-edge of each beam entry
};

// Grouped beam rows: with a dense model of Kp <= kQK, B <= kQB and one part
// per step, each 256-thread group (4 waves) of a block runs its own beam
// row, so a block has four beam steps in flight (the step is bound by
// latency: barriers, selection passes, log A row loads).
constexpr int kQThreads = 256;
constexpr int kQWaves = kQThreads / 64;
constexpr int kQGroups = kEngBlock / kQThreads;
constexpr int32_t kQK = 2048;
constexpr int32_t kQB = 256;

struct QBeamLds {                 // one group's share
    int32_t cs[kQB];              // candidates of a rebuild (one part: at most B)
    float cv[kQB];
    int32_t ca[kQB];
    float sc[kQK];                // scores and anchors of every destination
    int32_t an[kQK];
    int32_t bs[kQB];              // the rebuilt beam, in state order
    float bv[kQB];
    int32_t ba[kQB];
    uint32_t hist[256];
    int32_t wsum[kQWaves];
    unsigned long long wkey[kQWaves];
    int32_t misc[8];
};

struct QuarterLds {
    QBeamLds g[kQGroups];
    uint32_t gsync[kQGroups];     // per group: barrier arrivals
    int32_t gitem[kQGroups];      // per group: the row it claimed
};

// Column slabs (dense local rows, K = Kp = 512 or 1024): a chunk of rows'
// previous scores staged whole, one 64-bit partial key per output.
constexpr int32_t kSlabMaxKp = 1024;
constexpr int32_t kSlabChunkMax = kEngBlock / 64;   // rows of a chunk (16 at Kp = 1024, 8 at 512)
struct SlabLds {
    float d[kSlabChunkMax * kSlabMaxKp];
    unsigned long long key[kEngBlock];
    Row rows[kSlabChunkMax];
    int32_t upass[kSlabChunkMax];   // column pass of each unit of the chunk
};

union EngineLds {
    TileLds tile;
    SlabLds slab;
    WideLds wide;
    BeamLds beam;
    SpBeamLds spbeam;
    QuarterLds qbeam;
    ColLds col;
};
static_assert(sizeof(SpBeamLds) <= offsetof(BeamLds, bs), "sparse beam scratch overlaps the beam");

constexpr int kSchedGroup = kEngBlock / kXcd;
constexpr int kSchedGroupWaves = kSchedGroup / 64;

struct SchedLds {
    int32_t q_head, q_tail, max_rows;
    int32_t total_next;        // rows of the step the last admission prepared
    int32_t q_spawn;           // next free queue position while a step's rows spawn tasks
    int32_t out_cnt[kXcd][4];  // per XCD: next rows written (full, light, beam), slots freed
    int32_t n_free[kXcd];
    int32_t nblk[kXcd];        // compute blocks on each XCD
    int32_t admit[kXcd];
    int32_t n_next[kXcd][3];   // rows written for the next step: full, light, beam
    int32_t wave_sums[kXcd][kSchedGroupWaves][5];
};

static __shared__ __align__(16) EngineLds g_lds;
static __shared__ SchedLds g_sched;

// ---------------------------------------------------------------- row flags
// Row of `base`'s task at time t as a dense step (leaf: a leaf subtask).
__device__ Row make_dense_row(const Row& base, int32_t t, bool leaf, int32_t wsplit = 0) {
    Row r = base;
    const int32_t kind = r.kind, m = r.m, n = r.n, T = r.T, pp = r.pp;
    r.t = t;
    int32_t f = 0, aux = 0;
    if (kind == KIND_VANILLA) {
        f = F_NEED_ARG | F_PSI_TABLE;
        if (t == T - 1) f |= F_FINAL;
    } else if (kind == KIND_ROOT) {
        if (pp >= 2) {
            int64_t e0 = seg_end(T, pp, 0);
            if (t > e0) f |= F_NEED_ARG;
            if (div_index(T, pp, t - 1) >= 0) f |= F_ANC_FIRST;
            else if (t > e0 + 1) f |= F_ANC_CHAIN;
            int32_t d = div_index(T, pp, t);
            if (d >= 0) { f |= F_SNAP_ROOT; aux = d; }
        }
        if (t == T - 1) f |= F_FINAL;
    } else if (leaf) {
        f = F_NEED_ARG | F_LEAF_TABLE;
        aux = t - m;
    } else if (kind == KIND_SUB && wsplit > 2) {
        // the root's division rules over the subtask's own span [m, n]
        const int32_t L = n - m + 1, wp = sub_parts(m, n, wsplit);
        const int64_t e0 = m + seg_end(L, wp, 0);
        if (t > e0) f |= F_NEED_ARG;
        if (div_index(L, wp, t - 1 - m) >= 0) f |= F_ANC_FIRST;
        else if (t > e0 + 1) f |= F_ANC_CHAIN;
        const int32_t d = div_index(L, wp, t - m);
        if (d >= 0) { f |= F_SNAP_DIV; aux = d; }
    } else {
        int32_t tmid = (m + n) >> 1;
        if (t > tmid) f |= F_NEED_ARG;
        if (t == tmid + 1) f |= F_ANC_FIRST;
        else if (t > tmid + 1) f |= F_ANC_CHAIN;
        if (t == tmid) f |= F_SNAP_SUB;
    }
    r.flags = f;
    r.aux = aux;
    return r;
}

// Row of `base`'s task at time t as a light operation (leaf: a leaf subtask).
__device__ Row make_light_row(const Row& base, int32_t t, int32_t op, bool leaf = false, int32_t wsplit = 0) {
    Row r = base;
    const int32_t kind = r.kind, m = r.m, n = r.n, T = r.T, pp = r.pp;
    r.t = t;
    r.aux = op;
    int32_t f = 0;
    if (op == L_INIT) {
        if (kind == KIND_SUB && !leaf && wsplit > 2) {
            if (seg_end(n - m + 1, sub_parts(m, n, wsplit), 0) == 0) f |= F_SNAP_DIV;   // division 0 at m
        } else if (is_dense_sub(kind) && !leaf && ((m + n) >> 1) == m) f |= F_SNAP_SUB;
        if (kind == KIND_ROOT && pp >= 2 && seg_end(T, pp, 0) == 0) f |= F_SNAP_ROOT;
        if ((kind == KIND_VANILLA || kind == KIND_ROOT) && T == 1) f |= F_FINAL;
    }
    r.flags = f;
    return r;
}

// First row (the start step) of a task, from the per-sequence table.
__device__ Row row_from_task(cargs_t& a, const Task& tk, int32_t slot) {
    const SeqInfo& sq = a.seqs[tk.seq];
    Row b;
    b.seq = tk.seq; b.kind = tk.kind; b.m = tk.m; b.n = tk.n; b.t = tk.m; b.slot = slot;
    b.flags = 0; b.aux = 0;
    b.T = sq.T; b.pp = sq.pp;
    b.off = tk.kind == KIND_VANILLA ? sq.psi_off : sq.root_off;
    b.log_b = sq.log_b; b.ld = sq.ld;
    if (is_beam(tk.kind)) {
        b.aux = B_INIT;
        return b;
    }
    Row r = make_light_row(b, tk.m, L_INIT, is_leaf(a, tk.kind, tk.m, tk.n), a.wsplit);
    if (a.sparse) {   // a sparse start step is a row of the full list (see sparse_unit)
        r.flags |= F_START;
        r.aux = 0;    // division 0 for F_SNAP_ROOT
    }
    return r;
}

// List a task's first row goes to: 0 full (sparse start), 1 light, 2 beam.
__device__ __forceinline__ int32_t start_list(cargs_t& a, int32_t kind) {
    return is_beam(kind) ? 2 : (a.sparse ? 0 : 1);
}

// Row of a beam task at time t doing operation op.
__device__ Row make_beam_row(const Row& base, int32_t t, int32_t op) {
    Row r = base;
    r.t = t;
    r.aux = op;
    r.flags = 0;
    return r;
}

// ---------------------------------------------------------------- dense tile
// Partial (max, group) of 16 columns over predecessors [s0, s1) for the
// lane's row; drow = the row's delta_{t-1}, Ap = padded row-major log A.
__device__ __forceinline__ void tile_partial(cfloat_t* __restrict__ Ap, int32_t Kp, int32_t j0,
                                             gfloat_t* drow, int32_t s0, int32_t s1,
                                             float (&m)[kTileCols], int32_t (&g)[kTileCols]) {
#pragma unroll
    for (int c = 0; c < kTileCols; ++c) { m[c] = -INFINITY; g[c] = s0 / kGroup; }
    for (int32_t i0 = s0; i0 < s1; i0 += kGroup) {
        float gm[kTileCols];
#pragma unroll
        for (int c = 0; c < kTileCols; ++c) gm[c] = -INFINITY;
#pragma unroll
        for (int k = 0; k < kGroup; k += 4) {
            typedef float v4f_t __attribute__((ext_vector_type(4)));
            const v4f_t d = *reinterpret_cast<__attribute__((address_space(1))) const v4f_t*>(drow + i0 + k);
            cfloat_t* a0 = Ap + (int64_t)(i0 + k) * Kp + j0;
#pragma unroll
            for (int c = 0; c < kTileCols; ++c) {
                const float x0 = d.x + a0[c];
                const float x1 = d.y + a0[Kp + c];
                const float x2 = d.z + a0[2 * Kp + c];
                const float x3 = d.w + a0[3 * Kp + c];
                gm[c] = fmaxf(fmaxf(gm[c], x0), x1);
                gm[c] = fmaxf(fmaxf(gm[c], x2), x3);
            }
        }
        const int32_t gi = i0 / kGroup;
#pragma unroll
        for (int c = 0; c < kTileCols; ++c)
            if (gm[c] > m[c]) { m[c] = gm[c]; g[c] = gi; }
    }
}

// Partial results of the 16 waves of a block: [wave][column][row].

// Barrier of the nsplit waves of one tile group (an LDS arrival counter;
// the groups of a block run independently of each other).  Every wave of
// the group calls it the same number of times.
__device__ __forceinline__ void group_sync(uint32_t* ctr, int32_t nsplit) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & 63) == 0) {
        const uint32_t old = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint32_t target = old - old % (uint32_t)nsplit + (uint32_t)nsplit;
        uint32_t spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 26)) break;   // bounded: the group's waves always arrive
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One tile computed by a group of nsplit waves (4, 8 or 16), each wave
// taking a contiguous share of the predecessor groups; the waves of the
// group call this together (group barriers inside), other groups of the
// block run on independently.
//
// After the max-plus loop the partial maxima merge through LDS and each
// output's arg max is refined inside its winning group.  That epilogue is
// bound by memory latency, so its loads are issued together: the row's
// remaining fields come from an LDS copy made before the loop, the refine
// loads of two columns go out at once, and so do the anchor gathers.
__device__ __noinline__ void dense_tile(cargs_t& a_in, const float* __restrict__ Ap, const Row* rows,
                           int32_t nrows, int32_t tile, int32_t nsplit) {
    cargs_t& a = uniform_args(a_in);
    TileLds& lds = g_lds.tile;
    const bool active = true;
    const int32_t K = a.K, Kp = a.Kp;
    const int32_t ncb = Kp / kTileCols;
    const int32_t rg = tile / ncb;
    const int32_t j0 = (tile - rg * ncb) * kTileCols;
    const int32_t lane = threadIdx.x & 63;
    const int32_t bw = threadIdx.x >> 6;              // wave in block
    const int32_t wave = bw & (nsplit - 1);           // wave in tile group
    const int32_t wbase = bw - wave;                  // first wave of the group
    const int32_t grp = bw / nsplit;                  // tile group in block
    const int32_t cpw = kTileCols / nsplit;           // output columns per wave
    const int32_t ridx = rg * kTileRows + lane;
    const bool valid = active && ridx < nrows;
    const Row* rp = rows + (valid ? ridx : rg * kTileRows);
    // (t, slot), log_b and ld of the row; the group's first wave also copies
    // the fields the epilogue needs to LDS
    const uint64_t* rw = reinterpret_cast<const uint64_t*>(rp);
    const uint64_t w_ts = ld_c(rw + 2);
    const int32_t t0 = (int32_t)(uint32_t)w_ts, slot0 = clampi((int32_t)(w_ts >> 32), a.n_slots);
    const float* log_b = reinterpret_cast<const float*>(ld_c(rw + 6));
    const int64_t ld = (int64_t)ld_c(rw + 7);
    if (wave == 0) {
        lds.stash[grp][lane][0] = ld_c(rw + 0);
        lds.stash[grp][lane][1] = ld_c(rw + 3);
        lds.stash[grp][lane][2] = ld_c(rw + 4);
        lds.stash[grp][lane][3] = ld_c(rw + 5);
    }
    const float* drow = slot_delta(a, slot0, (t0 - 1) & 1);
    // emission scores of this thread's outputs, fetched before the max-plus loop
    const int32_t cq = wave * cpw;
    float bpre[4];
    {
        const float* bt = log_b + (int64_t)t0 * ld;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int32_t j = j0 + cq + cc;
            bpre[cc] = (valid && cc < cpw && j < K) ? bt[j] : 0.0f;
        }
    }

    // predecessor groups [g0, g1) of this wave
    const int32_t ng = Kp / kGroup;
    const int32_t g0 = __builtin_amdgcn_readfirstlane((wave * ng) / nsplit);
    const int32_t g1 = __builtin_amdgcn_readfirstlane(((wave + 1) * ng) / nsplit);
    {
        float m[kTileCols];
        int32_t g[kTileCols];
        tile_partial(uniform_const(Ap), __builtin_amdgcn_readfirstlane(Kp), __builtin_amdgcn_readfirstlane(j0),
                     as_global(drow), g0 * kGroup, active ? g1 * kGroup : g0 * kGroup, m, g);
#pragma unroll
        for (int c = 0; c < kTileCols; ++c) {
            lds.m[bw][c][lane] = m[c];
            lds.g[bw][c][lane] = g[c];
        }
    }
    group_sync(&lds.gsync[grp], nsplit);

    if (valid) {
        const uint64_t w0 = lds.stash[grp][lane][0], w3 = lds.stash[grp][lane][1];
        const uint64_t w4 = lds.stash[grp][lane][2], w5 = lds.stash[grp][lane][3];
        const int32_t seq = (int32_t)(uint32_t)w0;
        const int32_t f = (int32_t)(uint32_t)w3, aux = (int32_t)(w3 >> 32);
        const int32_t pp = (int32_t)(w4 >> 32);
        const int64_t off = (int64_t)w5;
        const int32_t t = t0, slot = slot0;
        float* dcur = slot_delta(a, slot, t & 1);
        int32_t* acur = nullptr;
        const int32_t* aprev = nullptr;
        if (a.has_anc) {
            acur = slot_anc(a, slot, t & 1);
            aprev = slot_anc(a, slot, (t - 1) & 1);
        }
        // merge the partial maxima of the group's waves (earliest group keeps ties)
        float mv[4];
        int32_t gi[4];
        bool live[4], need[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int32_t c = cq + cc;
            live[cc] = cc < cpw && j0 + c < K;
            mv[cc] = 0.0f;
            gi[cc] = 0;
            if (live[cc]) {
                float v = lds.m[wbase][c][lane];
                int32_t gg = lds.g[wbase][c][lane];
                for (int w = 1; w < nsplit; ++w) {
                    const float x = lds.m[wbase + w][c][lane];
                    if (x > v) { v = x; gg = lds.g[wbase + w][c][lane]; }
                }
                mv[cc] = v;
                gi[cc] = gg;
            }
            need[cc] = live[cc] && ((f & F_NEED_ARG) || mv[cc] == 0.0f);
        }
        // refine inside the winning group: the first candidate equal to the
        // maximum; its value is the one stored (signed zero)
        float val[4];
        int32_t psi[4];
#pragma unroll
        for (int cb = 0; cb < 4; cb += 2) {
            float av[2][kGroup], dv[2][kGroup];
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2) {
                const int cc = cb + c2;
                if (need[cc]) {
                    const int32_t src0 = gi[cc] * kGroup;
                    if (a.At) {   // the group's 16 values: one contiguous run of the transposed copy
                        const float4* at4 = reinterpret_cast<const float4*>(a.At + (int64_t)(j0 + cq + cc) * Kp + src0);
#pragma unroll
                        for (int k = 0; k < kGroup; k += 4) {
                            const float4 v = at4[k >> 2];
                            av[c2][k] = v.x; av[c2][k + 1] = v.y; av[c2][k + 2] = v.z; av[c2][k + 3] = v.w;
                        }
                    } else {
                        const float* ac = a.Acol + (int64_t)src0 * Kp + (j0 + cq + cc);
#pragma unroll
                        for (int k = 0; k < kGroup; ++k) av[c2][k] = ac[(int64_t)k * Kp];
                    }
#pragma unroll
                    for (int k = 0; k < kGroup; k += 4) {
                        const float4 d4 = *reinterpret_cast<const float4*>(drow + src0 + k);
                        dv[c2][k] = d4.x; dv[c2][k + 1] = d4.y; dv[c2][k + 2] = d4.z; dv[c2][k + 3] = d4.w;
                    }
                }
            }
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2) {
                const int cc = cb + c2;
                val[cc] = mv[cc];
                psi[cc] = 0;
                if (need[cc]) {
                    const int32_t src0 = gi[cc] * kGroup;
                    int32_t p = -1;
#pragma unroll
                    for (int k = 0; k < kGroup; ++k) {
                        const float x = dv[c2][k] + av[c2][k];
                        if (p < 0 && x == mv[cc]) { p = src0 + k; val[cc] = x; }
                    }
                    psi[cc] = clampi(p < 0 ? src0 : p, K);   // p < 0 is unreachable for finite/-inf inputs
                }
            }
        }
        // anchors (gathers issued together), then the stores
        int32_t anc[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            anc[cc] = 0;
            if (live[cc]) {
                if (f & F_ANC_FIRST) anc[cc] = psi[cc];
                else if (f & F_ANC_CHAIN) anc[cc] = aprev[psi[cc]];
            }
        }
        unsigned long long best_key = 0;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            if (!live[cc]) continue;
            const int32_t j = j0 + cq + cc;
            const float dnew = val[cc] + bpre[cc];
            dcur[j] = dnew;
            if (f & F_PSI_TABLE) a.psi16[off + (int64_t)t * K + j] = (uint16_t)psi[cc];
            if (f & F_LEAF_TABLE) slot_leaf(a, slot)[(int64_t)aux * Kp + j] = (uint16_t)psi[cc];
            if (f & (F_ANC_FIRST | F_ANC_CHAIN)) {
                anc[cc] = clampi(anc[cc], K);
                acur[j] = anc[cc];
            }
            if (f & F_SNAP_SUB) slot_snap(a, slot)[j] = dnew;
            if (f & F_SNAP_ROOT) {
                root_dsnap(a, off, aux)[j] = dnew;
                if (aux >= 1) root_link(a, off, pp, aux)[j] = anc[cc];
            }
            if (f & F_FINAL) {
                const unsigned long long k = order_key(dnew, j);
                if (k > best_key) best_key = k;
            }
        }
        if (f & F_FINAL) key_max(&a.keys[seq], best_key);
    }
    group_sync(&lds.gsync[grp], nsplit);   // partials and stash are reused by the group's next tile
}

// ---------------------------------------------------------------- wide rows
// Wide rows: each item is one chunk of 64 destination columns (one per lane)
// for up to 16 rows at once, computed by a whole block: the 16 waves split
// the predecessors, each streams its share of log A(i, chunk) from memory
// once for all the item's rows and keeps, per row and column, the maximum
// and the winning group of 16 predecessors; the previous step's scores are
// staged through LDS.  After a block barrier the partial maxima merge in
// wave order (the earliest group keeps ties), the winning group is refined
// and the outputs are written.  Row data crosses XCDs here, so it is read
// with coherent loads; the step barrier's release makes the stores visible.


__device__ __forceinline__ void wide_item(cargs_t& a, const float* __restrict__ Ap, const Row* list, int32_t nlist,
                                          int32_t rg, int32_t chunk, int32_t coh) {
    WideLds& L = g_lds.wide;
    const int32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t K = a.K, Kp = __builtin_amdgcn_readfirstlane(a.Kp);
    gfloat_t* Ag = as_global(Ap);
    const int32_t r0 = rg * kWideRows;
    const int32_t R = min(kWideRows, nlist - r0);
    const int32_t j = chunk * kWideCols + lane;
    if (tid < R) L.rows[tid] = ld_row(list + r0 + tid);
    __syncthreads();
    // this wave's output row (w < R): its emission score, fetched early
    float bpre = 0.0f;
    if (w < R && j < K) {
        const Row& rr = L.rows[w];
        bpre = as_global(rr.log_b)[(int64_t)rr.t * rr.ld + j];
    }
    // predecessors [i_lo, i_hi) of this wave, whole groups of 16 (wave-uniform,
    // so that each log A row's base address is scalar)
    const int32_t ng = Kp / kGroup;
    const int32_t i_lo = uni(((w * ng) / kEngWaves) * kGroup), i_hi = uni((((w + 1) * ng) / kEngWaves) * kGroup);
    float* stage = L.area[w];
    // log A rows i, lane column j: a scalar row base plus the lane's offset
    const int32_t jc = min(j, Kp - 1);
    if (R == 1) {
        // a single row (a long root pass or a vanilla decode at large K): the
        // step streams log A, so each lane keeps the loads of a whole stage
        // (64 predecessors) in flight before its arithmetic
        float m0 = -INFINITY;
        int32_t g0 = i_lo / kGroup;
        const Row& rr = L.rows[0];
        const float* dp = slot_delta(a, clampi(rr.slot, a.n_slots), (rr.t - 1) & 1);
        for (int32_t i0 = i_lo; i0 < i_hi; i0 += kWideStage) {
            const int32_t n = min(kWideStage, i_hi - i0);   // a multiple of 16
            float av[kWideStage];
#pragma unroll
            for (int k = 0; k < kWideStage; ++k)
                av[k] = k < n ? (Ag + (int64_t)(i0 + k) * Kp)[jc] : -INFINITY;
            if (lane < n) stage[lane] = coh ? ld_cg(dp + i0 + lane) : as_global(dp)[i0 + lane];
#pragma unroll
            for (int q = 0; q < kWideStage / kGroup; ++q) {
                if (q * kGroup < n) {
                    const float* sd = stage + q * kGroup;
                    float gm = -INFINITY;
#pragma unroll
                    for (int k = 0; k < kGroup; k += 2)
                        gm = fmaxf(fmaxf(gm, sd[k] + av[q * kGroup + k]), sd[k + 1] + av[q * kGroup + k + 1]);
                    const int32_t gi = (i0 + q * kGroup) / kGroup;
                    const bool up = gm > m0;
                    g0 = up ? gi : g0;
                    m0 = up ? gm : m0;
                }
            }
        }
        stage[lane] = m0;   // this wave's partial (its staging is done)
        reinterpret_cast<int32_t*>(stage)[kWideRows * kWideCols + lane] = g0;
    } else {
    float m[kWideRows];
    int32_t g[kWideRows];
#pragma unroll
    for (int r = 0; r < kWideRows; ++r) { m[r] = -INFINITY; g[r] = i_lo / kGroup; }
    // the next group's log A values are loaded while the current group's
    // arithmetic runs (one group ahead, across stage boundaries)
    float an[kGroup];
#pragma unroll
    for (int k = 0; k < kGroup; ++k) an[k] = i_lo < i_hi ? (Ag + (int64_t)(i_lo + k) * Kp)[jc] : 0.0f;
    for (int32_t i0 = i_lo; i0 < i_hi; i0 += kWideStage) {
        const int32_t n = min(kWideStage, i_hi - i0);   // a multiple of 16
        {
            // all rows' loads in flight before one wait (rows past R re-read
            // row 0, lanes past n their stage's first predecessor; neither
            // slot is read)
            const int32_t ic = i0 + (lane < n ? lane : 0);
            float sv[kWideRows];
#pragma unroll
            for (int r = 0; r < kWideRows; ++r) {
                const Row& rr = L.rows[r < R ? r : 0];
                const float* dp = slot_delta(a, clampi(rr.slot, a.n_slots), (rr.t - 1) & 1);
                sv[r] = coh ? ld_cg(dp + ic) : as_global(dp)[ic];
            }
#pragma unroll
            for (int r = 0; r < kWideRows; ++r) stage[r * kWideStage + lane] = sv[r];
        }
        for (int32_t k0 = 0; k0 < n; k0 += kGroup) {
            float av[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; ++k) av[k] = an[k];
            const int32_t inext = uni(i0 + k0 + kGroup);
            if (inext < i_hi) {
#pragma unroll
                for (int k = 0; k < kGroup; ++k) an[k] = (Ag + (int64_t)(inext + k) * Kp)[jc];
            }
            const int32_t gi = (i0 + k0) / kGroup;
#pragma unroll
            for (int r = 0; r < kWideRows; ++r) {
                if (r < R) {
                    const float* sd = stage + r * kWideStage + k0;
                    float gm = -INFINITY;
#pragma unroll
                    for (int k = 0; k < kGroup; k += 2) gm = fmaxf(fmaxf(gm, sd[k] + av[k]), sd[k + 1] + av[k + 1]);
                    // the first group reaching the running maximum keeps it
                    // (a select, not a maximum: no quieting of m)
                    const bool up = gm > m[r];
                    g[r] = up ? gi : g[r];
                    m[r] = up ? gm : m[r];
                }
            }
        }
    }
    // partials to this wave's area (its staging is done)
#pragma unroll
    for (int r = 0; r < kWideRows; ++r) {
        if (r < R) {
            stage[r * kWideCols + lane] = m[r];
            reinterpret_cast<int32_t*>(stage)[kWideRows * kWideCols + r * kWideCols + lane] = g[r];
        }
    }
    }
    __syncthreads();
    unsigned long long key = 0;
    if (w < R && j < K) {
        const Row& rr = L.rows[w];
        const int32_t t = rr.t, f = rr.flags, slot = clampi(rr.slot, a.n_slots);
        float mv = L.area[0][w * kWideCols + lane];
        int32_t gi = reinterpret_cast<const int32_t*>(L.area[0])[kWideRows * kWideCols + w * kWideCols + lane];
        for (int v = 1; v < kEngWaves; ++v) {
            const float x = L.area[v][w * kWideCols + lane];
            if (x > mv) { mv = x; gi = reinterpret_cast<const int32_t*>(L.area[v])[kWideRows * kWideCols + w * kWideCols + lane]; }
        }
        const float* dprev = slot_delta(a, slot, (t - 1) & 1);
        float val = mv;
        int32_t psi = 0;
        if ((f & F_NEED_ARG) || mv == 0.0f) {
            const int32_t src0 = gi * kGroup;
            float av[kGroup], dv[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                av[k] = Ag[(int64_t)(src0 + k) * Kp + j];
                dv[k] = coh ? ld_cg(dprev + src0 + k) : as_global(dprev)[src0 + k];
            }
            int32_t p = -1;
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                const float x = dv[k] + av[k];
                if (p < 0 && x == mv) { p = src0 + k; val = x; }
            }
            psi = clampi(p < 0 ? src0 : p, K);   // p < 0 is unreachable for finite/-inf inputs
        }
        int32_t anc = 0;
        if (f & F_ANC_FIRST) anc = psi;
        else if (f & F_ANC_CHAIN) {
            const int32_t* ap = slot_anc(a, slot, (t - 1) & 1) + psi;
            anc = clampi(coh ? ld_c(ap) : *ap, K);
        }
        const float dnew = val + bpre;
        slot_delta(a, slot, t & 1)[j] = dnew;
        if (f & F_PSI_TABLE) a.psi16[rr.off + (int64_t)t * K + j] = (uint16_t)psi;
        if (f & F_LEAF_TABLE) slot_leaf(a, slot)[(int64_t)rr.aux * Kp + j] = (uint16_t)psi;
        if (f & (F_ANC_FIRST | F_ANC_CHAIN)) slot_anc(a, slot, t & 1)[j] = anc;
        if (f & F_SNAP_SUB) slot_snap(a, slot)[j] = dnew;
        if (f & F_SNAP_ROOT) {
            root_dsnap(a, rr.off, rr.aux)[j] = dnew;
            if (rr.aux >= 1) root_link(a, rr.off, rr.pp, rr.aux)[j] = anc;
        }
        if (f & F_SNAP_DIV) {
            slot_div_d(a, slot, rr.aux)[j] = dnew;
            if (rr.aux >= 1) slot_div_l(a, slot, rr.aux)[j] = anc;
        }
        if (f & F_FINAL) key = order_key(dnew, j);
    }
    if (w < R && (L.rows[w].flags & F_FINAL)) {   // wave-uniform: the whole wave reduces
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(key, off, 64);
            if (o > key) key = o;
        }
        if (lane == 0) key_max(&a.keys[L.rows[w].seq], key);
    }
    __syncthreads();
}

// Two-column items, for XCDs with few dense rows and Kp <= kColMaxKp: a block
// computes 8 rows x 128 destinations, each lane two of them (j and j + 64).
// The rows' previous scores are staged whole in LDS and read there as
// broadcasts; the 16 waves split the predecessors, each keeping per row and
// column the maximum and the winning group of 16 predecessors (the earliest
// on ties).  The partial results merge through 64-bit LDS max keys (score in
// total order with -0 folded into +0, then the complement of the group), which
// selects the earliest group holding the maximum, as a merge in wave order
// does.  All 1024 threads then take one output each and refine its group: the
// group's 16 log A values are one contiguous run of the transposed copy, its
// 16 scores come from LDS.
__device__ __forceinline__ uint32_t score_order(float v) {
    const uint32_t u = __float_as_uint(v + 0.0f);   // -0 + +0 = +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float score_from_order(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ __forceinline__ void col_item(cargs_t& a, const float* __restrict__ Ap, const Row* list, int32_t r0,
                                         int32_t R, int32_t chunk) {
    ColLds& L = g_lds.col;
    const int32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t K = a.K, Kp = __builtin_amdgcn_readfirstlane(a.Kp);
    gfloat_t* Ag = as_global(Ap);
    if (tid < R) L.rows[tid] = ld_row(list + r0 + tid);
    L.key[tid] = 0ull;
    __syncthreads();
    // stage the rows' previous scores (16-byte aligned rows of Kp floats)
    {
        const int32_t q4 = Kp >> 2;
        for (int32_t q = tid; q < R * q4; q += kEngBlock) {
            const int32_t r = q / q4, i = (q - r * q4) << 2;
            const Row& rr = L.rows[r];
            const float* dp = slot_delta(a, clampi(rr.slot, a.n_slots), (rr.t - 1) & 1);
            *reinterpret_cast<float4*>(&L.d[r * Kp + i]) = *reinterpret_cast<const float4*>(dp + i);
        }
    }
    // this thread's output (row ro, destination jo): its emission score, early
    const int32_t ro = tid >> 7, jo = chunk * kColCols + (tid & (kColCols - 1));
    const bool out_ok = ro < R && jo < K;
    float bpre = 0.0f;
    if (out_ok) {
        const Row& rr = L.rows[ro];
        bpre = as_global(rr.log_b)[(int64_t)rr.t * rr.ld + jo];
    }
    __syncthreads();
    // predecessors [i_lo, i_hi) of this wave, whole groups of 16
    const int32_t ng = Kp / kGroup;
    const int32_t i_lo = ((w * ng) / kEngWaves) * kGroup, i_hi = (((w + 1) * ng) / kEngWaves) * kGroup;
    const int32_t ja = chunk * kColCols + lane;
    const int32_t jb = ja + 64 < Kp ? ja + 64 : ja;   // the last chunk may hold one column only
    float m[kColRows][2];
    int32_t g[kColRows][2];
#pragma unroll
    for (int r = 0; r < kColRows; ++r) {
        m[r][0] = m[r][1] = -INFINITY;
        g[r][0] = g[r][1] = i_lo / kGroup;
    }
    for (int32_t i0 = i_lo; i0 < i_hi; i0 += kGroup) {
        float a0[kGroup], a1[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            a0[k] = Ag[(int64_t)(i0 + k) * Kp + ja];
            a1[k] = Ag[(int64_t)(i0 + k) * Kp + jb];
        }
        const int32_t gi = i0 / kGroup;
#pragma unroll
        for (int r = 0; r < kColRows; ++r) {
            if (r < R) {
                const float* sd = static_cast<const float*>(__builtin_assume_aligned(&L.d[r * Kp + i0], 16));
                float g0 = -INFINITY, g1 = -INFINITY;
#pragma unroll
                for (int k = 0; k < kGroup; k += 2) {
                    g0 = fmaxf(fmaxf(g0, sd[k] + a0[k]), sd[k + 1] + a0[k + 1]);
                    g1 = fmaxf(fmaxf(g1, sd[k] + a1[k]), sd[k + 1] + a1[k + 1]);
                }
                if (g0 > m[r][0]) { m[r][0] = g0; g[r][0] = gi; }
                if (g1 > m[r][1]) { m[r][1] = g1; g[r][1] = gi; }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kColRows; ++r) {
        if (r < R) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const unsigned long long k = ((unsigned long long)score_order(m[r][c]) << 32) |
                                             (uint32_t)(0xffffffffu - (uint32_t)g[r][c]);
                __hip_atomic_fetch_max(&L.key[r * kColCols + c * 64 + lane], k, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    unsigned long long fkey = 0;
    if (out_ok) {
        const Row& rr = L.rows[ro];
        const int32_t t = rr.t, f = rr.flags, slot = clampi(rr.slot, a.n_slots);
        const unsigned long long key = L.key[tid];
        const float mv = score_from_order((uint32_t)(key >> 32));
        const int32_t gi = clampi((int32_t)(0xffffffffu - (uint32_t)key), ng);
        float val = mv;
        int32_t psi = 0;
        if ((f & F_NEED_ARG) || mv == 0.0f) {
            // the first candidate of the group equal to the maximum; its value
            // is the one stored (signed zero)
            const int32_t src0 = gi * kGroup;
            const float4* at4 = reinterpret_cast<const float4*>(a.At + (int64_t)jo * Kp + src0);
            float av[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; k += 4) {
                const float4 v = at4[k >> 2];
                av[k] = v.x; av[k + 1] = v.y; av[k + 2] = v.z; av[k + 3] = v.w;
            }
            const float* sd = &L.d[ro * Kp + src0];
            int32_t p = -1;
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                const float x = sd[k] + av[k];
                if (p < 0 && x == mv) { p = src0 + k; val = x; }
            }
            psi = clampi(p < 0 ? src0 : p, K);   // p < 0 is unreachable for finite/-inf inputs
        }
        int32_t anc = 0;
        if (f & F_ANC_FIRST) anc = psi;
        else if (f & F_ANC_CHAIN) anc = clampi(slot_anc(a, slot, (t - 1) & 1)[psi], K);
        const float dnew = val + bpre;
        slot_delta(a, slot, t & 1)[jo] = dnew;
        if (f & F_PSI_TABLE) a.psi16[rr.off + (int64_t)t * K + jo] = (uint16_t)psi;
        if (f & F_LEAF_TABLE) slot_leaf(a, slot)[(int64_t)rr.aux * Kp + jo] = (uint16_t)psi;
        if (f & (F_ANC_FIRST | F_ANC_CHAIN)) slot_anc(a, slot, t & 1)[jo] = anc;
        if (f & F_SNAP_SUB) slot_snap(a, slot)[jo] = dnew;
        if (f & F_SNAP_ROOT) {
            root_dsnap(a, rr.off, rr.aux)[jo] = dnew;
            if (rr.aux >= 1) root_link(a, rr.off, rr.pp, rr.aux)[jo] = anc;
        }
        if (f & F_FINAL) fkey = order_key(dnew, jo);
    }
    // a wave holds 64 destinations of one row (wave-uniform test)
    if (ro < R && (L.rows[ro].flags & F_FINAL)) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(fkey, off, 64);
            if (o > fkey) fkey = o;
        }
        if (lane == 0) key_max(&a.keys[L.rows[ro].seq], fkey);
    }
    __syncthreads();
}

// ---------------------------------------------------------------- column slabs
// Local dense rows of a model with K = Kp = 512 or 1024 (KP).  Each block
// keeps a slab of log A in registers for a whole column pass: lane l of wave
// w holds A(i, j) for its destination j (one per lane) and the 64
// predecessors i = 64 pw + k of its wave's share (pw = w mod KP/64), so a
// pass covers 64 columns at KP = 1024 (16 waves over the predecessors) or
// 128 at 512 (two sets of 8 waves).  A row's previous scores are read from
// LDS four at a time with every lane of the wave at the same address (a
// broadcast), so a candidate costs one add and half a three-input max.  Each
// lane keeps, per row, the maximum of each group of 16 predecessors and the
// first group reaching its running maximum; partials meet in a 64-bit LDS
// atomic max (score in total order, then the complement of the group index,
// so ties go to the earliest group).  The epilogue refines the winning group
// from the transposed copy of log A exactly as a column item does.
//
// The work of a step on an XCD is nf rows x (KP^2 / 65536) column passes,
// split evenly over the XCD's compute blocks by unit ranges (a unit = one
// row in one pass, ordered pass-major), so every block gets the same number
// of units to within one and loads at most two slabs.

// Partial key of one row: the lane's 64 predecessors (its wave's share pw)
// for its destination; dr = the row's previous scores from predecessor 64 pw.
__device__ __forceinline__ unsigned long long slab_row_key(const float* dr, const float (&av)[64], int32_t pw) {
    float best = -INFINITY;
    int32_t bg = 0;
    const float4* d4 = reinterpret_cast<const float4*>(dr);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        float m = -INFINITY;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = d4[4 * g + q];   // the same address in every lane
            m = fmaxf(fmaxf(m, v.x + av[16 * g + 4 * q]), v.y + av[16 * g + 4 * q + 1]);
            m = fmaxf(fmaxf(m, v.z + av[16 * g + 4 * q + 2]), v.w + av[16 * g + 4 * q + 3]);
        }
        if (m > best) { best = m; bg = g; }
    }
    return ((unsigned long long)score_order(best) << 32) | (uint32_t)(0xffffffffu - (uint32_t)(pw * 4 + bg));
}

// One chunk of R units (u0 .., pass-major: unit u is row u mod nf of pass
// u / nf) that may span column passes: rows loaded and scores staged once,
// the slab reloaded where the pass changes, then one merge, refine and store
// (the outputs of a column item).
template <int KP>
__device__ __forceinline__ void slab_chunk(cargs_t& a, gfloat_t* Ag, const Row* list, int32_t nf, int64_t u0,
                                           int32_t R, float (&av)[64], int32_t& loaded, bool rows_ready = false) {
    constexpr int32_t wpc = KP / 64, pcols = (kEngWaves / wpc) * 64;
    SlabLds& L = g_lds.slab;
    const int32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t K = a.K;
    const int32_t csl = w / wpc, pw = w - csl * wpc;
    if (tid < R && !rows_ready) {   // (rows_ready: read while the step barrier was closing)
        const int64_t u = u0 + tid;
        const int32_t p = (int32_t)(u / nf);
        L.rows[tid] = ld_row(list + (int32_t)(u - (int64_t)p * nf));
        L.upass[tid] = p;
    }
    L.key[tid] = 0ull;
    __syncthreads();
    // this thread's output: its emission score first, so that its latency
    // overlaps the staging loads
    const int32_t ro = tid / pcols;
    const bool out_ok = ro < R;
    const int32_t jo = (out_ok ? L.upass[ro] : 0) * pcols + (tid - ro * pcols);
    float bpre = 0.0f;
    if (out_ok) {
        const Row& rr = L.rows[ro];
        bpre = as_global(rr.log_b)[(int64_t)rr.t * rr.ld + jo];
    }
    {
        // the rows' previous scores go straight from memory to LDS (LDS DMA,
        // 16 bytes per lane: a wave moves 1 KB of one row), so every load of
        // the chunk is in flight at once and holds no registers
        typedef __attribute__((address_space(1))) const void gvoid_t;
        typedef __attribute__((address_space(3))) void lvoid_t;
        constexpr int32_t q4 = KP / 4, nq = (kSlabChunkMax * q4 + kEngBlock - 1) / kEngBlock;
        const int32_t qn = R * q4;   // a multiple of 64: a wave's 64 entries share one row
#pragma unroll
        for (int u = 0; u < nq; ++u) {
            const int32_t qw = uni(u * kEngBlock + (tid & ~63));
            if (qw < qn) {
                const int32_t r = qw / q4, i0 = (qw - r * q4) * 4;
                const Row& rr = L.rows[r];
                const float* dp = slot_delta(a, clampi(rr.slot, a.n_slots), (rr.t - 1) & 1);
                lvoid_t* dst = reinterpret_cast<lvoid_t*>(
                    (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uintptr_t)&L.d[r * KP + i0]));
                __builtin_amdgcn_global_load_lds(reinterpret_cast<gvoid_t*>(reinterpret_cast<uintptr_t>(dp + i0 + 4 * lane)),
                                                 dst, 16, 0, 0);
            }
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
    for (int32_t rc = 0; rc < R; ++rc) {
        const int32_t p = L.upass[rc];   // block-uniform
        if (p != loaded) {
            gfloat_t* col = Ag + (int64_t)(pw * 64) * KP + p * pcols + csl * 64 + lane;
#pragma unroll
            for (int k = 0; k < 64; ++k) av[k] = col[k * KP];
            loaded = p;
        }
        const unsigned long long k = slab_row_key(&L.d[rc * KP + pw * 64], av, pw);
        __hip_atomic_fetch_max(&L.key[rc * pcols + csl * 64 + lane], k, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    unsigned long long fkey = 0;
    if (out_ok) {
        const Row& rr = L.rows[ro];
        const int32_t t = rr.t, f = rr.flags, slot = clampi(rr.slot, a.n_slots);
        const unsigned long long key = L.key[tid];
        const float mv = score_from_order((uint32_t)(key >> 32));
        float val = mv;
        int32_t psi = 0;
        if ((f & F_NEED_ARG) || mv == 0.0f) {
            const int32_t gi = clampi((int32_t)(0xffffffffu - (uint32_t)key), KP / kGroup);
            const int32_t src0 = gi * kGroup;
            const float4* at4 = reinterpret_cast<const float4*>(a.At + (int64_t)jo * KP + src0);
            float avr[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; k += 4) {
                const float4 v = at4[k >> 2];
                avr[k] = v.x; avr[k + 1] = v.y; avr[k + 2] = v.z; avr[k + 3] = v.w;
            }
            const float* sd = &L.d[ro * KP + src0];
            int32_t q = -1;
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                const float x = sd[k] + avr[k];
                if (q < 0 && x == mv) { q = src0 + k; val = x; }
            }
            psi = clampi(q < 0 ? src0 : q, K);
        }
        int32_t anc = 0;
        if (f & F_ANC_FIRST) anc = psi;
        else if (f & F_ANC_CHAIN) anc = clampi(slot_anc(a, slot, (t - 1) & 1)[psi], K);
        const float dnew = val + bpre;
        slot_delta(a, slot, t & 1)[jo] = dnew;
        if (f & F_PSI_TABLE) a.psi16[rr.off + (int64_t)t * K + jo] = (uint16_t)psi;
        if (f & F_LEAF_TABLE) slot_leaf(a, slot)[(int64_t)rr.aux * KP + jo] = (uint16_t)psi;
        if (f & (F_ANC_FIRST | F_ANC_CHAIN)) slot_anc(a, slot, t & 1)[jo] = anc;
        if (f & F_SNAP_SUB) slot_snap(a, slot)[jo] = dnew;
        if (f & F_SNAP_ROOT) {
            root_dsnap(a, rr.off, rr.aux)[jo] = dnew;
            if (rr.aux >= 1) root_link(a, rr.off, rr.pp, rr.aux)[jo] = anc;
        }
        if (f & F_FINAL) fkey = order_key(dnew, jo);
    }
    // a wave holds 64 destinations of one row (wave-uniform test)
    if (ro < R && (L.rows[ro].flags & F_FINAL)) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(fkey, off, 64);
            if (o > fkey) fkey = o;
        }
        if (lane == 0) key_max(&a.keys[L.rows[ro].seq], fkey);
    }
    __syncthreads();
}

// This block's share of the dense rows of its XCD at one step (rank among the
// XCD's nsl slab blocks; the scheduler block, rank -1, takes none).  When
// the blocks divide evenly over the column passes, each pass gets a team of
// nsl / npass blocks that split its rows, so no block loads two slabs; else
// the units (row, pass), pass-major, are split evenly, and a chunk may span
// two passes.
struct SlabShare {
    int64_t u, u1;   // this block's units
    int32_t nsl;     // blocks sharing the slab units (the others take block and light rows)
    int32_t nbx;     // block rows and light rows set aside for the other blocks
    int32_t lo_light;
};

// A block row (a finalize or a leaf's end) or a light row run after a full
// slab share would finish last: up to a quarter of the XCD's blocks take
// them instead (one block row per block, one light row per wave) and the
// others split the slab units.
__device__ __forceinline__ SlabShare slab_share(cargs_t& a, int32_t nx, int32_t rank, int32_t nf, int32_t nl,
                                                int32_t nbm) {
    SlabShare sh;
    sh.nsl = nx;
    sh.nbx = 0;
    sh.lo_light = 0;
    if (a.method != FV_BEAM && nx > 0) {
        const int32_t cap = nx / 4;
        sh.nbx = min(nbm, cap);
        const int32_t nlx = min((nl + kEngWaves - 1) / kEngWaves, cap - sh.nbx);
        sh.nsl = nx - sh.nbx - nlx;
        sh.lo_light = min(nl, nlx * kEngWaves);
    }
    const int32_t wpc = a.Kp / 64, pcols = (kEngWaves / wpc) * 64, npass = a.Kp / pcols;
    sh.u = sh.u1 = 0;
    if (rank < 0 || rank >= sh.nsl || nf <= 0) return sh;
    if (sh.nsl % npass == 0) {
        const int32_t team = sh.nsl / npass, p = rank / team, m = rank - p * team;
        sh.u = (int64_t)p * nf + ((int64_t)m * nf) / team;
        sh.u1 = (int64_t)p * nf + ((int64_t)(m + 1) * nf) / team;
    } else {
        const int64_t U = (int64_t)nf * npass;
        sh.u = U * rank / sh.nsl;
        sh.u1 = U * (rank + 1) / sh.nsl;
    }
    return sh;
}

template <int KP>
__device__ __forceinline__ void slab_items_kp(cargs_t& a, const float* __restrict__ Ap, const Row* list, int32_t nf,
                                              int64_t u, int64_t u1, bool first_ready) {
    constexpr int32_t pcols = (kEngWaves / (KP / 64)) * 64, crows = kEngBlock / pcols;
    gfloat_t* Ag = as_global(Ap);
    float av[64];
    int32_t loaded = -1;
    for (int64_t u0 = u; u0 < u1; u0 += crows)
        slab_chunk<KP>(a, Ag, list, nf, u0, (int32_t)min((int64_t)crows, u1 - u0), av, loaded,
                       first_ready && u0 == u);
}

// While the step barrier closes, once the next step's counts are known:
// read this block's first chunk of rows for that step into LDS (the
// scheduler wrote them before the counts word).  Returns the chunk's first
// unit, or -1.
__device__ __forceinline__ int64_t slab_prefetch_rows(cargs_t& a, uint32_t x, int32_t nx, int32_t rank, int nxt,
                                                      unsigned long long cw) {
    SlabLds& L = g_lds.slab;
    const int32_t nf = (int32_t)(cw & 0x3fff), nl = (int32_t)((cw >> 14) & 0x3fff), nbm = (int32_t)((cw >> 28) & 0x3fff);
    if (((cw >> 42) & 1) || nf <= 0 || nf > kLocalColRows || a.force_tiles || a.sparse) return -1;
    const SlabShare sh = slab_share(a, nx, rank, nf, nl, nbm);
    if (sh.u >= sh.u1) return -1;
    const int32_t pcols = (kEngWaves / (a.Kp / 64)) * 64, crows = kEngBlock / pcols;
    const int32_t R = (int32_t)min((int64_t)crows, sh.u1 - sh.u);
    const int32_t tid = threadIdx.x;
    if (tid < R) {
        const int64_t u = sh.u + tid;
        const int32_t p = (int32_t)(u / nf);
        L.rows[tid] = ld_row(list_full(a, nxt, x) + (int32_t)(u - (int64_t)p * nf));
        L.upass[tid] = p;
    }
    return sh.u;
}

// ---------------------------------------------------------------- sparse rows
// Sparse model (CSR): one wave computes 64 destinations j (one per lane) of
// one row by pulling over j's in-edges, which are in (source, edge) order:
//     c(j) = max over in-edges (i -> j) of delta_{t-1}(i) + log A(i, j)
// with the first maximum winning, so psi(j) is the lowest source on ties and
// the stored value is that candidate's.  A destination without in-edges gets
// -inf (and psi 0).  Vanilla backpointers hold the winning in-edge's slot
// within j's list.  F_START rows compute the task's start vector instead:
// log pi + log B_0 at m = 0, else the anchored boundary
// (alpha + log A(q*_{m-1}, j)) + log B_m(j), the edge found by binary search
// among j's in-edges (sources are sorted).  Rows and their buffers belong to
// this XCD, so plain loads see the previous step's stores.
__device__ __noinline__ void sparse_unit(cargs_t& a_in, const Row* list, int32_t ridx, int32_t c64) {
    cargs_t& a = uniform_args(a_in);
    const int32_t lane = threadIdx.x & 63;
    const int32_t K = a.K;
    const Row r = ld_row(list + ridx);
    const int32_t j = c64 * 64 + lane;
    const int32_t t = r.t, f = r.flags, slot = clampi(r.slot, a.n_slots);
    const int32_t* __restrict__ in_ptr = a.in_ptr;
    const int32_t* __restrict__ in_src = a.in_src;
    const float* __restrict__ in_val = a.in_val;
    unsigned long long key = 0;
    if (j < K) {
        const float bt = emission(a, r.log_b, r.ld, t, j);
        const int32_t e0 = in_ptr[j], e1 = in_ptr[j + 1];
        float dnew;
        int32_t psi = 0, pslot = 0;
        if (f & F_START) {
            if (t == 0) {
                dnew = a.log_pi ? a.log_pi[j] + bt : bt;
            } else {
                const SeqInfo& sq = a.seqs[r.seq];
                const int32_t q = ld_c(sq.path + t - 1);
                const float alpha = ld_cf(a.alpha_at + sq.alpha_off + t - 1);
                int32_t lo = e0, hi = e1;   // first in-edge with source >= q
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (in_src[mid] < q) lo = mid + 1; else hi = mid;
                }
                float c = -INFINITY;
                bool found = false;
                for (int32_t p = lo; p < e1 && in_src[p] == q; ++p) {
                    const float x = alpha + in_val[p];
                    if (!found || x > c) { c = x; found = true; }
                }
                dnew = found ? c + bt : -INFINITY;
            }
        } else {
            const float* dprev = slot_delta(a, slot, (t - 1) & 1);
            float best = -INFINITY;
            int32_t bp = -1;
            // four in-edges per round: their gathers are issued together
            for (int32_t p0 = e0; p0 < e1; p0 += 4) {
                int32_t sidx[4];
                float av[4], dv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int32_t p = min(p0 + k, e1 - 1);
                    sidx[k] = in_src[p];
                    av[k] = in_val[p];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) dv[k] = dprev[sidx[k]];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float x = dv[k] + av[k];
                    if (p0 + k < e1 && (bp < 0 || x > best)) { best = x; bp = p0 + k; }
                }
            }
            if (bp >= 0) {
                psi = in_src[bp];
                pslot = bp - e0;
            }
            dnew = best + bt;
        }
        int32_t anc = 0;
        if (f & F_ANC_FIRST) anc = psi;
        else if (f & F_ANC_CHAIN) anc = clampi(slot_anc(a, slot, (t - 1) & 1)[psi], K);
        slot_delta(a, slot, t & 1)[j] = dnew;
        if (f & F_PSI_TABLE) a.psi16[r.off + (int64_t)t * K + j] = (uint16_t)pslot;
        if (f & (F_ANC_FIRST | F_ANC_CHAIN)) slot_anc(a, slot, t & 1)[j] = anc;
        if (f & F_SNAP_SUB) slot_snap(a, slot)[j] = dnew;
        if (f & F_SNAP_ROOT) {
            root_dsnap(a, r.off, r.aux)[j] = dnew;
            if (r.aux >= 1) root_link(a, r.off, r.pp, r.aux)[j] = anc;
        }
        if (f & F_SNAP_DIV) {   // a division of a w-way subtask
            slot_div_d(a, slot, r.aux)[j] = dnew;
            if (r.aux >= 1) slot_div_l(a, slot, r.aux)[j] = anc;
        }
        if (f & F_FINAL) key = order_key(dnew, j);
    }
    if (f & F_FINAL) {   // wave-uniform
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(key, off, 64);
            if (o > key) key = o;
        }
        if (lane == 0) key_max(&a.keys[r.seq], key);
    }
}

// ---------------------------------------------------------------- light rows
__device__ __forceinline__ void wave_argmax(float& v, int32_t& idx) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float v2 = __shfl_xor(v, off, 64);
        const int32_t i2 = __shfl_xor(idx, off, 64);
        if (v2 > v || (v2 == v && i2 < idx)) { v = v2; idx = i2; }
    }
}

// One wave: the O(K) operations of a task (start step, end-only step,
// final selection and boundary resolution).
__device__ __noinline__ void light_row(cargs_t& a_in, const float* __restrict__ Ap, const Row& r) {
    cargs_t& a = uniform_args(a_in);
    const int32_t lane = threadIdx.x & 63;
    SeqInfo& sq = a.seqs[r.seq];
    const int32_t K = a.K, Kp = a.Kp;
    const int32_t slot = clampi(r.slot, a.n_slots);
    if (r.aux == L_INIT) {
        const int32_t m = r.m;
        float* dst = slot_delta(a, slot, m & 1);
        float* oth = slot_delta(a, slot, (m + 1) & 1);
        const float* bm = r.log_b + (int64_t)m * r.ld;
        int32_t q = -1;
        float alpha = 0.0f;
        if (m > 0) {
            q = ld_c(sq.path + m - 1);
            alpha = ld_cf(a.alpha_at + sq.alpha_off + m - 1);
            if (q >= K) q = -1;
        }
        unsigned long long best_key = 0;
        const float* arow = Ap + (int64_t)(q < 0 ? 0 : q) * Kp;
        // 8 destinations per lane per round: every load of a round is issued
        // before its stores (which might alias them)
        for (int32_t j0 = lane; j0 < Kp; j0 += 64 * 8) {
            float bv[8], xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t j = j0 + 64 * u;
                bv[u] = 0.0f;
                xv[u] = 0.0f;
                if (j < K) {
                    bv[u] = bm[j];
                    if (m == 0) xv[u] = a.log_pi ? a.log_pi[j] : 0.0f;
                    else if (q >= 0) xv[u] = arow[j];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t j = j0 + 64 * u;
                if (j >= Kp) break;
                float v = -INFINITY;
                if (j < K) {
                    if (m == 0) v = a.log_pi ? xv[u] + bv[u] : bv[u];
                    else if (q >= 0) { const float c = a.relative_init ? xv[u] : alpha + xv[u]; v = c + bv[u]; }
                    if (r.flags & F_SNAP_SUB) slot_snap(a, slot)[j] = v;
                    if (r.flags & F_SNAP_DIV) slot_div_d(a, slot, 0)[j] = v;
                    if (r.flags & F_SNAP_ROOT) root_dsnap(a, r.off, 0)[j] = v;
                    if (r.flags & F_FINAL) {
                        const unsigned long long k = order_key(v, j);
                        if (k > best_key) best_key = k;
                    }
                } else {
                    oth[j] = -INFINITY;
                }
                dst[j] = v;
            }
        }
        if (r.flags & F_FINAL) {
            for (int off = 32; off >= 1; off >>= 1) {
                const unsigned long long o = __shfl_xor(best_key, off, 64);
                if (o > best_key) best_key = o;
            }
            if (lane == 0) key_max(&a.keys[r.seq], best_key);
        }
    } else if (r.aux == L_END) {
        // only the known end state q*_n is evaluated at a subtask's last step
        if (ld_c(&sq.status) < 0) return;
        const int32_t n = r.n, tmid = (r.m + r.n) >> 1;
        const int32_t qn = ld_c(sq.path + n);
        if (qn < 0 || qn >= K) return;
        const float* dprev = slot_delta(a, slot, (n - 1) & 1);
        float best = -INFINITY;
        int32_t arg = 0x7fffffff;
        if (a.sparse) {
            // q*_n's in-edges in order; the lowest position wins ties
            const int32_t e0 = a.in_ptr[qn], e1 = a.in_ptr[qn + 1];
            for (int32_t p = e0 + lane; p < e1; p += 64) {
                const float x = dprev[a.in_src[p]] + a.in_val[p];
                if (arg == 0x7fffffff || x > best) { best = x; arg = p; }
            }
            wave_argmax(best, arg);
            arg = arg == 0x7fffffff ? 0 : a.in_src[arg];
        } else {
            const float* ac = a.Acol + qn;  // column q*_n of log A
            const bool coh = a.wide;
            for (int32_t i0 = lane; i0 < K; i0 += 64 * 8) {   // 8 candidates per lane in flight
                float dv[8], av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int32_t i = min(i0 + 64 * u, K - 1);
                    dv[u] = coh ? ld_cf(dprev + i) : dprev[i];
                    av[u] = ac[(int64_t)i * Kp];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float x = dv[u] + av[u];
                    if (i0 + 64 * u < K && (arg == 0x7fffffff || x > best)) { best = x; arg = i0 + 64 * u; }
                }
            }
            wave_argmax(best, arg);
        }
        if (lane == 0 && r.kind == KIND_SUB && a.wsplit > 2) {
            // w-way: the last division state from the anchors, then the chain
            // of division links down to the first; each with its score
            arg = clampi(arg, K);
            const int32_t L = n - r.m + 1, wp = sub_parts(r.m, n, a.wsplit);
            const int32_t last = r.m + (int32_t)seg_end(L, wp, wp - 2);
            const int32_t* ap = slot_anc(a, slot, (n - 1) & 1);
            int32_t q = clampi((n - 1 == last) ? arg : (a.wide ? ld_c(ap + arg) : ap[arg]), K);
            for (int32_t k = wp - 2; k >= 0; --k) {
                const int32_t e = r.m + (int32_t)seg_end(L, wp, k);
                const float* dk = slot_div_d(a, slot, k);
                st_c(sq.path + e, q);
                st_cf(a.alpha_at + sq.alpha_off + e, a.wide ? ld_cf(dk + q) : dk[q]);
                if (k >= 1) {
                    const int32_t* lk = slot_div_l(a, slot, k);
                    q = clampi(a.wide ? ld_c(lk + q) : lk[q], K);
                }
            }
        } else if (lane == 0) {
            arg = clampi(arg, K);
            const int32_t* ap = slot_anc(a, slot, (n - 1) & 1);
            const int32_t qmid = clampi((n == tmid + 1) ? arg : (a.wide ? ld_c(ap + arg) : ap[arg]), K);
            const float* sn = slot_snap(a, slot);
            st_c(sq.path + tmid, qmid);
            st_cf(a.alpha_at + sq.alpha_off + tmid, a.wide ? ld_cf(sn + qmid) : sn[qmid]);
        }
    }
    // L_BSPAWN: nothing to do (see its definition)
}

// ---------------------------------------------------------------- beam rows
// FLASH-BS (Sec. V-C): every step keeps at most B states, ranked by
// (score desc, state asc), -inf dropped.  A beam task's step is split into
// W parts, column ranges of about K/W destinations in state order, each
// computed by one block:
//   rebuild: the previous step's beam = the top B of the union of the
//            parts' kept lists (each in state order, so their concatenation
//            is too), by a radix select of the B-th largest score key with
//            ties at it going to the lowest states;
//   scores:  for each destination j of the part, c(j) = max over the beam
//            (in state order) of v_b + log A(s_b, j), the first maximum
//            wins; score(j) = c(j) + log B_t(j);
//   keep:    the part's own top B by the same rule, stored in state order.
// The union of the parts' top-B lists holds the global top B, so the
// rebuild is exact; W = 1 is the single-block case.  A beam record is a
// 64-word header (word 0 = entry count) followed by the state, score and
// anchor arrays (Bc entries each).  Slot of a beam task: records [0, W) are
// the parts of even t, [W, 2W) of odd t, record 2W the beam at t_mid (its
// header word 1 flags a task that needs the exact re-decode).  Root
// division beams are records in the root copy area.  Division and t_mid
// beams are written by the block that rebuilds that step's beam.


struct BeamRec {
    int32_t* hdr;
    int32_t* s;
    float* v;
    int32_t* a;
};

__device__ __forceinline__ BeamRec beam_rec(float* base, int32_t Bc) {
    BeamRec r;
    r.hdr = reinterpret_cast<int32_t*>(base);
    r.s = reinterpret_cast<int32_t*>(base + 64);
    r.v = base + 64 + Bc;
    r.a = reinterpret_cast<int32_t*>(base + 64 + 2 * (int64_t)Bc);
    return r;
}
__device__ __forceinline__ BeamRec slot_beam(cargs_t& a, int32_t slot, int32_t k) {
    return beam_rec(a.slot_base + (int64_t)slot * a.slot_floats + k * a.brec, a.Bc);
}
__device__ __forceinline__ BeamRec slot_part(cargs_t& a, int32_t slot, int32_t parity, int32_t part) {
    return slot_beam(a, slot, parity * a.bw + part);
}
__device__ __forceinline__ BeamRec slot_snap_beam(cargs_t& a, int32_t slot) {
    return slot_beam(a, slot, 2 * a.bw);
}
__device__ __forceinline__ BeamRec root_beam(cargs_t& a, int64_t root_off, int32_t d) {
    return beam_rec(a.root_copy + (root_off + d) * a.brec, a.Bc);
}
__device__ __forceinline__ int32_t* beam_fallback_flag(cargs_t& a, int32_t slot) {
    return slot_snap_beam(a, slot).hdr + 1;
}
// destinations [lo, hi) of part p of W
__device__ __forceinline__ int32_t part_lo(int32_t K, int32_t W, int32_t p) { return (int32_t)(((int64_t)p * K) / W); }

// Exclusive block-wide prefix sum of one int per thread; *total = the sum.
__device__ int32_t block_exscan(int32_t v, int32_t* total, int32_t* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int u = 0; u < kEngWaves; ++u) {
        const int32_t y = wsum[u];
        if (u < w) before += y;
        all += y;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// Orderable key of a score (-0 and +0 equal).
__device__ __forceinline__ uint32_t score_key(float v) {
    if (v == 0.0f) v = 0.0f;
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// The index held in the largest key over the block (keys: 0 = none).
__device__ int32_t block_argmax_key(unsigned long long key) {
    BeamLds& L = g_lds.beam;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        if (o > key) key = o;
    }
    if (lane == 0) L.wkey[w] = key;
    __syncthreads();
    unsigned long long best = 0;
    for (int u = 0; u < kEngWaves; ++u) best = L.wkey[u] > best ? L.wkey[u] : best;
    __syncthreads();
    return (int32_t)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull));
}

// Top B of n entries given in state order (score v[k], state s ? s[k] :
// s0 + k, anchor an[k]) by (score desc, state asc), -inf dropped.  out(p,
// state, score, anchor) receives the kept entries in state order; returns
// how many were kept.
template <typename Out>
__device__ int32_t beam_select(int32_t n, int32_t B, const float* v, const int32_t* s, int32_t s0,
                               const int32_t* an, Out out) {
    BeamLds& L = g_lds.beam;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t per = (n + kEngBlock - 1) / kEngBlock;
    const int32_t k0 = min(n, tid * per), k1 = min(n, k0 + per);
    // finite entries, and the bits all their keys share (AND and OR of the keys)
    int32_t nfin = 0;
    uint32_t kand = 0xffffffffu, kor = 0u;
    for (int32_t k = k0; k < k1; ++k) {
        if (v[k] == -INFINITY) continue;
        const uint32_t u = score_key(v[k]);
        ++nfin;
        kand &= u;
        kor |= u;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        kand &= (uint32_t)__shfl_xor((int32_t)kand, off, 64);
        kor |= (uint32_t)__shfl_xor((int32_t)kor, off, 64);
    }
    if (lane == 0) L.wkey[wv] = ((unsigned long long)kand << 32) | kor;
    int32_t n_finite;
    block_exscan(nfin, &n_finite, L.wsum);   // (its barriers also publish wkey)
    const bool all = n_finite <= B;
    // The threshold: radix passes of 8 bits from the highest byte in which
    // the finite keys differ; a pass whose chosen bin holds exactly the
    // entries still needed ends the search (the whole bin is kept), else the
    // last pass leaves the exact B-th key, whose equal entries are taken in
    // index order (the same set as the full four passes).
    uint32_t prefix = 0, mask = 0;
    int32_t rem = B;
    bool exact = false;
    if (!all) {
        uint32_t gand = 0xffffffffu, gor = 0u;
#pragma unroll
        for (int u = 0; u < kEngWaves; ++u) {
            gand &= (uint32_t)(L.wkey[u] >> 32);
            gor |= (uint32_t)L.wkey[u];
        }
        const uint32_t diff = gand ^ gor;
        if (diff == 0u) {   // every finite key equal: the first B in index order
            prefix = gor;
            mask = 0xffffffffu;
            exact = true;
        } else {
            const int32_t hb = 31 - __builtin_clz(diff);
            const int32_t sh0 = (hb >> 3) << 3;
            mask = sh0 >= 24 ? 0u : ~((1u << (sh0 + 8)) - 1u);
            prefix = gor & mask;
            for (int shift = sh0; shift >= 0; shift -= 8) {
                for (int k = tid; k < 256; k += kEngBlock) L.hist[k] = 0;
                __syncthreads();
                for (int32_t k = k0; k < k1; ++k) {
                    const float x = v[k];
                    if (x == -INFINITY) continue;
                    const uint32_t u = score_key(x);
                    if ((u & mask) == prefix) atomicAdd(&L.hist[(u >> shift) & 255u], 1u);
                }
                __syncthreads();
                if (tid < 64) {
                    // lane l owns digits 4l..4l+3; find the digit where the
                    // count from the top reaches rem
                    int32_t c[4];
#pragma unroll
                    for (int d = 0; d < 4; ++d) c[d] = (int32_t)L.hist[4 * tid + d];
                    const int32_t own = c[0] + c[1] + c[2] + c[3];
                    int32_t incl = own;  // sum over lanes >= tid
#pragma unroll
                    for (int off = 1; off < 64; off <<= 1) {
                        const int32_t y = __shfl_down(incl, off, 64);
                        if (tid + off < 64) incl += y;
                    }
                    int32_t above = incl - own;
                    for (int d = 3; d >= 0; --d) {
                        if (above < rem && above + c[d] >= rem) {
                            L.misc[0] = 4 * tid + d;
                            L.misc[1] = rem - above;
                            L.misc[2] = c[d];
                        }
                        above += c[d];
                    }
                }
                __syncthreads();
                prefix |= (uint32_t)L.misc[0] << shift;
                mask |= 255u << shift;
                rem = L.misc[1];
                const int32_t cbin = L.misc[2];
                __syncthreads();
                if (cbin == rem) break;      // the whole bin is kept (block-uniform)
                if (shift == 0) exact = true;
            }
        }
    }
    int32_t eq_before = 0;
    if (exact) {
        int32_t neq = 0;
        for (int32_t k = k0; k < k1; ++k) neq += (v[k] != -INFINITY && score_key(v[k]) == prefix);
        int32_t dummy;
        eq_before = block_exscan(neq, &dummy, L.wsum);
    }
    int32_t nsel = 0;
    {
        int32_t r = eq_before;
        for (int32_t k = k0; k < k1; ++k) {
            const float x = v[k];
            if (x == -INFINITY) continue;
            const uint32_t u = score_key(x);
            bool keep = all || (!exact && (u & mask) >= prefix) || (exact && u > prefix);
            if (exact && u == prefix) keep = r++ < rem;
            nsel += keep;
        }
    }
    int32_t n_kept;
    int32_t p = block_exscan(nsel, &n_kept, L.wsum);
    {
        int32_t r = eq_before;
        for (int32_t k = k0; k < k1; ++k) {
            const float x = v[k];
            if (x == -INFINITY) continue;
            const uint32_t u = score_key(x);
            bool keep = all || (!exact && (u & mask) >= prefix) || (exact && u > prefix);
            if (exact && u == prefix) keep = r++ < rem;
            if (keep) { out(p, s ? s[k] : s0 + k, x, an[k]); ++p; }
        }
    }
    __syncthreads();
    return n_kept;
}

// The beam of the step whose parts are stored at `parity`, into L.bs/bv/ba.
// States are clamped to [0, K) (they address rows of log A).
__device__ int32_t beam_rebuild(cargs_t& a, int32_t slot, int32_t parity) {
    BeamLds& L = g_lds.beam;
    const int tid = threadIdx.x;
    const int32_t W = a.bw, B = a.B, K = a.K;
    if (tid < W) L.pofs[tid + 1] = clampi(slot_part(a, slot, parity, tid).hdr[0], B + 1);
    if (tid == 0) L.pofs[0] = 0;
    __syncthreads();
    if (tid == 0)
        for (int32_t p = 1; p <= W; ++p) L.pofs[p] += L.pofs[p - 1];
    __syncthreads();
    for (int32_t p = 0; p < W; ++p) {
        const BeamRec rp = slot_part(a, slot, parity, p);
        const int32_t o = L.pofs[p], np = L.pofs[p + 1] - o;
        for (int32_t k = tid; k < np; k += kEngBlock) {
            L.cs[o + k] = clampi(rp.s[k], K);
            L.cv[o + k] = rp.v[k];
            L.ca[o + k] = rp.a[k];
        }
    }
    __syncthreads();
    return beam_select(L.pofs[W], B, L.cv, L.cs, 0, L.ca, [&](int32_t p, int32_t st, float sv, int32_t av) {
        L.bs[p] = st; L.bv[p] = sv; L.ba[p] = av;
    });
}

// Copies the rebuilt beam (L.bs/bv/ba, nb entries) to a record.
__device__ void beam_store(const BeamRec& rec, int32_t nb) {
    const BeamLds& L = g_lds.beam;
    for (int32_t k = threadIdx.x; k < nb; k += kEngBlock) {
        rec.s[k] = L.bs[k];
        rec.v[k] = L.bv[k];
        rec.a[k] = L.ba[k];
    }
    if (threadIdx.x == 0) rec.hdr[0] = nb;
}

// Position of state q in an LDS beam of nb entries sorted by state, or -1.
__device__ __forceinline__ int32_t beam_find_lds(const int32_t* bs, int32_t nb, int32_t q) {
    int32_t lo = 0, hi = nb;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (bs[mid] == q) return mid;
        if (bs[mid] < q) lo = mid + 1; else hi = mid;
    }
    return -1;
}

// Ascending bitonic sort of n2 (a power of two) keys in LDS by the block.
__device__ void lds_bitonic_sort(uint64_t* key, int32_t n2) {
    for (int32_t k = 2; k <= n2; k <<= 1) {
        for (int32_t h = k >> 1; h > 0; h >>= 1) {
            for (int32_t i = threadIdx.x; i < n2; i += kEngBlock) {
                const int32_t l = i ^ h;
                if (l > i) {
                    const uint64_t x = key[i], y = key[l];
                    if ((x > y) == ((i & k) == 0)) { key[i] = y; key[l] = x; }
                }
            }
            __syncthreads();
        }
    }
}

// Beam entry owning candidate position p: the b with offs[b] <= p < offs[b+1].
__device__ __forceinline__ int32_t sp_owner(const int32_t* offs, int32_t nb, int32_t p) {
    int32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (offs[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

// Clamped out-edge range [e0, e1) of source s.
__device__ __forceinline__ void sp_out_range(const int32_t* row_ptr, int64_t nnz, int32_t s, int32_t& e0,
                                             int32_t& e1) {
    int64_t x0 = row_ptr[s], x1 = row_ptr[s + 1];
    x0 = x0 < 0 ? 0 : (x0 > nnz ? nnz : x0);
    x1 = x1 < x0 ? x0 : (x1 > nnz ? nnz : x1);
    e0 = (int32_t)x0;
    e1 = (int32_t)x1;
}

// Sparse beam step (push): the candidates are the out-edges of the beam's
// states (L.bs/bv/ba, nb entries in state order), at positions in (beam
// entry, edge) order.  Sorting the keys (destination << 32 | position) puts
// each destination's candidates together in that order, so the first
// maximum of a run is the one the dense scan over the beam would keep.
// Writes the distinct destinations in state order to S.ds/dv/da with
// dv = c + log B_t(j) and the anchor chosen by mode (0 none, 1 the
// predecessor, 2 its anchor); returns their count.  More than kSpCandMax
// candidates: the sequence fails with FV_E_UNSUPPORTED (the first
// kSpCandMax are used, so every access stays in range).
// lb, ld, t: the emission data of the destinations' step.
__device__ int32_t sparse_push(cargs_t& a, SeqInfo& sq, int32_t nb, int32_t mode, const float* lb, int64_t ld,
                               int32_t t) {
    BeamLds& L = g_lds.beam;
    SpBeamLds& S = g_lds.spbeam;
    const int tid = threadIdx.x;
    const int32_t K = a.K;
    const int32_t per = (nb + kEngBlock - 1) / kEngBlock;
    const int32_t b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
    int32_t sum = 0;
    for (int32_t b = b0; b < b1; ++b) {
        int32_t e0, e1;
        sp_out_range(a.row_ptr, a.nnz, clampi(L.bs[b], K), e0, e1);
        S.estart[b] = e0;
        S.offs[b] = e1 - e0;   // degree for now
        sum += e1 - e0;
    }
    int32_t total;
    int32_t pos = block_exscan(sum, &total, L.wsum);
    for (int32_t b = b0; b < b1; ++b) {
        const int32_t d = S.offs[b];
        S.offs[b] = pos;
        pos += d;
    }
    if (tid == 0) S.offs[nb] = total;
    int32_t nc = total;
    if (nc > kSpCandMax) {
        if (tid == 0) {
            atomicOr(a.csr_flag, kCsrBeamCands);
            st_c(&sq.status, (int32_t)FV_E_UNSUPPORTED);
        }
        nc = kSpCandMax;
    }
    __syncthreads();
    int32_t n2 = 1;
    while (n2 < nc) n2 <<= 1;
    for (int32_t p = tid; p < n2; p += kEngBlock) {
        uint64_t k = ~0ull;
        if (p < nc) {
            const int32_t b = sp_owner(S.offs, nb, p);
            const int32_t e = S.estart[b] + (p - S.offs[b]);
            const int32_t j = a.col[e];
            S.cval[p] = L.bv[b] + a.val[e];
            if (j >= 0 && j < K) k = ((uint64_t)(uint32_t)j << 32) | (uint32_t)p;
        }
        S.key[p] = k;
    }
    __syncthreads();
    lds_bitonic_sort(S.key, n2);
    const int32_t per2 = (n2 + kEngBlock - 1) / kEngBlock;
    const int32_t k0 = min(n2, tid * per2), k1 = min(n2, k0 + per2);
    int32_t nh = 0;
    for (int32_t k = k0; k < k1; ++k) {
        const uint64_t x = S.key[k];
        nh += x != ~0ull && (k == 0 || (S.key[k - 1] >> 32) != (x >> 32));
    }
    int32_t nd;
    int32_t o = block_exscan(nh, &nd, L.wsum);
    for (int32_t k = k0; k < k1; ++k) {
        const uint64_t x = S.key[k];
        if (x == ~0ull || (k > 0 && (S.key[k - 1] >> 32) == (x >> 32))) continue;
        const uint32_t j = (uint32_t)(x >> 32);
        int32_t w = (int32_t)(uint32_t)x;
        float c = S.cval[w];
        for (int32_t u = k + 1; u < n2 && (uint32_t)(S.key[u] >> 32) == j; ++u) {
            const int32_t p = (int32_t)(uint32_t)S.key[u];
            const float y = S.cval[p];
            if (y > c) { c = y; w = p; }
        }
        const int32_t b = sp_owner(S.offs, nb, w);
        S.ds[o] = (int32_t)j;
        S.dv[o] = c + emission(a, lb, ld, t, (int32_t)j);
        S.da[o] = mode == 1 ? L.bs[b] : (mode == 2 ? L.ba[b] : -1);
        ++o;
    }
    __syncthreads();
    return nd;
}

__device__ __noinline__ void beam_chain_walk(cargs_t& a, const Row& r, int32_t q);

// One part of one beam task's step (parts beyond the first return at once
// for the single-block operations END and FINAL).
__device__ __noinline__ void beam_row(cargs_t& a_in, const float* __restrict__ Ap, const Row& r, int32_t part,
                                     int32_t W) {
    cargs_t& a = uniform_args(a_in);
    BeamLds& L = g_lds.beam;
    const int tid = threadIdx.x;
    SeqInfo& sq = a.seqs[r.seq];
    const int32_t K = a.K, Kp = a.Kp, B = a.B;
    gfloat_t* Ag = as_global(Ap);
    const int32_t slot = clampi(r.slot, a.n_slots);
    const bool root = r.kind == KIND_BROOT;
    // this step runs W of the a.bw parts; part 0 marks the other records of
    // the parity it writes empty, so the next rebuild merges W lists
    auto clear_unused = [&](int32_t parity) {
        if (part == 0 && tid >= W && tid < a.bw) slot_part(a, slot, parity, tid).hdr[0] = 0;
    };
    const int32_t T = r.T, pp = r.pp, m = r.m, n = r.n, t = r.t;
    const int32_t tmid = (m + n) >> 1;
    const int32_t jlo = part_lo(K, W, part), jhi = part_lo(K, W, part + 1), nj = jhi - jlo;
    if (r.aux == B_INIT) {
        // start step: pi + log B_0 at m = 0, the anchored boundary otherwise
        if (tid == 0) {
            L.misc[2] = m > 0 ? ld_c(sq.path + m - 1) : -1;
            L.misc[3] = m > 0 ? (int32_t)__float_as_uint(ld_cf(a.alpha_at + sq.alpha_off + m - 1)) : 0;
            if (part == 0) st_c(beam_fallback_flag(a, slot), 0);
        }
        __syncthreads();
        int32_t q = L.misc[2];
        const float alpha = __uint_as_float((uint32_t)L.misc[3]);
        if (q < 0 || q >= K) q = -1;
        const float* bm = r.log_b + (int64_t)m * r.ld;
        if (a.sparse) {   // one part
            const BeamRec out = slot_part(a, slot, m & 1, 0);
            int32_t nk = 0;
            if (m == 0) {
                // every state: chunks merged into a running top B (L.bs/bv/ba)
                for (int32_t c0 = 0; c0 < K; c0 += kBeamPartMax) {
                    const int32_t nc = min(kBeamPartMax, K - c0);
                    for (int32_t k = tid; k < nk; k += kEngBlock) {
                        L.cs[k] = L.bs[k]; L.cv[k] = L.bv[k]; L.ca[k] = L.ba[k];
                    }
                    for (int32_t k = tid; k < nc; k += kEngBlock) {
                        const int32_t j = c0 + k;
                        const float e = emission(a, r.log_b, r.ld, 0, j);
                        L.cs[nk + k] = j;
                        L.cv[nk + k] = a.log_pi ? a.log_pi[j] + e : e;
                        L.ca[nk + k] = -1;
                    }
                    __syncthreads();
                    nk = beam_select(nk + nc, B, L.cv, L.cs, 0, L.ca, [&](int32_t p, int32_t st, float sv, int32_t av) {
                        L.bs[p] = st; L.bv[p] = sv; L.ba[p] = av;
                    });
                }
                beam_store(out, nk);
            } else {
                // the boundary state alone, with its anchor score, pushed
                if (tid == 0) { L.bs[0] = q; L.bv[0] = alpha; L.ba[0] = -1; }
                __syncthreads();
                const SpBeamLds& S = g_lds.spbeam;
                const int32_t nd = q >= 0 ? sparse_push(a, sq, 1, 0, r.log_b, r.ld, m) : 0;
                nk = beam_select(nd, B, S.dv, S.ds, 0, S.da, [&](int32_t p, int32_t st, float sv, int32_t av) {
                    out.s[p] = st; out.v[p] = sv; out.a[p] = av;
                });
                if (tid == 0) out.hdr[0] = nk;
            }
            return;
        }
        for (int32_t k = tid; k < nj; k += kEngBlock) {
            const int32_t j = jlo + k;
            float v = -INFINITY;
            if (m == 0) v = a.log_pi ? a.log_pi[j] + bm[j] : bm[j];
            else if (q >= 0) {
                const float aq = Ap[(int64_t)q * Kp + j];
                const float c = a.relative_init ? aq : alpha + aq;
                v = c + bm[j];
            }
            L.sc[k] = v;
            L.an[k] = -1;
        }
        __syncthreads();
        const BeamRec out = slot_part(a, slot, m & 1, part);
        const int32_t nk = beam_select(nj, B, L.sc, nullptr, jlo, L.an, [&](int32_t p, int32_t st, float sv, int32_t av) {
            out.s[p] = st; out.v[p] = sv; out.a[p] = av;
        });
        if (tid == 0) out.hdr[0] = nk;
        clear_unused(m & 1);
    } else if (r.aux == B_STEP) {
        const int32_t nb = beam_rebuild(a, slot, (t - 1) & 1);
        if (part == 0) {
            // division / t_mid beams are taken from the rebuilt step t - 1
            if (root && pp >= 2) {
                const int32_t d = div_index(T, pp, t - 1);
                if (d >= 0) beam_store(root_beam(a, r.off, d), nb);
            }
            if (!root && t - 1 == tmid) beam_store(slot_snap_beam(a, slot), nb);
        }
        int32_t mode;  // anchor: 0 none, 1 the predecessor, 2 the predecessor's anchor
        if (root) {
            if (pp >= 2 && div_index(T, pp, t - 1) >= 0) mode = 1;
            else if (pp >= 2 && t > seg_end(T, pp, 0) + 1) mode = 2;
            else mode = 0;
        } else {
            mode = t == tmid + 1 ? 1 : (t > tmid + 1 ? 2 : 0);
        }
        const float* bt = r.log_b + (int64_t)t * r.ld;
        if (a.sparse) {
            const SpBeamLds& S = g_lds.spbeam;
            const int32_t nd = sparse_push(a, sq, nb, mode, r.log_b, r.ld, t);
            const BeamRec out = slot_part(a, slot, t & 1, 0);
            const int32_t nk = beam_select(nd, B, S.dv, S.ds, 0, S.da, [&](int32_t p, int32_t st, float sv, int32_t av) {
                out.s[p] = st; out.v[p] = sv; out.a[p] = av;
            });
            if (tid == 0) out.hdr[0] = nk;
            return;
        }
        for (int32_t k = tid; k < nj; k += kEngBlock) {
            const int32_t j = jlo + k;
            float c = -INFINITY;
            int32_t w = -1;
            // 16 loads in flight, then the candidates in beam order; a beam
            // entry's state and score are the same for every lane (scalars)
            for (int32_t b0 = 0; b0 < nb; b0 += 16) {
                float av[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int32_t sb = __builtin_amdgcn_readfirstlane(L.bs[min(b0 + u, nb - 1)]);
                    av[u] = Ag[(int64_t)sb * Kp + j];
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    if (b0 + u < nb) {
                        const float x = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                                            __builtin_bit_cast(int32_t, L.bv[b0 + u]))) + av[u];
                        if (w < 0 || x > c) { c = x; w = b0 + u; }
                    }
                }
            }
            L.sc[k] = w < 0 ? -INFINITY : c + bt[j];
            L.an[k] = w < 0 ? -1 : (mode == 1 ? L.bs[w] : (mode == 2 ? L.ba[w] : -1));
        }
        __syncthreads();
        const BeamRec out = slot_part(a, slot, t & 1, part);
        const int32_t nk = beam_select(nj, B, L.sc, nullptr, jlo, L.an, [&](int32_t p, int32_t st, float sv, int32_t av) {
            out.s[p] = st; out.v[p] = sv; out.a[p] = av;
        });
        if (tid == 0) out.hdr[0] = nk;
        clear_unused(t & 1);
    } else if (r.aux == B_END) {
        if (part != 0) return;
        // only the known end state q*_n is evaluated
        if (tid == 0) L.misc[4] = ld_c(&sq.status) < 0 ? -1 : ld_c(sq.path + n);
        __syncthreads();
        const int32_t qn = L.misc[4];
        __syncthreads();
        if (qn < 0 || qn >= K) return;
        const int32_t nb = beam_rebuild(a, slot, (n - 1) & 1);
        unsigned long long key = 0;
        for (int32_t b = tid; b < nb; b += kEngBlock) {
            float x = -INFINITY;
            if (a.sparse) {   // the edges s_b -> q*_n (the first maximum among duplicates)
                int32_t e0, e1;
                sp_out_range(a.row_ptr, a.nnz, L.bs[b], e0, e1);
                bool found = false;
                for (int32_t e = e0; e < e1; ++e) {
                    if (a.col[e] != qn) continue;
                    const float y = L.bv[b] + a.val[e];
                    if (!found || y > x) { x = y; found = true; }
                }
            } else {
                x = L.bv[b] + Ap[(int64_t)L.bs[b] * Kp + qn];
            }
            if (x != -INFINITY) {
                const unsigned long long k = order_key(x, b);
                if (k > key) key = k;
            }
        }
        unsigned long long kk = key;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(kk, off, 64);
            if (o > kk) kk = o;
        }
        if ((tid & 63) == 0) L.wkey[tid >> 6] = kk;
        __syncthreads();
        unsigned long long best = 0;
        for (int u = 0; u < kEngWaves; ++u) best = L.wkey[u] > best ? L.wkey[u] : best;
        __syncthreads();
        if (tid == 0) {
            if (best == 0) {
                // the beam lost q*_n: exact re-decode of this task
                st_c(beam_fallback_flag(a, slot), 1);
                if (ld_c(&sq.status) == FV_OK) st_c(&sq.status, (int32_t)FV_W_BEAM_FALLBACK);
            } else {
                const int32_t w = clampi((int32_t)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull)), nb);
                const int32_t qmid = (n == tmid + 1) ? L.bs[w] : L.ba[w];
                float amid = __builtin_nanf("");
                if (qmid >= 0 && qmid < K) {
                    if (n - 1 == tmid) {   // the t_mid beam is the one just rebuilt
                        const int32_t at = beam_find_lds(L.bs, nb, qmid);
                        if (at >= 0) amid = L.bv[at];
                    } else {
                        const BeamRec snap = slot_snap_beam(a, slot);
                        const int32_t ns = clampi(snap.hdr[0], B + 1);
                        int32_t lo = 0, hi = ns;
                        while (lo < hi) {
                            const int32_t mid = (lo + hi) >> 1;
                            const int32_t sm = snap.s[mid];
                            if (sm == qmid) { amid = snap.v[mid]; break; }
                            if (sm < qmid) lo = mid + 1; else hi = mid;
                        }
                    }
                }
                st_c(sq.path + tmid, qmid);
                st_cf(a.alpha_at + sq.alpha_off + tmid, amid);
            }
        }
    } else {  // B_FINAL: the root's best end state and the division chain
        if (part != 0) return;
        const int32_t nb = beam_rebuild(a, slot, (T - 1) & 1);
        if (nb == 0) {
            for (int32_t k = tid; k < T; k += kEngBlock) st_c(sq.path + k, -1);
            if (tid == 0) {
                st_cf(sq.score, -INFINITY);
                st_c(&sq.status, (int32_t)FV_E_INFEASIBLE);
            }
            return;
        }
        unsigned long long key = 0;
        for (int32_t k = tid; k < nb; k += kEngBlock) {
            const unsigned long long kk = order_key(L.bv[k], L.bs[k]);
            if (kk > key) key = kk;
        }
        const int32_t top_state = block_argmax_key(key);
        if (tid == 0) {
            const int32_t top = clampi(beam_find_lds(L.bs, nb, top_state), nb);
            st_c(sq.path + T - 1, top_state);
            L.misc[5] = L.ba[top];
        }
        __syncthreads();
        if (pp >= 2) beam_chain_walk(a, r, L.misc[5]);
    }
}

// Division chain of a finished beam root: q*_{e_d} for d = P'-2 .. 0, each
// found in the division's beam (state-sorted), whose score is the anchor
// alpha and whose anchor is the next state down.  Division records are
// copied to LDS in chunks (coalesced) and walked there.
__device__ __noinline__ void beam_chain_walk(cargs_t& a_in, const Row& r, int32_t q) {
    cargs_t& a = uniform_args(a_in);
    BeamLds& L = g_lds.beam;
    const int tid = threadIdx.x;
    SeqInfo& sq = a.seqs[r.seq];
    const int32_t K = a.K, B = a.B, T = r.T, pp = r.pp;
    int32_t* buf = L.cs;                        // L.cs, L.cv, L.ca: 3 * kBeamCandMax ints
    const int32_t stride = 1 + 3 * B;           // count, states, scores, anchors
    const int32_t per = max(1, (3 * kBeamCandMax) / stride);
    for (int32_t dhi = pp - 2; dhi >= 0; dhi -= per) {
        const int32_t dlo = max(0, dhi - per + 1);
        for (int32_t d = dlo; d <= dhi; ++d) {
            const BeamRec rs = root_beam(a, r.off, d);
            int32_t* dst = buf + (d - dlo) * stride;
            const int32_t n = clampi(rs.hdr[0], B + 1);
            if (tid == 0) dst[0] = n;
            for (int32_t k = tid; k < n; k += kEngBlock) {
                dst[1 + k] = rs.s[k];
                dst[1 + B + k] = __float_as_int(rs.v[k]);
                dst[1 + 2 * B + k] = rs.a[k];
            }
        }
        __syncthreads();
        if (tid == 0) {
            int32_t* const path = sq.path;   // (registers: see leaf_end)
            float* const alpha = a.alpha_at + sq.alpha_off;
            for (int32_t d = dhi; d >= dlo; --d) {
                const int32_t* rec = buf + (d - dlo) * stride;
                const int64_t e = seg_end(T, pp, d);
                st_cg(path + e, q);
                int32_t at = -1;
                for (int32_t lo = 0, hi = rec[0]; lo < hi;) {
                    const int32_t mid = (lo + hi) >> 1;
                    const int32_t sm = rec[1 + mid];
                    if (sm == q) { at = mid; break; }
                    if (sm < q) lo = mid + 1; else hi = mid;
                }
                st_cg(reinterpret_cast<uint32_t*>(alpha + e), at >= 0 ? (uint32_t)rec[1 + B + at] : 0x7fc00000u);
                if (d >= 1) q = (at >= 0 && q >= 0 && q < K) ? rec[1 + 2 * B + at] : -1;
            }
            L.misc[6] = q;
        }
        __syncthreads();
        q = L.misc[6];
        __syncthreads();
    }
}


// Finalize of a vanilla pass or a FLASH root (one block): the final state,
// the score, and for a root the division chain q*_{e_d} = Link_{d+1}(q*_{e_{d+1}})
// with the anchors alpha = Dsnap_d(q*_{e_d}).  Link rows are copied to LDS in
// chunks (coalesced) and the chain is walked there; the anchors are then
// gathered in parallel.
__device__ __noinline__ void dense_finalize(cargs_t& a_in, const Row& r) {
    cargs_t& a = uniform_args(a_in);
    EngineLds& lds = g_lds;
    const int tid = threadIdx.x;
    SeqInfo& sq = a.seqs[r.seq];
    const int32_t K = a.K, T = r.T, pp = r.pp;
    const int32_t slot = clampi(r.slot, a.n_slots);
    __shared__ int32_t sv[4];
    int32_t* buf = reinterpret_cast<int32_t*>(&lds);
    constexpr int32_t kBufInts = (int32_t)(sizeof(EngineLds) / 4);
    const bool coh = a.wide != 0;   // with wide rows the row data was written on other XCDs
    if (tid == 0) {
        const unsigned long long key = ld_c(a.keys + r.seq);
        const int32_t qT = clampi((int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull)), K);
        const float* dp = slot_delta(a, slot, (T - 1) & 1) + qT;
        const int32_t* ap = slot_anc(a, slot, (T - 1) & 1) + qT;
        const float sc = coh ? ld_cf(dp) : *dp;
        sv[0] = qT;
        sv[1] = __float_as_int(sc);
        sv[2] = (r.kind == KIND_ROOT && pp >= 2) ? clampi(coh ? ld_c(ap) : *ap, K) : -1;
    }
    __syncthreads();
    const int32_t qT = sv[0];
    const float sc = __int_as_float(sv[1]);
    int32_t q = sv[2];
    if (sc == -INFINITY) {
        for (int32_t t = tid; t < T; t += kEngBlock) st_c(sq.path + t, -1);
        if (tid == 0) {
            st_cf(sq.score, sc);
            st_c(&sq.status, (int32_t)FV_E_INFEASIBLE);
        }
        __syncthreads();
        return;
    }
    if (tid == 0) {
        st_cf(sq.score, sc);
        st_c(sq.path + T - 1, qT);
    }
    if (r.kind != KIND_ROOT || pp < 2) {
        __syncthreads();
        return;
    }
    if (K > kBufInts) {   // a link row does not fit in LDS: walk in global memory
        if (tid == 0) {
            int32_t* const path = sq.path;   // (a register: see leaf_end)
            for (int32_t d = pp - 2; d >= 0; --d) {
                st_cg(path + seg_end(T, pp, d), q);
                const int32_t* lp = root_link(a, r.off, pp, d) + q;
                if (d >= 1) q = clampi(coh ? ld_c(lp) : *lp, K);
            }
        }
        __syncthreads();
    }
    const int32_t per = max(1, kBufInts / K);
    for (int32_t dhi = K > kBufInts ? -1 : pp - 2; dhi >= 0; dhi -= per) {
        const int32_t dlo = max(0, dhi - per + 1);
        const int32_t l0 = max(dlo, 1);   // Link_0 is never followed
        const int32_t n = (dhi - l0 + 1) * K;
        for (int32_t idx = tid; idx < n; idx += kEngBlock) {
            const int32_t d = l0 + idx / K, j = idx % K;
            const int32_t* lp = root_link(a, r.off, pp, d) + j;
            buf[(d - dlo) * K + j] = coh ? ld_c(lp) : *lp;
        }
        __syncthreads();
        if (tid == 0) {
            int32_t* const path = sq.path;   // (a register: see leaf_end)
            for (int32_t d = dhi; d >= dlo; --d) {
                st_cg(path + seg_end(T, pp, d), q);
                if (d >= 1) q = clampi(buf[(d - dlo) * K + q], K);
            }
            sv[3] = q;
        }
        __syncthreads();
        q = sv[3];
        __syncthreads();
    }
    for (int32_t d = tid; d <= pp - 2; d += kEngBlock) {
        const int64_t e = seg_end(T, pp, d);
        const int32_t qd = clampi(ld_c(sq.path + e), K);
        const float* dp = root_dsnap(a, r.off, d) + qd;
        st_cf(a.alpha_at + sq.alpha_off + e, coh ? ld_cf(dp) : *dp);
    }
    __syncthreads();
}

// End of a leaf subtask (one block): the end-only step at the known end
// state q*_n gives q*_{n-1} (first maximum of delta_{n-1}(i) + log A(i, q*_n),
// lowest i on ties), then the leaf's backpointer rows are walked back,
// q*_{t-1} = psi_t(q*_t) for t = n-1 .. m+1.  Table rows are copied to LDS in
// chunks (16-byte loads) and walked there by one thread.
__device__ __noinline__ void leaf_end(cargs_t& a_in, const Row& r) {
    cargs_t& a = uniform_args(a_in);
    const int tid = threadIdx.x;
    SeqInfo& sq = a.seqs[r.seq];
    const int32_t K = a.K, Kp = a.Kp, m = r.m, n = r.n;
    const int32_t slot = clampi(r.slot, a.n_slots);
    __shared__ int32_t lv[2];
    if (tid == 0) lv[0] = ld_c(&sq.status) < 0 ? -1 : ld_c(sq.path + n);
    __syncthreads();
    const int32_t qn = lv[0];
    __syncthreads();
    if (qn < 0 || qn >= K) return;
    const float* dprev = slot_delta(a, slot, (n - 1) & 1);
    const float* ac = a.Acol + qn;
    unsigned long long key = 0;
    for (int32_t i = tid; i < K; i += kEngBlock) {
        const unsigned long long k = order_key(dprev[i] + ac[(int64_t)i * Kp], i);
        if (k > key) key = k;
    }
    int32_t q = clampi(block_argmax_key(key), K);
    if (tid == 0) st_c(sq.path + n - 1, q);
    uint4* buf = reinterpret_cast<uint4*>(&g_lds);
    constexpr int32_t kBufU16 = (int32_t)(sizeof(EngineLds) / 16) * 8;
    const int32_t per = max(1, kBufU16 / Kp);   // table rows per chunk
    const uint16_t* tab = slot_leaf(a, slot);
    for (int32_t hi = n - 1; hi >= m + 1; hi -= per) {   // table rows of t in [lo, hi]
        const int32_t lo = max(m + 1, hi - per + 1);
        const int32_t n16 = (hi - lo + 1) * Kp / 8;      // Kp is a multiple of 64
        const uint4* src = reinterpret_cast<const uint4*>(tab + (int64_t)(lo - m) * Kp);
        for (int32_t k0 = tid; k0 < n16; k0 += kEngBlock * 8) {
            // eight loads in flight per thread (indices past the chunk re-read
            // its last entry, and are not stored)
            uint4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src[min(k0 + u * kEngBlock, n16 - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t k = k0 + u * kEngBlock;
                if (k < n16) buf[k] = v[u];
            }
        }
        __syncthreads();
        if (tid == 0) {
            // the path pointer in a register: read from the sequence record
            // inside the loop, it would be reloaded (and waited for) after
            // every store, which might alias it
            int32_t* const path = sq.path;
            const uint16_t* b16 = reinterpret_cast<const uint16_t*>(buf);
            for (int32_t t = hi; t >= lo; --t) {
                q = clampi(b16[(int64_t)(t - lo) * Kp + q], K);
                st_cg(path + t - 1, q);
            }
            lv[1] = q;
        }
        __syncthreads();
        q = lv[1];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- grouped beam rows
// The same operations as beam_row (dense model, one part), computed by one
// 256-thread group with barriers among its 4 waves (LDS arrival counters).
__device__ __forceinline__ int32_t q_grp() { return threadIdx.x / kQThreads; }
__device__ __forceinline__ int32_t q_tid() { return threadIdx.x % kQThreads; }
__device__ __forceinline__ void q_sync() { group_sync(&g_lds.qbeam.gsync[q_grp()], kQWaves); }

// Exclusive prefix sum of one int per thread over the group; *total = the sum.
__device__ int32_t q_exscan(int32_t v, int32_t* total, int32_t* wsum) {
    const int lane = threadIdx.x & 63, w = q_tid() >> 6;
    int32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    q_sync();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int u = 0; u < kQWaves; ++u) {
        const int32_t y = wsum[u];
        if (u < w) before += y;
        all += y;
    }
    q_sync();
    *total = all;
    return before + x - v;
}

// The index held in the largest key over the group (keys: 0 = none).
__device__ int32_t q_argmax_key(QBeamLds& L, unsigned long long key) {
    const int lane = threadIdx.x & 63, w = q_tid() >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        if (o > key) key = o;
    }
    if (lane == 0) L.wkey[w] = key;
    q_sync();
    unsigned long long best = 0;
    for (int u = 0; u < kQWaves; ++u) best = L.wkey[u] > best ? L.wkey[u] : best;
    q_sync();
    return (int32_t)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull));
}

// beam_select for one group: top B of n entries in state order by (score
// desc, state asc), -inf dropped; out(p, state, score, anchor) in state order.
template <typename Out>
__device__ int32_t q_select(QBeamLds& L, int32_t n, int32_t B, const float* v, const int32_t* s, int32_t s0,
                            const int32_t* an, Out out) {
    const int tid = q_tid(), lane = threadIdx.x & 63, wv = tid >> 6;
    const int32_t per = (n + kQThreads - 1) / kQThreads;
    const int32_t k0 = min(n, tid * per), k1 = min(n, k0 + per);
    // finite entries, and the bits all their keys share (AND and OR of the keys)
    int32_t nfin = 0;
    uint32_t kand = 0xffffffffu, kor = 0u;
    for (int32_t k = k0; k < k1; ++k) {
        if (v[k] == -INFINITY) continue;
        const uint32_t u = score_key(v[k]);
        ++nfin;
        kand &= u;
        kor |= u;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        kand &= (uint32_t)__shfl_xor((int32_t)kand, off, 64);
        kor |= (uint32_t)__shfl_xor((int32_t)kor, off, 64);
    }
    if (lane == 0) L.wkey[wv] = ((unsigned long long)kand << 32) | kor;
    int32_t n_finite;
    q_exscan(nfin, &n_finite, L.wsum);   // (its barriers also publish wkey)
    const bool all = n_finite <= B;
    // The threshold: radix passes of 8 bits over the keys, from the highest
    // byte in which the finite keys differ (the bytes above are common, so
    // their passes would keep every entry).  A pass whose chosen bin holds
    // exactly the entries still needed ends the search: the whole bin is
    // kept.  Otherwise the last pass leaves the exact B-th key, whose equal
    // entries are taken in index order.
    uint32_t prefix = 0, mask = 0;
    int32_t rem = B;
    bool exact = false;
    if (!all) {
        uint32_t gand = 0xffffffffu, gor = 0u;
#pragma unroll
        for (int u = 0; u < kQWaves; ++u) {
            gand &= (uint32_t)(L.wkey[u] >> 32);
            gor |= (uint32_t)L.wkey[u];
        }
        const uint32_t diff = gand ^ gor;
        if (diff == 0u) {   // every finite key equal: the first B in index order
            prefix = gor;
            mask = 0xffffffffu;
            exact = true;
        } else {
            const int32_t hb = 31 - __builtin_clz(diff);
            const int32_t sh0 = (hb >> 3) << 3;
            mask = sh0 >= 24 ? 0u : ~((1u << (sh0 + 8)) - 1u);
            prefix = gor & mask;
            for (int shift = sh0; shift >= 0; shift -= 8) {
                for (int k = tid; k < 256; k += kQThreads) L.hist[k] = 0;
                q_sync();
                for (int32_t k = k0; k < k1; ++k) {
                    const float x = v[k];
                    if (x == -INFINITY) continue;
                    const uint32_t u = score_key(x);
                    if ((u & mask) == prefix) atomicAdd(&L.hist[(u >> shift) & 255u], 1u);
                }
                q_sync();
                if (tid < 64) {
                    int32_t c[4];
#pragma unroll
                    for (int d = 0; d < 4; ++d) c[d] = (int32_t)L.hist[4 * tid + d];
                    const int32_t own = c[0] + c[1] + c[2] + c[3];
                    int32_t incl = own;   // sum over lanes >= tid
#pragma unroll
                    for (int off = 1; off < 64; off <<= 1) {
                        const int32_t y = __shfl_down(incl, off, 64);
                        if (tid + off < 64) incl += y;
                    }
                    int32_t above = incl - own;
                    for (int d = 3; d >= 0; --d) {
                        if (above < rem && above + c[d] >= rem) {
                            L.misc[0] = 4 * tid + d;
                            L.misc[1] = rem - above;
                            L.misc[2] = c[d];
                        }
                        above += c[d];
                    }
                }
                q_sync();
                prefix |= (uint32_t)L.misc[0] << shift;
                mask |= 255u << shift;
                rem = L.misc[1];
                const int32_t cbin = L.misc[2];
                q_sync();
                if (cbin == rem) break;      // the whole bin is kept (group-uniform)
                if (shift == 0) exact = true;
            }
        }
    }
    // keep: everything (all), a masked key at or above the threshold's bits
    // (a search ended on a whole bin), or a key above the exact threshold
    // plus its first rem equal entries in index order
    int32_t eq_before = 0;
    if (exact) {
        int32_t neq = 0;
        for (int32_t k = k0; k < k1; ++k) neq += (v[k] != -INFINITY && score_key(v[k]) == prefix);
        int32_t dummy;
        eq_before = q_exscan(neq, &dummy, L.wsum);
    }
    int32_t nsel = 0;
    {
        int32_t r = eq_before;
        for (int32_t k = k0; k < k1; ++k) {
            const float x = v[k];
            if (x == -INFINITY) continue;
            const uint32_t u = score_key(x);
            bool keep = all || (!exact && (u & mask) >= prefix) || (exact && u > prefix);
            if (exact && u == prefix) keep = r++ < rem;
            nsel += keep;
        }
    }
    int32_t n_kept;
    int32_t p = q_exscan(nsel, &n_kept, L.wsum);
    {
        int32_t r = eq_before;
        for (int32_t k = k0; k < k1; ++k) {
            const float x = v[k];
            if (x == -INFINITY) continue;
            const uint32_t u = score_key(x);
            bool keep = all || (!exact && (u & mask) >= prefix) || (exact && u > prefix);
            if (exact && u == prefix) keep = r++ < rem;
            if (keep) { out(p, s ? s[k] : s0 + k, x, an[k]); ++p; }
        }
    }
    q_sync();
    return n_kept;
}

// The beam of the step stored at `parity` (one part) into L.bs/bv/ba.
__device__ int32_t q_rebuild(cargs_t& a, QBeamLds& L, int32_t slot, int32_t parity) {
    const int tid = q_tid();
    const int32_t B = a.B, K = a.K;
    const BeamRec rp = slot_part(a, slot, parity, 0);
    // the count and the first B entries are read together (B <= the group's
    // threads; entries past the count are read but not used)
    int32_t es = 0, ea = 0;
    float ev = 0.0f;
    if (tid < B) { es = rp.s[tid]; ev = rp.v[tid]; ea = rp.a[tid]; }
    const int32_t np = clampi(rp.hdr[0], B + 1);
    if (np <= B) {
        // a record of this group's kind is already the beam: at most B finite
        // entries in state order (the selection that wrote it dropped -inf)
        if (tid < np) {
            L.bs[tid] = clampi(es, K);
            L.bv[tid] = ev;
            L.ba[tid] = ea;
        }
        q_sync();
        return np;
    }
    for (int32_t k = tid; k < np; k += kQThreads) {
        L.cs[k] = clampi(rp.s[k], K);
        L.cv[k] = rp.v[k];
        L.ca[k] = rp.a[k];
    }
    q_sync();
    return q_select(L, np, B, L.cv, L.cs, 0, L.ca, [&](int32_t p, int32_t st, float sv, int32_t av) {
        L.bs[p] = st; L.bv[p] = sv; L.ba[p] = av;
    });
}

__device__ void q_store(const QBeamLds& L, const BeamRec& rec, int32_t nb) {
    for (int32_t k = q_tid(); k < nb; k += kQThreads) {
        rec.s[k] = L.bs[k];
        rec.v[k] = L.bv[k];
        rec.a[k] = L.ba[k];
    }
    if (q_tid() == 0) rec.hdr[0] = nb;
}

// Division chain of a finished beam root (beam_chain_walk for one group; the
// score/anchor area holds the records).
__device__ void q_chain_walk(cargs_t& a, QBeamLds& L, const Row& r, int32_t q) {
    const int tid = q_tid();
    SeqInfo& sq = a.seqs[r.seq];
    const int32_t K = a.K, B = a.B, T = r.T, pp = r.pp;
    int32_t* buf = reinterpret_cast<int32_t*>(L.sc);   // sc and an: 2 * kQK ints
    const int32_t stride = 1 + 3 * B;
    const int32_t per = max(1, (2 * kQK) / stride);
    for (int32_t dhi = pp - 2; dhi >= 0; dhi -= per) {
        const int32_t dlo = max(0, dhi - per + 1);
        for (int32_t d = dlo; d <= dhi; ++d) {
            const BeamRec rs = root_beam(a, r.off, d);
            int32_t* dst = buf + (d - dlo) * stride;
            const int32_t n = clampi(rs.hdr[0], B + 1);
            if (tid == 0) dst[0] = n;
            for (int32_t k = tid; k < n; k += kQThreads) {
                dst[1 + k] = rs.s[k];
                dst[1 + B + k] = __float_as_int(rs.v[k]);
                dst[1 + 2 * B + k] = rs.a[k];
            }
        }
        q_sync();
        if (tid == 0) {
            int32_t* const path = sq.path;   // (registers: see leaf_end)
            float* const alpha = a.alpha_at + sq.alpha_off;
            for (int32_t d = dhi; d >= dlo; --d) {
                const int32_t* rec = buf + (d - dlo) * stride;
                const int64_t e = seg_end(T, pp, d);
                st_cg(path + e, q);
                int32_t at = -1;
                for (int32_t lo = 0, hi = rec[0]; lo < hi;) {
                    const int32_t mid = (lo + hi) >> 1;
                    const int32_t sm = rec[1 + mid];
                    if (sm == q) { at = mid; break; }
                    if (sm < q) lo = mid + 1; else hi = mid;
                }
                st_cg(reinterpret_cast<uint32_t*>(alpha + e), at >= 0 ? (uint32_t)rec[1 + B + at] : 0x7fc00000u);
                if (d >= 1) q = (at >= 0 && q >= 0 && q < K) ? rec[1 + 2 * B + at] : -1;
            }
            L.misc[6] = q;
        }
        q_sync();
        q = L.misc[6];
        q_sync();
    }
}

// One beam task step (dense model, one part) by this thread's group.
__device__ __noinline__ void beam_row_q(cargs_t& a_in, const Row& r) {
    cargs_t& a = uniform_args(a_in);
    const float* __restrict__ Ap = a.Acol;
    QBeamLds& L = g_lds.qbeam.g[q_grp()];
    const int tid = q_tid();
    SeqInfo& sq = a.seqs[r.seq];
    const int32_t K = a.K, Kp = a.Kp, B = a.B;
    gfloat_t* Ag = as_global(Ap);
    const int32_t slot = clampi(r.slot, a.n_slots);
    const bool root = r.kind == KIND_BROOT;
    const int32_t T = r.T, pp = r.pp, m = r.m, n = r.n, t = r.t;
    const int32_t tmid = (m + n) >> 1;
    if (r.aux == B_INIT) {
        if (tid == 0) {
            L.misc[2] = m > 0 ? ld_c(sq.path + m - 1) : -1;
            L.misc[3] = m > 0 ? (int32_t)__float_as_uint(ld_cf(a.alpha_at + sq.alpha_off + m - 1)) : 0;
            st_c(beam_fallback_flag(a, slot), 0);
        }
        q_sync();
        int32_t q = L.misc[2];
        const float alpha = __uint_as_float((uint32_t)L.misc[3]);
        if (q < 0 || q >= K) q = -1;
        const float* bm = r.log_b + (int64_t)m * r.ld;
        for (int32_t j = tid; j < K; j += kQThreads) {
            float v = -INFINITY;
            if (m == 0) v = a.log_pi ? a.log_pi[j] + bm[j] : bm[j];
            else if (q >= 0) {
                const float aq = Ap[(int64_t)q * Kp + j];
                const float c = a.relative_init ? aq : alpha + aq;
                v = c + bm[j];
            }
            L.sc[j] = v;
            L.an[j] = -1;
        }
        q_sync();
        const BeamRec out = slot_part(a, slot, m & 1, 0);
        const int32_t nk = q_select(L, K, B, L.sc, nullptr, 0, L.an, [&](int32_t p, int32_t st, float sv, int32_t av) {
            out.s[p] = st; out.v[p] = sv; out.a[p] = av;
        });
        if (tid == 0) out.hdr[0] = nk;
    } else if (r.aux == B_STEP) {
        const int32_t nb = q_rebuild(a, L, slot, (t - 1) & 1);
        if (root && pp >= 2) {
            const int32_t d = div_index(T, pp, t - 1);
            if (d >= 0) q_store(L, root_beam(a, r.off, d), nb);
        }
        if (!root && t - 1 == tmid) q_store(L, slot_snap_beam(a, slot), nb);
        int32_t mode;  // anchor: 0 none, 1 the predecessor, 2 the predecessor's anchor
        if (root) {
            if (pp >= 2 && div_index(T, pp, t - 1) >= 0) mode = 1;
            else if (pp >= 2 && t > seg_end(T, pp, 0) + 1) mode = 2;
            else mode = 0;
        } else {
            mode = t == tmid + 1 ? 1 : (t > tmid + 1 ? 2 : 0);
        }
        gfloat_t* bt = as_global(r.log_b) + (int64_t)t * r.ld;
        // four consecutive destinations per thread (j0 .. j0 + 3), read as
        // one 16-byte load per beam state: Kp is a multiple of 64, so the
        // load stays inside the (padded) row; the loads of 16 beam states are
        // in flight together
        constexpr int32_t kJ = 4;
        typedef float v4f_t __attribute__((ext_vector_type(4), aligned(4)));
        typedef __attribute__((address_space(1))) const v4f_t gv4f_t;
        for (int32_t j0 = kJ * tid; j0 < K; j0 += kQThreads * kJ) {
            float c[kJ];
            int32_t w[kJ];
#pragma unroll
            for (int jj = 0; jj < kJ; ++jj) { c[jj] = -INFINITY; w[jj] = -1; }
            for (int32_t b0 = 0; b0 < nb; b0 += 16) {
                v4f_t av[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int32_t sb = __builtin_amdgcn_readfirstlane(L.bs[min(b0 + u, nb - 1)]);
                    av[u] = *reinterpret_cast<gv4f_t*>(Ag + (int64_t)sb * Kp + j0);
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    if (b0 + u < nb) {
                        const float bvu = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                                              __builtin_bit_cast(int32_t, L.bv[b0 + u])));
#pragma unroll
                        for (int jj = 0; jj < kJ; ++jj) {
                            const float x = bvu + av[u][jj];
                            if (w[jj] < 0 || x > c[jj]) { c[jj] = x; w[jj] = b0 + u; }
                        }
                    }
                }
            }
#pragma unroll
            for (int jj = 0; jj < kJ; ++jj) {
                const int32_t j = j0 + jj;
                if (j < K) {
                    L.sc[j] = w[jj] < 0 ? -INFINITY : c[jj] + bt[j];
                    L.an[j] = w[jj] < 0 ? -1 : (mode == 1 ? L.bs[w[jj]] : (mode == 2 ? L.ba[w[jj]] : -1));
                }
            }
        }
        q_sync();
        const BeamRec out = slot_part(a, slot, t & 1, 0);
        const int32_t nk = q_select(L, K, B, L.sc, nullptr, 0, L.an, [&](int32_t p, int32_t st, float sv, int32_t av) {
            out.s[p] = st; out.v[p] = sv; out.a[p] = av;
        });
        if (tid == 0) out.hdr[0] = nk;
    } else if (r.aux == B_END) {
        if (tid == 0) L.misc[4] = ld_c(&sq.status) < 0 ? -1 : ld_c(sq.path + n);
        q_sync();
        const int32_t qn = L.misc[4];
        q_sync();
        if (qn < 0 || qn >= K) return;
        const int32_t nb = q_rebuild(a, L, slot, (n - 1) & 1);
        unsigned long long key = 0;
        for (int32_t b = tid; b < nb; b += kQThreads) {
            const float x = L.bv[b] + Ap[(int64_t)L.bs[b] * Kp + qn];
            if (x != -INFINITY) {
                const unsigned long long k = order_key(x, b);
                if (k > key) key = k;
            }
        }
        const int32_t wb = q_argmax_key(L, key);   // 0xFFFFFFFF - 0 when no key: no beam state reaches q*_n
        if (tid == 0) {
            if (wb < 0 || wb >= nb) {
                st_c(beam_fallback_flag(a, slot), 1);
                if (ld_c(&sq.status) == FV_OK) st_c(&sq.status, (int32_t)FV_W_BEAM_FALLBACK);
            } else {
                const int32_t qmid = (n == tmid + 1) ? L.bs[wb] : L.ba[wb];
                float amid = __builtin_nanf("");
                if (qmid >= 0 && qmid < K) {
                    if (n - 1 == tmid) {
                        const int32_t at = beam_find_lds(L.bs, nb, qmid);
                        if (at >= 0) amid = L.bv[at];
                    } else {
                        const BeamRec snap = slot_snap_beam(a, slot);
                        const int32_t ns = clampi(snap.hdr[0], B + 1);
                        int32_t lo = 0, hi = ns;
                        while (lo < hi) {
                            const int32_t mid = (lo + hi) >> 1;
                            const int32_t sm = snap.s[mid];
                            if (sm == qmid) { amid = snap.v[mid]; break; }
                            if (sm < qmid) lo = mid + 1; else hi = mid;
                        }
                    }
                }
                st_c(sq.path + tmid, qmid);
                st_cf(a.alpha_at + sq.alpha_off + tmid, amid);
            }
        }
    } else {  // B_FINAL
        const int32_t nb = q_rebuild(a, L, slot, (T - 1) & 1);
        if (nb == 0) {
            for (int32_t k = tid; k < T; k += kQThreads) st_c(sq.path + k, -1);
            if (tid == 0) {
                st_cf(sq.score, -INFINITY);
                st_c(&sq.status, (int32_t)FV_E_INFEASIBLE);
            }
            return;
        }
        unsigned long long key = 0;
        for (int32_t k = tid; k < nb; k += kQThreads) {
            const unsigned long long kk = order_key(L.bv[k], L.bs[k]);
            if (kk > key) key = kk;
        }
        const int32_t top_state = q_argmax_key(L, key);
        if (tid == 0) {
            const int32_t top = clampi(beam_find_lds(L.bs, nb, top_state), nb);
            st_c(sq.path + T - 1, top_state);
            L.misc[5] = L.ba[top];
        }
        q_sync();
        if (pp >= 2) q_chain_walk(a, L, r, L.misc[5]);
    }
}

// ---------------------------------------------------------------- scheduler
// What a row of step s turns into at step s+1 (its XCD never changes).
struct Next {
    int32_t list;   // -1: none, else the list of the successor row (0 full, 1 light, 2 beam)
    int32_t freed, spawn;
    Row row;
};

__device__ int32_t root_segments(int32_t T, int32_t pp) {
    int32_t c = 0;
    for (int32_t d = 0; d < pp; ++d) {
        const int64_t m = d == 0 ? 0 : seg_end(T, pp, d - 1) + 1, n = seg_end(T, pp, d);
        if (n - m >= 1) ++c;
    }
    return c;
}

__device__ __forceinline__ int32_t child_count(const Row& r) {
    const int32_t len = r.n - r.m;
    return len > 2 ? 2 : (len == 2 ? 1 : 0);
}

// Children of a w-way subtask: its segments of at least two positions.
__device__ __forceinline__ int32_t wchild_count(const Row& r, int32_t wsplit) {
    const int32_t L = r.n - r.m + 1, wp = sub_parts(r.m, r.n, wsplit);
    int32_t c = 0, lo = 0;
    for (int32_t k = 0; k < wp; ++k) {
        const int32_t hi = k < wp - 1 ? (int32_t)seg_end(L, wp, k) : L - 1;
        c += hi - lo >= 1;
        lo = hi + 1;
    }
    return c;
}

// src: the list r came from (0 full, 1 light, 2 block rows: beam tasks and
// the finalize of dense roots and vanilla passes).
__device__ Next classify(cargs_t& a, const Row& r, int src) {
    Next x;
    x.list = -1;
    x.freed = x.spawn = 0;
    const int32_t T = r.T, pp = r.pp;
    if (src == 2 && !is_beam(r.kind)) {  // finalize of a vanilla pass or FLASH root, or a leaf's end
        x.freed = 1;
        if (r.kind == KIND_ROOT && pp >= 2) x.spawn = root_segments(T, pp);
        return x;
    }
    if (src == 2) {
        const bool root = r.kind == KIND_BROOT;
        if (r.aux == B_INIT || r.aux == B_STEP) {
            const int32_t nt = r.t + 1;
            x.list = 2;
            if (root) x.row = nt < T ? make_beam_row(r, nt, B_STEP) : make_beam_row(r, T, B_FINAL);
            else x.row = nt < r.n ? make_beam_row(r, nt, B_STEP) : make_beam_row(r, r.n, B_END);
        } else if (r.aux == B_END) {
            // its fallback flag is written while this runs: decide next step
            x.list = 1;
            x.row = make_light_row(r, r.n, L_BSPAWN);
        } else {  // B_FINAL
            x.freed = 1;
            if (pp >= 2) x.spawn = root_segments(T, pp);
        }
        return x;
    }
    const bool sub = is_dense_sub(r.kind);
    if (src == 0 || r.aux == L_INIT) {
        const int32_t nt = src == 0 ? r.t + 1 : r.m + 1;
        if (sub) {
            const bool leaf = is_leaf(a, r.kind, r.m, r.n);
            if (nt < r.n) { x.list = 0; x.row = make_dense_row(r, nt, leaf, a.wsplit); }
            else if (leaf) { x.list = 2; x.row = make_light_row(r, r.n, L_LEAF_END, true); }
            else { x.list = 1; x.row = make_light_row(r, r.n, L_END); }
        } else {
            if (nt < T) { x.list = 0; x.row = make_dense_row(r, nt, false); }
            else { x.list = 2; x.row = make_light_row(r, T, L_FINALIZE); }
        }
    } else if (r.aux == L_END) {
        x.freed = 1;
        x.spawn = (r.kind == KIND_SUB && a.wsplit > 2) ? wchild_count(r, a.wsplit) : child_count(r);
    } else {  // L_BSPAWN
        x.freed = 1;
        x.spawn = ld_c(beam_fallback_flag(a, clampi(r.slot, a.n_slots))) ? 1 : child_count(r);
    }
    return x;
}

// Children per Alg. 1 (end of a subtask), the P'-way segments of a finished
// root, or the exact re-decode of a beam subtask that lost its end state.
__device__ void write_spawns(cargs_t& a, const Row& r, int src, int64_t pos) {
    const bool beam_end = src == 1 && r.aux == L_BSPAWN;
    if (beam_end || (src == 1 && r.aux == L_END)) {
        if (beam_end && ld_c(beam_fallback_flag(a, clampi(r.slot, a.n_slots)))) {
            a.queue[pos] = Task{r.seq, KIND_FSUB, r.m, r.n};
            return;
        }
        const int32_t kind = (beam_end || r.kind == KIND_FSUB) ? KIND_BSUB : KIND_SUB;
        if (!beam_end && r.kind == KIND_SUB && a.wsplit > 2) {
            const int32_t L = r.n - r.m + 1, wp = sub_parts(r.m, r.n, a.wsplit);
            int32_t lo = 0;
            for (int32_t k = 0; k < wp; ++k) {
                const int32_t hi = k < wp - 1 ? (int32_t)seg_end(L, wp, k) : L - 1;
                if (hi - lo >= 1) a.queue[pos++] = Task{r.seq, KIND_SUB, r.m + lo, r.m + hi};
                lo = hi + 1;
            }
            return;
        }
        const int32_t tmid = (r.m + r.n) >> 1;
        const int32_t len = r.n - r.m;
        if (len >= 2) a.queue[pos++] = Task{r.seq, kind, r.m, tmid};
        if (len > 2) a.queue[pos++] = Task{r.seq, kind, tmid + 1, r.n};
    } else {
        const int32_t kind = is_beam(r.kind) ? KIND_BSUB : KIND_SUB;
        const int32_t T = r.T, pp = r.pp;
        for (int32_t d = 0; d < pp; ++d) {
            const int64_t m = d == 0 ? 0 : seg_end(T, pp, d - 1) + 1, n = seg_end(T, pp, d);
            if (n - m >= 1) a.queue[pos++] = Task{r.seq, kind, (int32_t)m, (int32_t)n};
        }
    }
}

// The scheduler block splits into kXcd groups of 128 threads; group x
// handles the rows of XCD x.  Its state lives in LDS.


// Exclusive scan of N counters over the 128 threads of a scheduler group.
template <int N>
__device__ void group_scan(int32_t (&v)[N], int32_t (&tot)[N], int32_t (&ws)[kSchedGroupWaves][5]) {
    const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) % kSchedGroupWaves;
    int32_t inc[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int32_t x = v[k];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        inc[k] = x;
        if (lane == 63) ws[w][k] = x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int32_t before = 0, all = 0;
#pragma unroll
        for (int u = 0; u < kSchedGroupWaves; ++u) {
            const int32_t y = ws[u][k];
            if (u < w) before += y;
            all += y;
        }
        tot[k] = all;
        v[k] = before + inc[k] - v[k];
    }
    __syncthreads();
}

// Admit queued tasks to the free slots of the XCDs that have compute
// blocks, in proportion to their free slots, and write their start rows
// (beam tasks to the beam list, the others to the light list).  Called by
// the whole scheduler block; sl.n_next holds the rows already written for
// step nxt.
__device__ __noinline__ void admit(cargs_t& a_in, int nxt, uint32_t tag) {
    cargs_t& a = uniform_args(a_in);
    SchedLds& sl = g_sched;
    if (threadIdx.x == 0) {
        // water filling: XCD x gets rows up to level L * nblk[x] (its share of
        // the compute blocks), at most its free slots; L is the lowest level
        // (in 1/16 rows per block) that places every admissible task
        int32_t load[kXcd], cap[kXcd], cap_total = 0;
        for (int y = 0; y < kXcd; ++y) {
            load[y] = sl.n_next[y][0] + sl.n_next[y][1] + sl.n_next[y][2];
            cap[y] = sl.nblk[y] > 0 ? sl.n_free[y] : 0;
            cap_total += cap[y];
        }
        const int32_t n_admit = min(cap_total, sl.q_tail - sl.q_head);
        // level in 1/16 rows per block; 32-bit arithmetic, shifts only
        auto placed = [&](int32_t L16, int y) -> int32_t {
            const int32_t want = ((L16 * sl.nblk[y]) >> 4) - load[y];
            return want < 0 ? 0 : (want > cap[y] ? cap[y] : want);
        };
        int32_t max_load = 0;
        for (int y = 0; y < kXcd; ++y) max_load = max(max_load, load[y]);
        // at this level every XCD with blocks wants at least max_load + n_admit rows
        int32_t lo = 0, hi = ((max_load + n_admit) << 4) + 16;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            int32_t tot = 0;
            for (int y = 0; y < kXcd; ++y) tot += placed(mid, y);
            if (tot >= n_admit) hi = mid; else lo = mid + 1;
        }
        int32_t given = 0;
        for (int y = 0; y < kXcd; ++y) { sl.admit[y] = n_admit > 0 ? placed(lo, y) : 0; given += sl.admit[y]; }
        for (int y = kXcd - 1; y >= 0 && given > n_admit; --y) {
            const int32_t cut = min(sl.admit[y], given - n_admit);
            sl.admit[y] -= cut;
            given -= cut;
        }
        if (a.wide && a.method != FV_BEAM) {
            // wide rows are computed by every block whatever their list, in
            // groups of kWideRows per list, and each group streams log A
            // once per step: fill the lists in order so that rows share
            // groups (spread over the XCDs, eight single rows would stream
            // log A eight times).  Beam tasks run on their own XCD's blocks
            // and stay spread.
            int32_t left = n_admit;
            for (int y = 0; y < kXcd; ++y) {
                sl.admit[y] = min(cap[y], left);
                left -= sl.admit[y];
            }
        }
    }
    __syncthreads();
    const int x = threadIdx.x / kSchedGroup, tg = threadIdx.x % kSchedGroup;
    // the admitted tasks are dealt over the XCDs in proportion to their
    // quotas: XCD y's i-th task has the key (2i + 1) / admit[y] (the middle
    // of its share of the batch), and the batch is taken in key order, so
    // that with the queue sorted longest first every XCD gets the same mix of
    // long and short tasks whatever its quota.  Equal keys go up the XCDs for
    // even i and down for odd i (a snake: with equal quotas no XCD always gets
    // the longest task of a round).  XCD x's k-th task is batch entry q_head
    // + k + the number of other XCDs' tasks before it.
    int32_t qa[kXcd];
#pragma unroll
    for (int y = 0; y < kXcd; ++y) qa[y] = sl.admit[y];
    auto before = [&](int32_t y, int32_t i, int32_t k) -> bool {   // (y, i) ahead of (x, k)
        const int64_t l = (int64_t)(2 * i + 1) * qa[x], r = (int64_t)(2 * k + 1) * qa[y];
        if (l != r) return l < r;
        const int32_t sy = (i & 1) ? kXcd - 1 - y : y, sx = (k & 1) ? kXcd - 1 - x : x;
        return sy != sx ? sy < sx : y < x;
    };
    auto dealt = [&](int32_t k) -> int32_t {
        int32_t pos = sl.q_head + k;
        for (int y = 0; y < kXcd; ++y) {
            if (y == x || qa[y] == 0) continue;
            int32_t lo = 0, hi = qa[y];   // tasks of y ahead of (x, k): a prefix of its range
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (before(y, mid, k)) lo = mid + 1; else hi = mid;
            }
            pos += lo;
        }
        return pos;
    };
    const int32_t ax = sl.admit[x];
    // this thread's tasks: a contiguous range, so list order follows the deal
    const int32_t per = (ax + kSchedGroup - 1) / kSchedGroup;
    const int32_t lo = min(ax, tg * per), hi = min(ax, lo + per);
    int32_t c[3] = {0, 0, 0}, tot[3];
    for (int32_t k = lo; k < hi; ++k) c[start_list(a, a.queue[dealt(k)].kind)]++;
    group_scan<3>(c, tot, sl.wave_sums[x]);
    Row* out[3] = {list_full(a, nxt, x), list_light(a, nxt, x), list_beam(a, nxt, x)};
    for (int32_t k = lo; k < hi; ++k) {
        const Task tk = a.queue[dealt(k)];
        const int32_t slot = a.free_stack[(int64_t)x * a.pool + sl.n_free[x] - 1 - k];
        const Row r = row_from_task(a, tk, slot);
        const int32_t li = start_list(a, tk.kind);
        st_row(out[li] + sl.n_next[x][li] + c[li]++, r);
    }
    // every row of the coming step (successors and admissions) is written
    // before the counts word that announces it: compute blocks read their
    // first rows as soon as they see that word, before the barrier opens
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (tg == 0) {
        for (int k = 0; k < 3; ++k) sl.n_next[x][k] += tot[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t all = 0;
        for (int y = 0; y < kXcd; ++y) {
            sl.q_head += sl.admit[y];
            sl.n_free[y] -= sl.admit[y];
            for (int k = 0; k < 3; ++k) {
                st_c(&a.st->cnt[nxt][y][k], sl.n_next[y][k]);
                all += sl.n_next[y][k];
            }
            st_c(&a.st->claim[nxt][y][0], 0);
            st_c(&a.st->claim[nxt][y][8], 0);
            st_c(&a.st->claim[nxt][y][16], 0);
        }
        st_c(&a.st->wclaim[nxt][0], 0);
        st_c(&a.st->total[nxt], all);
        for (int y = 0; y < kXcd; ++y)
            st_c(&a.st->cntw[y][0], pack_counts(tag, all == 0, sl.n_next[y][0], sl.n_next[y][1], sl.n_next[y][2]));
        sl.total_next = all;
        if (all > sl.max_rows) sl.max_rows = all;
        st_c(&a.st->max_rows, sl.max_rows);
    }
    __syncthreads();
}

// One pass over this step's rows of each XCD (a 128-thread group per XCD):
// each row is loaded once, classified, and its successor row, freed slot and
// spawned tasks take their positions from LDS counters.  The order of the
// next lists, of the free stack and of the spawned tasks then depends on
// timing; no result does (every row and task is computed on its own).
__device__ __noinline__ void scheduler(cargs_t& a_in, int32_t s, uint32_t tag) {
    cargs_t& a = uniform_args(a_in);
    SchedLds& sl = g_sched;
    const int cur = s & 1, nxt = cur ^ 1;
    const int x = threadIdx.x / kSchedGroup, tg = threadIdx.x % kSchedGroup;
    // this step's counts: the previous admission left them in LDS
    const int32_t nf = sl.n_next[x][0];
    const int32_t nl = sl.n_next[x][1];
    const int32_t nbm = sl.n_next[x][2];
    __syncthreads();
    if (tg < 4) sl.out_cnt[x][tg] = 0;   // full, light, beam, freed
    if (threadIdx.x == 0) sl.q_spawn = sl.q_tail;
    __syncthreads();
    const int32_t total = nf + nl + nbm;
    const Row* lists[3] = {list_full(a, cur, x), list_light(a, cur, x), list_beam(a, cur, x)};
    Row* out[3] = {list_full(a, nxt, x), list_light(a, nxt, x), list_beam(a, nxt, x)};
    for (int32_t i = tg; i < total; i += kSchedGroup) {
        const int src = i < nf ? 0 : (i < nf + nl ? 1 : 2);
        const int32_t k = src == 0 ? i : (src == 1 ? i - nf : i - nf - nl);
        const Row r = ld_row(lists[src] + k);
        const Next n = classify(a, r, src);
        if (n.list >= 0) {
            const int32_t pos = atomicAdd(&sl.out_cnt[x][n.list], 1);
            st_row(out[n.list] + pos, n.row);
        }
        if (n.freed) {
            const int32_t pos = atomicAdd(&sl.out_cnt[x][3], 1);
            a.free_stack[(int64_t)x * a.pool + sl.n_free[x] + pos] = r.slot;
        }
        if (n.spawn) write_spawns(a, r, src, (int64_t)atomicAdd(&sl.q_spawn, n.spawn));
    }
    __syncthreads();
    if (threadIdx.x == 0) sl.q_tail = sl.q_spawn;
    if (tg == 0) {
        sl.n_free[x] += sl.out_cnt[x][3];
        for (int k = 0; k < 3; ++k) sl.n_next[x][k] = sl.out_cnt[x][k];
    }
    __syncthreads();
    admit(a, nxt, tag);
}

// ---------------------------------------------------------------- step barrier
// Compute blocks publish their writes (agent-scope release), store their
// arrival flag, wait for their XCD's release flag and acquire (agent scope).
// The scheduler block is the master: it waits for every arrival, acquires,
// releases, then raises the 8 release flags.  One block per CU keeps the
// per-block cache maintenance of the fences to 256 operations per step.
// Spins are bounded; on overrun the error flag is raised and every block
// leaves the step loop.

// The go word of a step barrier: the epoch, with this bit set when the engine
// has an error (so a waiting block learns it without another load).
constexpr uint32_t kGoErr = 0x80000000u;

// Step-barrier memory ordering.  With wide rows, plain stores of one XCD
// are read by others: the agent-scope release writes the L2 back.
// Otherwise every plain store is read on its own XCD (through its L2) and
// all data crossing XCDs moves by coherent atomics, so a block only waits
// for its stores to complete.  The acquire side is the agent-scope fence in
// both cases: it invalidates the vector L1 (an L1-only invalidate does not
// on this device) and leaves the XCD's L2 lines of device memory in place.
__device__ __forceinline__ void step_release(bool wide) {
    if (wide) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}
__device__ __forceinline__ void step_acquire(bool) { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// The wait also returns the counts word the scheduler published for the
// step after this barrier (tagged with this epoch; both words are polled
// together, so the counts need no load of their own after the release).
__device__ bool barrier_arrive_wait(cargs_t& a, uint32_t epoch, uint32_t x, unsigned long long& counts,
                                    bool with_counts = true) {
    __shared__ int s_err;
    __shared__ unsigned long long s_counts;
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool wide = a.wide != 0;
        step_release(wide);
        st_c(a.arrive + blockIdx.x, epoch);
        int err = 0;
        int64_t spins = 0;
        const unsigned long long want = (unsigned long long)(epoch & kTagMask);
        unsigned long long cw = 0;
        uint32_t g = 0;
        for (;;) {
            g = ld_c(&a.st->go[x][0]);
            cw = ld_c(&a.st->cntw[x][0]);
            if ((g & ~kGoErr) >= epoch && (!with_counts || (cw >> kTagShift) == want)) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > a.spin_limit) { st_c(&a.st->error, 1); err = 1; break; }
            if ((spins & 255) == 0 && ld_c(&a.st->error)) { err = 1; break; }
        }
        step_acquire(wide);
        s_err = err || (g & kGoErr) != 0;
        s_counts = cw;
    }
    __syncthreads();
    counts = s_counts;
    return s_err == 0;
}

// The step barrier of a compute block of a slab model: arrive; as soon as
// the scheduler has published the next step's counts (it does so before the
// barrier opens), read the block's first rows for that step; then wait for
// the barrier.  ready_u: the first unit of the rows read, or -1.
__device__ __forceinline__ bool barrier_slab(cargs_t& a, uint32_t epoch, uint32_t x, int32_t nx, int32_t rank, int nxt,
                                             unsigned long long& counts, int64_t& ready_u) {
    __shared__ int s_err2, s_open2;
    __shared__ unsigned long long s_counts2;
    __syncthreads();
    if (threadIdx.x == 0) {
        step_release(false);
        st_c(a.arrive + blockIdx.x, epoch);
        int err = 0, open = 0;
        int64_t spins = 0;
        const unsigned long long want = (unsigned long long)(epoch & kTagMask);
        unsigned long long cw = 0;
        uint32_t g = 0;
        for (;;) {   // until the counts word of the coming step is there
            g = ld_c(&a.st->go[x][0]);
            cw = ld_c(&a.st->cntw[x][0]);
            if ((cw >> kTagShift) == want) { open = (g & ~kGoErr) >= epoch; break; }
            __builtin_amdgcn_s_sleep(1);
            if (++spins > a.spin_limit) { st_c(&a.st->error, 1); err = 1; break; }
            if ((spins & 255) == 0 && ld_c(&a.st->error)) { err = 1; break; }
        }
        s_err2 = err || (open && (g & kGoErr) != 0);
        s_open2 = open;
        s_counts2 = cw;
    }
    __syncthreads();
    const unsigned long long cw = s_counts2;
    counts = cw;
    ready_u = s_err2 == 0 ? slab_prefetch_rows(a, x, nx, rank, nxt, cw) : -1;
    if (threadIdx.x == 0) {
        int err = s_err2;
        int64_t spins = 0;
        if (!err && !s_open2) {
            for (;;) {   // until the barrier opens
                const uint32_t g = ld_c(&a.st->go[x][0]);
                if ((g & ~kGoErr) >= epoch) { err = (g & kGoErr) != 0; break; }
                __builtin_amdgcn_s_sleep(1);
                if (++spins > a.spin_limit) { st_c(&a.st->error, 1); err = 1; break; }
                if ((spins & 255) == 0 && ld_c(&a.st->error)) { err = 1; break; }
            }
        }
        step_acquire(false);
        s_err2 = err;
    }
    __syncthreads();
    return s_err2 == 0;
}

__device__ bool barrier_master(cargs_t& a, uint32_t epoch) {
    __shared__ int s_err;
    __syncthreads();
    int64_t spins = 0;
    int err = 0;
    uint32_t e_seen = 0;   // the error word, read with the arrivals (thread 0)
    for (;;) {
        int ok = 1;
        if (threadIdx.x == 0) e_seen = ld_c(&a.st->error);
        for (int32_t b = 1 + threadIdx.x; b <= a.n_compute_blocks; b += kEngBlock)
            if (ld_c(a.arrive + b) < epoch) ok = 0;
        if (__syncthreads_and(ok)) break;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > a.spin_limit) { err = 1; break; }
    }
    if (threadIdx.x == 0) {
        const bool wide = a.wide != 0;
        step_acquire(wide);
        step_release(wide);
        s_err = err || e_seen != 0;
    }
    __syncthreads();
    const int err_all = s_err;
    if (threadIdx.x < kXcd) {
        if (err) st_c(&a.st->error, 1);
        // the error travels with the go word
        st_c(&a.st->go[threadIdx.x][0], epoch | (err_all ? kGoErr : 0u));
    }
    __syncthreads();
    return err_all == 0;
}

// ---------------------------------------------------------------- engine
// Wide-row phase of a step: items (XCD list, group of 16 rows, 64-column
// chunk) over the dense rows of every XCD, taken by all blocks of the chip:
// first by global rank, then claimed from one counter.
__device__ __forceinline__ void run_wide(cargs_t& a_in, int cur) {
    cargs_t& a = uniform_args(a_in);
    const float* __restrict__ Ap = a.Acol;
    __shared__ int32_t s_item;
    const int32_t nch = a.Kp / kWideCols;
    int32_t nf[kXcd], base[kXcd + 1];
    base[0] = 0;
    for (int y = 0; y < kXcd; ++y) {
        nf[y] = ld_c(&a.st->cnt[cur][y][0]);
        base[y + 1] = base[y] + (nf[y] + kWideRows - 1) / kWideRows;
    }
    const int32_t ngrp = base[kXcd], total = ngrp * nch;
    int32_t item = blockIdx.x >= 1 ? (int32_t)blockIdx.x - 1 : -1;
    for (;;) {
        if (item < 0) {
            if (threadIdx.x == 0)
                s_item = a.n_compute_blocks +
                         __hip_atomic_fetch_add(&a.st->wclaim[cur][0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            item = s_item;
            __syncthreads();
        }
        if (item >= total) break;
        // chunk-major: the row groups of one column chunk are consecutive
        // items, taken at about the same time, so they share its log A reads
        const int32_t chunk = item / ngrp, gq = item - chunk * ngrp;
        int y = 0;
        while (gq >= base[y + 1]) ++y;
        wide_item(a, Ap, list_full(a, cur, y), nf[y], gq - base[y], chunk, 1);
        item = -1;
    }
}

// Column items of an XCD with few dense rows, claimed from its counter.  The
// item body is inlined here: one call per step instead of one per item
// (a call saves and restores the callee-saved registers the body uses).
__device__ __forceinline__ void local_col_items(cargs_t& a_in, uint32_t x, int32_t nx, int32_t rank, int cur,
                                             int32_t nf) {
    cargs_t& a = uniform_args(a_in);
    const float* __restrict__ Ap = a.Acol;
    __shared__ int32_t s_citem;
    const bool two = a.At != nullptr;   // two-column items (Kp <= kColMaxKp)
    const int32_t nch = two ? (a.Kp + kColCols - 1) / kColCols : a.Kp / kWideCols;
    // row groups of two-column items, at most kColRows rows each.  When one
    // round of items fits on the XCD's blocks, as many groups as fit, rows
    // spread evenly; otherwise full groups with the remainder last, so that
    // the items claimed in a second round are the cheapest, unless two
    // rounds of evenly spread groups cost less.
    const int32_t gmin = (nf + kColRows - 1) / kColRows, gfit = nx / nch;
    bool spread = two && gmin <= gfit;
    int32_t ngrp = two ? (spread ? min(nf, gfit) : gmin) : (nf + kWideRows - 1) / kWideRows;
    if (two && !spread && nx > 0) {
        // full groups need a second round: compare with rows spread evenly
        // over two rounds' worth of groups (cost in rows, fixed part
        // kColItemFixed per item)
        const int32_t over = gmin * nch - nx;   // items beyond the first round
        const int32_t rem = nf - (gmin - 1) * kColRows;   // rows of the last group
        const int32_t c_full = over <= nch ? (kColItemFixed + kColRows) + (kColItemFixed + rem)
                                           : ((gmin * nch + nx - 1) / nx) * (kColItemFixed + kColRows);
        const int32_t g2 = max(gmin, min(nf, (2 * nx) / nch));
        const int32_t c_spread = ((g2 * nch + nx - 1) / nx) * (kColItemFixed + (nf + g2 - 1) / g2);
        if (c_spread < c_full) { spread = true; ngrp = g2; }
    }
    const int32_t total = ngrp * nch;
    const Row* Fl = list_full(a, cur, x);
    int32_t item = rank;
    for (;;) {
        if (item < 0) {
            if (threadIdx.x == 0)
                s_citem = nx + __hip_atomic_fetch_add(&a.st->claim[cur][x][8], 1, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            item = s_citem;
            __syncthreads();
        }
        if (item >= total) break;
        if (two) {
            const int32_t gq = item / nch;
            const int32_t r0 = spread ? (gq * nf) / ngrp : gq * kColRows;
            const int32_t r1 = spread ? ((gq + 1) * nf) / ngrp : min(nf, r0 + kColRows);
            col_item(a, Ap, Fl, r0, r1 - r0, item - gq * nch);
        }
        else wide_item(a, Ap, Fl, nf, item % ngrp, item / ngrp, 0);   // chunk-major, as run_wide
        item = -1;
    }
}

// Work of one XCD at one step.  Phase 1: dense tiles and light rows, taken
// by tile groups (nsplit waves) one item at a time: a tile, or nsplit light
// rows (one per wave).  Groups run independently, so one group's
// latency-bound epilogue overlaps the others' max-plus loops.  Phase 2:
// beam rows, one per block.  Each phase hands items out from a per-XCD
// counter; every block (and the scheduler block once its own work is done)
// takes a first item by rank, then claims until none are left.
template <bool WIDE, bool SLAB>
__device__ __forceinline__ void run_units(cargs_t& a, const float* __restrict__ Ap, uint32_t x, int32_t nx,
                                          int32_t rank, int cur, int32_t nf, int32_t nl, int32_t nbm,
                                          int64_t ready_u) {
    EngineLds& lds = g_lds;
    __shared__ int32_t s_unit;
    // few rows on this XCD: lane tiles would run mostly empty, so its rows are
    // computed as column items (lanes = destinations) by its own blocks
    const bool local_cols = !WIDE && !a.sparse && nf > 0 && nf <= kLocalColRows && !a.force_tiles;
    const int32_t n_tiles =
        (WIDE || local_cols || a.sparse) ? 0 : ((nf + kTileRows - 1) / kTileRows) * (a.Kp / kTileCols);
    if constexpr (WIDE) run_wide(a, cur);
    if (a.sparse && nf > 0) {
        // sparse rows: units of (row, 64 destinations), one per wave, 16 per block item
        __shared__ int32_t s_sitem;
        const int32_t nch = a.Kp / 64;
        const int32_t n_units = nf * nch;
        const int32_t n_items = (n_units + kEngWaves - 1) / kEngWaves;
        const Row* Fl = list_full(a, cur, x);
        int32_t item = rank;
        for (;;) {
            if (item < 0) {
                if (threadIdx.x == 0)
                    s_sitem = nx + __hip_atomic_fetch_add(&a.st->claim[cur][x][8], 1, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                item = s_sitem;
                __syncthreads();
            }
            if (item >= n_items) break;
            const int32_t u = item * kEngWaves + (threadIdx.x >> 6);
            if (u < n_units) sparse_unit(a, Fl, u / nch, u % nch);
            item = -1;
        }
    }
    // light and block rows below these indices are taken by blocks set aside
    // from the slab share; the rest go to the claims below
    int32_t lo_light = 0, lo_block = 0;
    if constexpr (SLAB) {
        if (local_cols) {
            // A block row (a finalize or a leaf's end) or a light row run
            // after a full slab share would finish last: up to a quarter of
            // the XCD's blocks take them instead (one block row per block, one
            // light row per wave) and the others split the slab units.
            const SlabShare sh = slab_share(a, nx, rank, nf, nl, nbm);
            const int32_t nsl = sh.nsl;
            if (a.method != FV_BEAM && nx > 0) {
                const int32_t nbx = sh.nbx;
                lo_block = nbx;
                lo_light = sh.lo_light;
                if (rank >= nsl) {
                    const int32_t e = rank - nsl;
                    if (e < nbx) {
                        const Row r = ld_row(list_beam(a, cur, x) + e);
                        if (r.aux == L_LEAF_END) leaf_end(a, r);
                        else dense_finalize(a, r);
                    } else {
                        const int32_t li = (e - nbx) * kEngWaves + (threadIdx.x >> 6);
                        if (li < lo_light) light_row(a, Ap, ld_row(list_light(a, cur, x) + li));
                    }
                }
            }
            if (sh.u < sh.u1) {
                const bool ready = ready_u == sh.u;
                if (a.Kp == 1024) slab_items_kp<1024>(a, Ap, list_full(a, cur, x), nf, sh.u, sh.u1, ready);
                else slab_items_kp<512>(a, Ap, list_full(a, cur, x), nf, sh.u, sh.u1, ready);
            }
        }
    } else {
        if (local_cols) local_col_items(a, x, nx, rank, cur, nf);
    }
    // waves per tile: 4 (one per SIMD) while every group gets two tiles or
    // more, else more waves per tile (fewer, faster groups); at most one wave
    // per 16 predecessors.  Decided from a nominal XCD of 32 blocks, so that
    // all XCDs take the same choice for the same row count.
    int32_t nsplit = 4;
    {
        constexpr int32_t kNominalBlocks = 32;
        while (nsplit < kEngWaves && n_tiles * 2 <= kNominalBlocks * (kEngWaves / nsplit)) nsplit <<= 1;
        while (nsplit > 4 && nsplit * kGroup > a.Kp) nsplit >>= 1;
    }
    const int32_t ngrp = kEngWaves / nsplit;
    const int32_t bw = threadIdx.x >> 6, grp = bw / nsplit, wv = bw & (nsplit - 1);
    const int32_t n_lu = (nl - lo_light + nsplit - 1) / nsplit;
    const int32_t n1 = n_tiles + n_lu;
    const Row* F = list_full(a, cur, x);
    const Row* L = list_light(a, cur, x);
    if (threadIdx.x < 4) lds.tile.gsync[threadIdx.x] = 0;
    __syncthreads();
    if (n1 > 0) {
        int32_t* ctr = &a.st->claim[cur][x][0];
        int32_t item = rank >= 0 ? rank * ngrp + grp : -1;
        for (;;) {
            if (item < 0) {
                if (wv == 0 && (threadIdx.x & 63) == 0)
                    lds.tile.gitem[grp] =
                        nx * ngrp + __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                group_sync(&lds.tile.gsync[grp], nsplit);
                item = lds.tile.gitem[grp];
            }
            if (item >= n1) break;
            if (item < n_tiles) {
                dense_tile(a, Ap, F, nf, item, nsplit);
            } else {
                const int32_t li = lo_light + (item - n_tiles) * nsplit + wv;
                if (li < nl) light_row(a, Ap, ld_row(L + li));
            }
            item = -1;
        }
    }
    nbm -= lo_block;
    if (nbm == 0) return;
    __syncthreads();
    const Row* Bl = list_beam(a, cur, x) + lo_block;
    int32_t* ctr2 = &a.st->claim[cur][x][16];
    if (a.beam_q) {   // beam rows four to a block: each 256-thread group claims rows
        QuarterLds& Q = g_lds.qbeam;
        if (threadIdx.x < kQGroups) Q.gsync[threadIdx.x] = 0;
        __syncthreads();
        const int32_t g = q_grp();
        int32_t item = rank >= 0 ? rank * kQGroups + g : -1;
        for (;;) {
            if (item < 0) {
                if (q_tid() == 0)
                    Q.gitem[g] = nx * kQGroups + __hip_atomic_fetch_add(ctr2, 1, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT);
                q_sync();
                item = Q.gitem[g];
            }
            if (item >= nbm) break;
            beam_row_q(a, ld_row(Bl + item));
            item = -1;
        }
        return;
    }
    // parts per beam row this step: all a.bw while the XCD's blocks
    // outnumber its rows' parts, fewer (down to the LDS limit) when many beam
    // rows are in flight; the results do not depend on the count
    const int32_t Wu = a.bw > 1 ? max(a.bw_min, min(a.bw, nx / max(nbm, 1))) : 1;
    int32_t u = rank;
    for (;;) {
        if (u < 0) {
            if (threadIdx.x == 0) s_unit = nx + __hip_atomic_fetch_add(ctr2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            u = s_unit;
            __syncthreads();
        }
        if (u >= nbm * Wu) break;   // item = (row, part); finalizes use part 0
        const int32_t part = u % Wu;
        const Row r = ld_row(Bl + u / Wu);
        if (is_beam(r.kind)) beam_row(a, Ap, r, part, Wu);
        else if (part == 0 && r.aux == L_LEAF_END) leaf_end(a, r);
        else if (part == 0) dense_finalize(a, r);
        u = -1;
    }
}

// Every step of one model's decode (its own state, lists and buffers),
// specialised for wide or local rows: each step loop inlines its own per-step
// work function, so no call saves registers at every step.
template <bool WIDE, bool SLAB>
__device__ __noinline__ void engine_model(cargs_t& a_in) {
    cargs_t& a = uniform_args(a_in);
    const float* __restrict__ Ap = a.Acol;
    const bool is_sched = blockIdx.x == 0;
    const uint32_t x = my_xcd();
    __shared__ int32_t s_rank;
    if (threadIdx.x == 0)   // rank among the compute blocks of this XCD (the scheduler has none)
        s_rank = is_sched ? -1
                          : (int32_t)__hip_atomic_fetch_add(&a.st->xcd_blocks[x][0], 1u, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_SYSTEM);
    uint32_t epoch = 1;
    unsigned long long cw = 0;   // counts word of the coming step (compute blocks)
    // the first barrier publishes no counts (the first admission follows it)
    bool ok = is_sched ? barrier_master(a, epoch) : barrier_arrive_wait(a, epoch, x, cw, false);
    const int32_t rank = s_rank;
    const int32_t nx = (int32_t)ld_c(&a.st->xcd_blocks[x][0]);

    if (is_sched) {
        SchedLds& sl = g_sched;
        if (threadIdx.x == 0) {
            sl.q_head = 0;
            sl.q_tail = ld_c(&a.st->q_tail0);
            sl.max_rows = 0;
            for (int y = 0; y < kXcd; ++y) {
                sl.n_free[y] = a.pool;
                sl.nblk[y] = (int32_t)ld_c(&a.st->xcd_blocks[y][0]);
                if (a.slab) {
                    // an XCD whose compute blocks do not divide evenly over
                    // the column passes (the scheduler's: 31) splits its
                    // units across passes, and some blocks load two slabs:
                    // it is admitted rows as if it had 4 blocks fewer
                    const int32_t npass = a.Kp / ((kEngWaves / (a.Kp / 64)) * 64);
                    if (sl.nblk[y] % npass != 0) sl.nblk[y] = max(1, sl.nblk[y] - 4);
                }
                for (int k = 0; k < 3; ++k) sl.n_next[y][k] = 0;
            }
        }
        __syncthreads();
        if (ok) admit(a, 0, epoch + 1);
    }
    ++epoch;
    if (ok) ok = is_sched ? barrier_master(a, epoch) : barrier_arrive_wait(a, epoch, x, cw);

    int32_t s = 0;
    int64_t ready_u = -1;   // slab models: first unit of the rows read at the last barrier
    for (; ok; ++s) {
        const int cur = s & 1;
        // this step's counts on this XCD, and whether any row is left anywhere
        int32_t nf, nl, nbm;
        bool done;
        if (is_sched) {
            SchedLds& sl = g_sched;
            nf = sl.n_next[x][0]; nl = sl.n_next[x][1]; nbm = sl.n_next[x][2];
            done = sl.total_next == 0;
            __syncthreads();   // read before the scheduler rewrites them
        } else {
            nf = (int32_t)(cw & 0x3fff); nl = (int32_t)((cw >> 14) & 0x3fff); nbm = (int32_t)((cw >> 28) & 0x3fff);
            done = ((cw >> 42) & 1) != 0;
        }
        if (done) break;
        if (s > a.max_steps) {  // schedule longer than any valid one: report, stop
            if (is_sched && threadIdx.x == 0) st_c(&a.st->error, 2);
            break;
        }
        unsigned long long* tr = (a.trace && s < a.trace_steps) ? a.trace + (int64_t)s * kTraceWords : nullptr;
        if (tr && is_sched && threadIdx.x == 0) {
            tr[TR_START] = __builtin_amdgcn_s_memrealtime();
            int32_t c[kXcd][3];   // every load issued before the sums
#pragma unroll
            for (int y = 0; y < kXcd; ++y)
#pragma unroll
                for (int q = 0; q < 3; ++q) c[y][q] = ld_c(&a.st->cnt[cur][y][q]);
            int32_t nf = 0, nl = 0, nb = 0;
#pragma unroll
            for (int y = 0; y < kXcd; ++y) { nf += c[y][0]; nl += c[y][1]; nb += c[y][2]; }
            tr[TR_ROWS] = (unsigned long long)nf | ((unsigned long long)nl << 21) | ((unsigned long long)nb << 42);
        }
        if (is_sched) scheduler(a, s, epoch + 1);
        if (tr && is_sched && threadIdx.x == 0) tr[TR_SCHED] = __builtin_amdgcn_s_memrealtime();
        run_units<WIDE, SLAB>(a, Ap, x, nx, rank, cur, nf, nl, nbm, ready_u);
        if (tr && !is_sched) {
            __syncthreads();
            if (threadIdx.x == 0) {
                const unsigned long long now = __builtin_amdgcn_s_memrealtime();
                __hip_atomic_fetch_min(&tr[TR_END_MIN], now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&tr[TR_END_MAX], now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&tr[TR_END_SUM], now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&tr[TR_NBLK], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&tr[TR_XCD_END + x], now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        ++epoch;
        if constexpr (SLAB)
            ok = is_sched ? barrier_master(a, epoch)
                          : barrier_slab(a, epoch, x, nx, rank, (s + 1) & 1, cw, ready_u);
        else
            ok = is_sched ? barrier_master(a, epoch) : barrier_arrive_wait(a, epoch, x, cw);
    }
    if (is_sched && threadIdx.x == 0) st_c(&a.st->steps, s);
}

// One cooperative launch decodes the batches of n_models models in turn
// (table: their argument blocks, in the workspace).
extern "C" __global__ __launch_bounds__(kEngBlock) void fv_engine_kernel(const EngineArgs* __restrict__ table,
                                                                         int32_t n_models) {
    for (int32_t mi = 0; mi < n_models; ++mi) {
        __syncthreads();
        cargs_t& a = *reinterpret_cast<cargs_t*>(reinterpret_cast<uint64_t>(table + mi));
        if (a.wide) engine_model<true, false>(a);
        else if (a.slab) engine_model<false, true>(a);
        else engine_model<false, false>(a);
    }
}

// ---------------------------------------------------------------- small single decode
// Vanilla decodes of a small dense model (K <= 64), one wave (block) per
// sequence, in place of the persistent engine: lane l keeps destination l's
// column of log A in registers and reads the previous step's scores from the
// lanes that hold them (readlane), so a step needs no barrier and no
// scheduling.  (64 < K <= kSmallK runs two waves per sequence, below.)
// The arithmetic and tie rules are the engine's: per destination the first
// maximum over predecessors in index order, its own value kept, delta = that
// + log B_t(j); the final state is the lowest index of the largest score (-0
// and +0 equal).  The backpointers go to the same table as an engine
// decode's, and one lane walks them back at the end.  Emission rows are read
// kSmallPrefetch steps ahead.
constexpr int32_t kSmallPrefetch = 4;

// The candidate loop of both one-wave kernels, over a compile-time width
// KMAX >= K: states K..KMAX-1 have score -inf and log A -inf, so their
// candidates are -inf and never win the strict comparison; no per-candidate
// test of K is needed.  Even and odd predecessors are two independent
// chains (first maximum each), merged so that the larger value wins and
// equal values (-0 == +0) go to the lower index: the same result as one
// scan in index order.
template <int KMAX, int NJ>
__device__ __forceinline__ void small_candidates(const float (&col)[NJ][KMAX], const float (&d)[NJ],
                                                 float (&best)[NJ], int32_t (&arg)[NJ]) {
    float b1[NJ];
    int32_t a1[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        best[c] = -INFINITY;
        arg[c] = 0;
        b1[c] = -INFINITY;
        a1[c] = 0;
    }
#pragma unroll
    for (int i = 0; i < KMAX; i += 2) {
        const float d0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d[i / 64]), i % 64));
        const float d1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d[(i + 1) / 64]), (i + 1) % 64));
#pragma unroll
        for (int c = 0; c < NJ; ++c) {
            const float x0 = d0 + col[c][i];
            const float x1 = d1 + col[c][i + 1];
            if (x0 > best[c]) { best[c] = x0; arg[c] = i; }
            if (x1 > b1[c]) { b1[c] = x1; a1[c] = i + 1; }
        }
    }
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        if (b1[c] > best[c] || (b1[c] == best[c] && a1[c] < arg[c])) {
            best[c] = b1[c];
            arg[c] = a1[c];
        }
    }
}

template <int KMAX>
__device__ __forceinline__ void small_vanilla(cargs_t& a, SeqInfo& sq) {
    constexpr int NJ = KMAX > 64 ? 2 : 1;
    const int32_t lane = threadIdx.x;
    const int32_t K = a.K, T = sq.T;
    bool on[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) on[c] = lane + 64 * c < K;
    gfloat_t* lb = as_global(sq.log_b);
    const int64_t ld = sq.ld;
    float col[NJ][KMAX];
#pragma unroll
    for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            col[c][i] = (on[c] && i < K) ? a.Acol[(int64_t)i * a.Kp + lane + 64 * c] : -INFINITY;
    float bq[NJ][kSmallPrefetch];
#pragma unroll
    for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int k = 0; k < kSmallPrefetch; ++k)
            bq[c][k] = (on[c] && 1 + k < T) ? lb[(int64_t)(1 + k) * ld + lane + 64 * c] : 0.0f;
    float d[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        d[c] = -INFINITY;
        if (on[c]) {
            const int32_t j = lane + 64 * c;
            d[c] = a.log_pi ? a.log_pi[j] + lb[j] : lb[j];
        }
    }
    uint16_t* psi = a.psi16 + sq.psi_off;
    for (int32_t t = 1; t < T; ++t) {
        float bt[NJ];
#pragma unroll
        for (int c = 0; c < NJ; ++c) {
            bt[c] = bq[c][0];
#pragma unroll
            for (int k = 0; k + 1 < kSmallPrefetch; ++k) bq[c][k] = bq[c][k + 1];
            bq[c][kSmallPrefetch - 1] =
                (on[c] && t + kSmallPrefetch < T) ? lb[(int64_t)(t + kSmallPrefetch) * ld + lane + 64 * c] : 0.0f;
        }
        float best[NJ];
        int32_t arg[NJ];
        small_candidates<KMAX, NJ>(col, d, best, arg);
#pragma unroll
        for (int c = 0; c < NJ; ++c) {
            if (on[c]) psi[(int64_t)t * K + lane + 64 * c] = (uint16_t)arg[c];
            d[c] = on[c] ? best[c] + bt[c] : -INFINITY;
        }
    }
    unsigned long long key = 0;
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        const unsigned long long k = on[c] ? order_key(d[c], lane + 64 * c) : 0ull;
        if (k > key) key = k;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        if (o > key) key = o;
    }
    const int32_t qT = clampi((int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull)), K);
    float sc = __shfl(d[0], qT % 64, 64);
    if (NJ > 1 && qT >= 64) sc = __shfl(d[NJ - 1], qT % 64, 64);
    if (sc == -INFINITY) {
        for (int32_t t = lane; t < T; t += 64) sq.path[t] = -1;
        if (lane == 0) {
            *sq.score = sc;
            sq.status = FV_E_INFEASIBLE;
        }
        return;
    }
    if (lane == 0) {
        *sq.score = sc;
        sq.path[T - 1] = qT;
    }
    // backtrace from q*_{T-1} by one lane, while the table rows this wave
    // wrote are still in its XCD's L2 (the finish kernel skips the walk)
    __syncthreads();
    if (lane == 0) {
        int32_t q = qT;
        for (int32_t t = T - 1; t > 0; --t) {
            q = clampi(psi[(int64_t)t * K + q], K);
            sq.path[t - 1] = q;
        }
    }
}

// One kernel per width (K <= 32, 64), so each gets the register allocation
// of its own step loop.
#define FV_SMALL_VANILLA(NAME, KMAX)                                                                   \
    extern "C" __global__ __launch_bounds__(64) void NAME(const EngineArgs* __restrict__ table) {       \
        cargs_t& a = *reinterpret_cast<cargs_t*>(reinterpret_cast<uint64_t>(table));                    \
        if ((int32_t)blockIdx.x >= a.n_seqs) return;                                                    \
        SeqInfo& sq = a.seqs[blockIdx.x];                                                               \
        if (sq.status != FV_OK || sq.T <= 0 || a.K > KMAX) return;                                      \
        small_vanilla<KMAX>(a, sq);                                                                     \
    }
FV_SMALL_VANILLA(fv_small_vanilla32_kernel, 32)
FV_SMALL_VANILLA(fv_small_vanilla64_kernel, 64)
#undef FV_SMALL_VANILLA

// 64 < K <= 256: KMAX / 64 waves per sequence (KMAX = 128 or 256), thread j
// for destination j (its column of log A in registers; one wave with
// several columns per lane would need more than the whole register file).  Each step publishes the
// scores in LDS, double-buffered so that one barrier per step suffices, and
// every thread reads them back four at a time (broadcast reads).  Same
// candidate order, tie rules, finalize and in-kernel backtrace as above.
template <int KMAX>
__device__ __forceinline__ void small_vanilla_waves(const EngineArgs* __restrict__ table) {
    cargs_t& a = *reinterpret_cast<cargs_t*>(reinterpret_cast<uint64_t>(table));
    if ((int32_t)blockIdx.x >= a.n_seqs) return;
    SeqInfo& sq = a.seqs[blockIdx.x];
    if (sq.status != FV_OK || sq.T <= 0 || a.K > KMAX) return;
    __shared__ __align__(16) float dsh[2][KMAX];
    __shared__ unsigned long long wkey[KMAX / 64];
    const int32_t j = threadIdx.x;
    const int32_t K = a.K, T = sq.T;
    const bool on = j < K;
    gfloat_t* lb = as_global(sq.log_b);
    const int64_t ld = sq.ld;
    float col[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) col[i] = (on && i < K) ? a.Acol[(int64_t)i * a.Kp + j] : -INFINITY;
    float bq[kSmallPrefetch];
#pragma unroll
    for (int k = 0; k < kSmallPrefetch; ++k) bq[k] = (on && 1 + k < T) ? lb[(int64_t)(1 + k) * ld + j] : 0.0f;
    float d = on ? (a.log_pi ? a.log_pi[j] + lb[j] : lb[j]) : -INFINITY;
    uint16_t* psi = a.psi16 + sq.psi_off;
    int32_t cur = 0;
    for (int32_t t = 1; t < T; ++t) {
        const float bt = bq[0];
#pragma unroll
        for (int k = 0; k + 1 < kSmallPrefetch; ++k) bq[k] = bq[k + 1];
        bq[kSmallPrefetch - 1] = (on && t + kSmallPrefetch < T) ? lb[(int64_t)(t + kSmallPrefetch) * ld + j] : 0.0f;
        dsh[cur][j] = d;
        __syncthreads();
        float b0 = -INFINITY, b1 = -INFINITY;
        int32_t a0 = 0, a1 = 0;
#pragma unroll
        for (int i = 0; i < KMAX; i += 4) {
            const float4 v = *reinterpret_cast<const float4*>(&dsh[cur][i]);
            const float x0 = v.x + col[i], x1 = v.y + col[i + 1], x2 = v.z + col[i + 2], x3 = v.w + col[i + 3];
            if (x0 > b0) { b0 = x0; a0 = i; }
            if (x1 > b1) { b1 = x1; a1 = i + 1; }
            if (x2 > b0) { b0 = x2; a0 = i + 2; }
            if (x3 > b1) { b1 = x3; a1 = i + 3; }
        }
        if (b1 > b0 || (b1 == b0 && a1 < a0)) { b0 = b1; a0 = a1; }
        if (on) psi[(int64_t)t * K + j] = (uint16_t)a0;
        d = on ? b0 + bt : -INFINITY;
        cur ^= 1;
    }
    // final state: the lowest index of the largest score (-0 and +0 equal)
    unsigned long long key = on ? order_key(d, j) : 0ull;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        if (o > key) key = o;
    }
    if ((j & 63) == 0) wkey[j >> 6] = key;
    dsh[cur][j] = d;
    __syncthreads();
    key = wkey[0];
#pragma unroll
    for (int w = 1; w < KMAX / 64; ++w) key = wkey[w] > key ? wkey[w] : key;
    const int32_t qT = clampi((int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull)), K);
    const float sc = dsh[cur][qT];
    if (sc == -INFINITY) {
        for (int32_t t = j; t < T; t += KMAX) sq.path[t] = -1;
        if (j == 0) {
            *sq.score = sc;
            sq.status = FV_E_INFEASIBLE;
        }
        return;
    }
    if (j == 0) {
        *sq.score = sc;
        sq.path[T - 1] = qT;
        int32_t q = qT;
        for (int32_t t = T - 1; t > 0; --t) {
            q = clampi(psi[(int64_t)t * K + q], K);
            sq.path[t - 1] = q;
        }
    }
}

extern "C" __global__ __launch_bounds__(128) void fv_small_vanilla128_kernel(const EngineArgs* __restrict__ table) {
    small_vanilla_waves<128>(table);
}

extern "C" __global__ __launch_bounds__(256) void fv_small_vanilla256_kernel(const EngineArgs* __restrict__ table) {
    small_vanilla_waves<256>(table);
}

// ---------------------------------------------------------------- small single FLASH decode
// FLASH (Alg. 1 and 2, Sec. V-A/V-B) for sequences of a dense model with
// K <= 64, one wave (block) per sequence, with the persistent engine's task
// structure, so the decode keeps the method's O(P K) state.  State s lives
// in lane s, which holds s's column of log A; each step reads the previous
// scores from the other lanes, as in the one-wave vanilla kernel.
// (64 < K <= kSmallFlashK runs two waves per sequence, below.)
//   - Root pass over the whole sequence: each state keeps MidState (the state
//     at the most recent division point on its best path) and, at each
//     division point e_d (d <= P'-2), stores its score and, for d >= 1, its
//     MidState (the link to e_{d-1}) in the sequence's root copies.
//   - The first-level segments are then taken from the last to the first,
//     following the links back from q*_{T-1}; each segment's subtasks run
//     depth first from a stack in LDS.  A subtask (m, n) starts from the
//     single state q*_{m-1} with its carried score (the relative start drops
//     the score, as the engine's does), tracks MidState from t_mid + 1 and
//     yields q*_{t_mid}; its children are (m, t_mid) and (t_mid + 1, n).
//   - Subtasks of at most the engine's leaf length (and kSmallLeafRows) keep
//     their steps' backpointers in LDS and are walked back from q*_n.
// Ties and the final arg max follow the engine's rules, so the path and the
// score equal the engine's FLASH decode bit for bit.
constexpr int32_t kSmallLeafRows = 128;
constexpr int32_t kSmallStack = 64;

struct SmallTask {
    int32_t m, n, q_prev, q_n;
    float alpha;
};

// Per-lane state of the one-wave FLASH kernel: NJ destinations per lane.
template <int KMAX_>
struct SmallWave {
    static constexpr int32_t KMAX = KMAX_;
    static constexpr int NJ = KMAX > 64 ? 2 : 1;
    int32_t lane, K;
    bool on[NJ];
    float col[NJ][KMAX];
    float bq[NJ][kSmallPrefetch];
    gfloat_t* lb;
    int64_t ld;

    // emission scores of steps t0.. of a pass ending at n, kSmallPrefetch rows in flight
    __device__ __forceinline__ void ring_start(int32_t t0, int32_t n) {
#pragma unroll
        for (int c = 0; c < NJ; ++c)
#pragma unroll
            for (int k = 0; k < kSmallPrefetch; ++k)
                bq[c][k] = (on[c] && t0 + k <= n) ? lb[(int64_t)(t0 + k) * ld + lane + 64 * c] : 0.0f;
    }
    // one step at t of a pass ending at n: first maximum over predecessors
    // of d_i + log A(i, j), its own value kept, + log B_t(j)
    __device__ __forceinline__ void step(float (&d)[NJ], int32_t (&arg)[NJ], int32_t t, int32_t n) {
        float bt[NJ], best[NJ];
#pragma unroll
        for (int c = 0; c < NJ; ++c) {
            bt[c] = bq[c][0];
#pragma unroll
            for (int k = 0; k + 1 < kSmallPrefetch; ++k) bq[c][k] = bq[c][k + 1];
            bq[c][kSmallPrefetch - 1] =
                (on[c] && t + kSmallPrefetch <= n) ? lb[(int64_t)(t + kSmallPrefetch) * ld + lane + 64 * c] : 0.0f;
        }
        small_candidates<KMAX, NJ>(col, d, best, arg);
#pragma unroll
        for (int c = 0; c < NJ; ++c) d[c] = on[c] ? best[c] + bt[c] : -INFINITY;
    }
};

// v of state s (s < 64 * NJ), for every lane's own s
template <int NJ, typename V>
__device__ __forceinline__ V small_at(const V (&v)[NJ], int32_t s) {
    V r = __shfl(v[0], s & 63, 64);
    if (NJ > 1) {
        const V hi = __shfl(v[NJ - 1], s & 63, 64);
        if (s >= 64) r = hi;
    }
    return r;
}

template <int KMAX>
__device__ __forceinline__ void small_flash(cargs_t& a, SeqInfo& sq, uint16_t* leaf_tab, SmallTask* stack) {
    const int32_t K = a.K, T = sq.T, pp = sq.pp;
    constexpr int NJ = SmallWave<KMAX>::NJ;
    SmallWave<KMAX> w;
    w.lane = threadIdx.x;
    w.K = K;
    w.lb = as_global(sq.log_b);
    w.ld = sq.ld;
    const int32_t lane = w.lane;
#pragma unroll
    for (int c = 0; c < NJ; ++c) w.on[c] = lane + 64 * c < K;
#pragma unroll
    for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            w.col[c][i] = (w.on[c] && i < K) ? a.Acol[(int64_t)i * a.Kp + lane + 64 * c] : -INFINITY;
    int32_t* path = sq.path;
    const int32_t leaf_max = a.leaf_len < kSmallLeafRows ? a.leaf_len : kSmallLeafRows;
    float d0[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        const int32_t j = lane + 64 * c;
        d0[c] = w.on[c] ? (a.log_pi ? a.log_pi[j] + w.lb[j] : w.lb[j]) : -INFINITY;
    }
    float* const dsnap = a.root_copy + sq.root_off * (int64_t)a.Kp;                     // [pp-1][Kp]
    int32_t* const link = reinterpret_cast<int32_t*>(dsnap + (int64_t)(pp - 1) * a.Kp);  // [pp-1][Kp]

    // ---- root pass
    float d[NJ];
    int32_t mid[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) { d[c] = d0[c]; mid[c] = 0; }
    int32_t d_next = 0;
    const int64_t e0 = pp > 1 ? seg_end(T, pp, 0) : (int64_t)T;
    if (pp > 1 && e0 == 0) {
#pragma unroll
        for (int c = 0; c < NJ; ++c)
            if (w.on[c]) dsnap[lane + 64 * c] = d[c];
        d_next = 1;
    }
    int64_t e_prev = d_next >= 1 ? 0 : -1;
    int64_t e_next = d_next < pp - 1 ? seg_end(T, pp, d_next) : -1;
    w.ring_start(1, T - 1);
    for (int32_t t = 1; t < T; ++t) {
        int32_t pre[NJ];
        w.step(d, pre, t, T - 1);
        if (d_next >= 1 && e_prev == t - 1) {
#pragma unroll
            for (int c = 0; c < NJ; ++c) mid[c] = pre[c];
        } else if (pp > 1 && t > e0 + 1) {
            int32_t nm[NJ];
#pragma unroll
            for (int c = 0; c < NJ; ++c) nm[c] = small_at<NJ>(mid, pre[c]);
#pragma unroll
            for (int c = 0; c < NJ; ++c) mid[c] = nm[c];
        }
        if (e_next == t) {
#pragma unroll
            for (int c = 0; c < NJ; ++c) {
                if (w.on[c]) {
                    dsnap[(int64_t)d_next * a.Kp + lane + 64 * c] = d[c];
                    if (d_next >= 1) link[(int64_t)d_next * a.Kp + lane + 64 * c] = mid[c];
                }
            }
            e_prev = t;
            ++d_next;
            e_next = d_next < pp - 1 ? seg_end(T, pp, d_next) : -1;
        }
    }
    unsigned long long key = 0;
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        const unsigned long long k = w.on[c] ? order_key(d[c], lane + 64 * c) : 0ull;
        if (k > key) key = k;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        if (o > key) key = o;
    }
    const int32_t qT = clampi((int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull)), K);
    const float sc = small_at<NJ>(d, qT);
    if (sc == -INFINITY) {
        for (int32_t t = lane; t < T; t += 64) path[t] = -1;
        if (lane == 0) {
            *sq.score = sc;
            sq.status = FV_E_INFEASIBLE;
        }
        return;
    }
    if (lane == 0) {
        *sq.score = sc;
        path[T - 1] = qT;
    }
    const int32_t q_last_div = small_at<NJ>(mid, qT);   // q* at e_{P'-2}
    __syncthreads();   // the division copies are read back across lanes below

    // ---- first-level segments, last to first, each with its subtasks
    int32_t qe = qT;
    for (int32_t ds = pp - 1; ds >= 0; --ds) {
        const int32_t n0 = (int32_t)seg_end(T, pp, ds);
        const int32_t m0 = ds == 0 ? 0 : (int32_t)seg_end(T, pp, ds - 1) + 1;
        int32_t qp = 0;
        float alpha = 0.0f;
        if (ds >= 1) {
            qp = ds == pp - 1 ? q_last_div : link[(int64_t)ds * a.Kp + qe];
            qp = clampi(qp, K);
            alpha = dsnap[(int64_t)(ds - 1) * a.Kp + qp];
            if (lane == 0) path[m0 - 1] = qp;
        }
        if (n0 - m0 >= 1) {
            if (lane == 0) stack[0] = SmallTask{m0, n0, qp, qe, alpha};
            int32_t sp = 1;
            __syncthreads();
            while (sp > 0) {
                const SmallTask tk = stack[--sp];
                const int32_t m = tk.m, n = tk.n;
                float x[NJ];
#pragma unroll
                for (int c = 0; c < NJ; ++c) {
                    x[c] = d0[c];
                    if (m > 0) {
                        const int32_t j = lane + 64 * c;
                        const float arow = w.on[c] ? a.Acol[(int64_t)tk.q_prev * a.Kp + j] : -INFINITY;
                        const float cc = a.relative_init ? arow : tk.alpha + arow;
                        x[c] = w.on[c] ? cc + w.lb[(int64_t)m * w.ld + j] : -INFINITY;
                    }
                }
                w.ring_start(m + 1, n);
                if (n - m + 1 <= leaf_max) {
                    for (int32_t t = m + 1; t <= n; ++t) {
                        int32_t pre[NJ];
                        w.step(x, pre, t, n);
#pragma unroll
                        for (int c = 0; c < NJ; ++c)
                            if (w.on[c]) leaf_tab[(t - m - 1) * KMAX + lane + 64 * c] = (uint16_t)pre[c];
                    }
                    __syncthreads();
                    if (lane == 0) {
                        int32_t q = tk.q_n;
                        for (int32_t t = n; t > m; --t) {
                            q = leaf_tab[(t - m - 1) * KMAX + q];
                            path[t - 1] = q;
                        }
                    }
                    __syncthreads();
                    continue;
                }
                const int32_t tmid = (m + n) / 2;
                float snap[NJ];
                int32_t md[NJ];
#pragma unroll
                for (int c = 0; c < NJ; ++c) { snap[c] = x[c]; md[c] = 0; }
                for (int32_t t = m + 1; t <= n; ++t) {
                    int32_t pre[NJ];
                    w.step(x, pre, t, n);
                    if (t == tmid + 1) {
#pragma unroll
                        for (int c = 0; c < NJ; ++c) md[c] = pre[c];
                    } else if (t > tmid + 1) {
                        int32_t nm[NJ];
#pragma unroll
                        for (int c = 0; c < NJ; ++c) nm[c] = small_at<NJ>(md, pre[c]);
#pragma unroll
                        for (int c = 0; c < NJ; ++c) md[c] = nm[c];
                    }
                    if (t == tmid) {
#pragma unroll
                        for (int c = 0; c < NJ; ++c) snap[c] = x[c];
                    }
                }
                const int32_t qmid = clampi(small_at<NJ>(md, tk.q_n), K);
                const float amid = small_at<NJ>(snap, qmid);
                if (n - m >= 2 && sp + 2 > kSmallStack) {   // deeper than any sequence of 2^31 steps needs
                    if (lane == 0) sq.status = FV_E_DEVICE;
                    return;
                }
                if (lane == 0) {
                    path[tmid] = qmid;
                    if (n - m > 2) {
                        stack[sp] = SmallTask{m, tmid, tk.q_prev, qmid, tk.alpha};
                        stack[sp + 1] = SmallTask{tmid + 1, n, qmid, tk.q_n, amid};
                    } else if (n - m == 2) {
                        stack[sp] = SmallTask{m, tmid, tk.q_prev, qmid, tk.alpha};
                    }
                }
                sp += n - m > 2 ? 2 : (n - m == 2 ? 1 : 0);
                __syncthreads();
            }
        }
        qe = qp;
    }
}

// One kernel per width (K <= 32, 64), so each gets the register allocation
// of its own step loop.
#define FV_SMALL_FLASH(NAME, KMAX)                                                                     \
    extern "C" __global__ __launch_bounds__(64) void NAME(const EngineArgs* __restrict__ table) {       \
        cargs_t& a = *reinterpret_cast<cargs_t*>(reinterpret_cast<uint64_t>(table));                    \
        if ((int32_t)blockIdx.x >= a.n_seqs) return;                                                    \
        SeqInfo& sq = a.seqs[blockIdx.x];                                                               \
        if (sq.status != FV_OK || sq.T <= 0 || a.K > KMAX || sq.pp < 1 || sq.pp > sq.T) return;         \
        __shared__ uint16_t leaf_tab[kSmallLeafRows * KMAX];                                            \
        __shared__ SmallTask stack[kSmallStack];                                                        \
        small_flash<KMAX>(a, sq, leaf_tab, stack);                                                      \
    }
FV_SMALL_FLASH(fv_small_flash32_kernel, 32)
FV_SMALL_FLASH(fv_small_flash64_kernel, 64)
#undef FV_SMALL_FLASH

// 64 < K <= 256: the same FLASH schedule with KMAX / 64 waves per sequence
// (KMAX = 128 or 256), thread j for state j (one column of log A in
// registers).  Each step
// publishes the scores and the tracked MidState in double-buffered LDS, so
// one barrier per step serves both the candidates and the MidState gather;
// one-off gathers (q* at a midpoint, its anchor score, the final state) go
// through LDS as well.  Every barrier is on block-uniform control flow.
template <int KMAX>
__device__ __forceinline__ void small_flash_waves(const EngineArgs* __restrict__ table) {
    cargs_t& a = *reinterpret_cast<cargs_t*>(reinterpret_cast<uint64_t>(table));
    if ((int32_t)blockIdx.x >= a.n_seqs) return;
    SeqInfo& sq = a.seqs[blockIdx.x];
    if (sq.status != FV_OK || sq.T <= 0 || a.K > KMAX || sq.pp < 1 || sq.pp > sq.T) return;
    __shared__ uint16_t leaf_tab[kSmallLeafRows * KMAX];
    __shared__ SmallTask stack[kSmallStack];
    __shared__ __align__(16) float dsh[2][KMAX];
    __shared__ int32_t msh[2][KMAX];
    __shared__ float xsh[KMAX];
    __shared__ int32_t ish[KMAX];
    __shared__ unsigned long long wkey[KMAX / 64];
    const int32_t K = a.K, T = sq.T, pp = sq.pp;
    const int32_t j = threadIdx.x;
    const bool on = j < K;
    gfloat_t* lb = as_global(sq.log_b);
    const int64_t ld = sq.ld;
    int32_t* path = sq.path;
    const int32_t leaf_max = a.leaf_len < kSmallLeafRows ? a.leaf_len : kSmallLeafRows;
    float col[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) col[i] = (on && i < K) ? a.Acol[(int64_t)i * a.Kp + j] : -INFINITY;
    const float d0 = on ? (a.log_pi ? a.log_pi[j] + lb[j] : lb[j]) : -INFINITY;
    float* const dsnap = a.root_copy + sq.root_off * (int64_t)a.Kp;                     // [pp-1][Kp]
    int32_t* const link = reinterpret_cast<int32_t*>(dsnap + (int64_t)(pp - 1) * a.Kp);  // [pp-1][Kp]
    float bq[kSmallPrefetch];
    auto ring_start = [&](int32_t t0, int32_t n) {
#pragma unroll
        for (int k = 0; k < kSmallPrefetch; ++k) bq[k] = (on && t0 + k <= n) ? lb[(int64_t)(t0 + k) * ld + j] : 0.0f;
    };
    auto ring_next = [&](int32_t t, int32_t n) {
        const float v = bq[0];
#pragma unroll
        for (int k = 0; k + 1 < kSmallPrefetch; ++k) bq[k] = bq[k + 1];
        bq[kSmallPrefetch - 1] = (on && t + kSmallPrefetch <= n) ? lb[(int64_t)(t + kSmallPrefetch) * ld + j] : 0.0f;
        return v;
    };
    // first maximum over the published scores dsh[c] (even and odd chains,
    // merged by value, equal values to the lower index)
    auto candidates = [&](int32_t c, int32_t& arg) {
        float b0 = -INFINITY, b1 = -INFINITY;
        int32_t a0 = 0, a1 = 0;
#pragma unroll
        for (int i = 0; i < KMAX; i += 4) {
            const float4 v = *reinterpret_cast<const float4*>(&dsh[c][i]);
            const float x0 = v.x + col[i], x1 = v.y + col[i + 1], x2 = v.z + col[i + 2], x3 = v.w + col[i + 3];
            if (x0 > b0) { b0 = x0; a0 = i; }
            if (x1 > b1) { b1 = x1; a1 = i + 1; }
            if (x2 > b0) { b0 = x2; a0 = i + 2; }
            if (x3 > b1) { b1 = x3; a1 = i + 3; }
        }
        if (b1 > b0 || (b1 == b0 && a1 < a0)) { b0 = b1; a0 = a1; }
        arg = a0;
        return b0;
    };
    int32_t cur = 0;

    // ---- root pass
    float d = d0;
    int32_t mid = 0;
    int32_t d_next = 0;
    const int64_t e0 = pp > 1 ? seg_end(T, pp, 0) : (int64_t)T;
    if (pp > 1 && e0 == 0) {
        if (on) dsnap[j] = d;
        d_next = 1;
    }
    int64_t e_prev = d_next >= 1 ? 0 : -1;
    int64_t e_next = d_next < pp - 1 ? seg_end(T, pp, d_next) : -1;
    ring_start(1, T - 1);
    for (int32_t t = 1; t < T; ++t) {
        const float bt = ring_next(t, T - 1);
        dsh[cur][j] = d;
        msh[cur][j] = mid;
        __syncthreads();
        int32_t pre;
        const float best = candidates(cur, pre);
        if (d_next >= 1 && e_prev == t - 1) mid = pre;
        else if (pp > 1 && t > e0 + 1) mid = msh[cur][pre];
        d = on ? best + bt : -INFINITY;
        if (e_next == t) {
            if (on) {
                dsnap[(int64_t)d_next * a.Kp + j] = d;
                if (d_next >= 1) link[(int64_t)d_next * a.Kp + j] = mid;
            }
            e_prev = t;
            ++d_next;
            e_next = d_next < pp - 1 ? seg_end(T, pp, d_next) : -1;
        }
        cur ^= 1;
    }
    unsigned long long key = on ? order_key(d, j) : 0ull;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        if (o > key) key = o;
    }
    if ((j & 63) == 0) wkey[j >> 6] = key;
    dsh[cur][j] = d;
    msh[cur][j] = mid;
    __syncthreads();   // also orders the division copies before they are read back
    key = wkey[0];
#pragma unroll
    for (int w = 1; w < KMAX / 64; ++w) key = wkey[w] > key ? wkey[w] : key;
    const int32_t qT = clampi((int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull)), K);
    const float sc = dsh[cur][qT];
    const int32_t q_last_div = msh[cur][qT];   // q* at e_{P'-2}
    cur ^= 1;
    if (sc == -INFINITY) {
        for (int32_t t = j; t < T; t += KMAX) path[t] = -1;
        if (j == 0) {
            *sq.score = sc;
            sq.status = FV_E_INFEASIBLE;
        }
        return;
    }
    if (j == 0) {
        *sq.score = sc;
        path[T - 1] = qT;
    }

    // ---- first-level segments, last to first, each with its subtasks
    int32_t qe = qT;
    for (int32_t ds = pp - 1; ds >= 0; --ds) {
        const int32_t n0 = (int32_t)seg_end(T, pp, ds);
        const int32_t m0 = ds == 0 ? 0 : (int32_t)seg_end(T, pp, ds - 1) + 1;
        int32_t qp = 0;
        float alpha = 0.0f;
        if (ds >= 1) {
            qp = ds == pp - 1 ? q_last_div : link[(int64_t)ds * a.Kp + qe];
            qp = clampi(qp, K);
            alpha = dsnap[(int64_t)(ds - 1) * a.Kp + qp];
            if (j == 0) path[m0 - 1] = qp;
        }
        if (n0 - m0 >= 1) {
            __syncthreads();   // earlier readers of stack[0] are done
            if (j == 0) stack[0] = SmallTask{m0, n0, qp, qe, alpha};
            int32_t sp = 1;
            __syncthreads();
            while (sp > 0) {
                const SmallTask tk = stack[--sp];
                const int32_t m = tk.m, n = tk.n;
                float x = d0;
                if (m > 0) {
                    const float arow = on ? a.Acol[(int64_t)tk.q_prev * a.Kp + j] : -INFINITY;
                    const float cc = a.relative_init ? arow : tk.alpha + arow;
                    x = on ? cc + lb[(int64_t)m * ld + j] : -INFINITY;
                }
                ring_start(m + 1, n);
                if (n - m + 1 <= leaf_max) {
                    for (int32_t t = m + 1; t <= n; ++t) {
                        const float bt = ring_next(t, n);
                        dsh[cur][j] = x;
                        __syncthreads();
                        int32_t pre;
                        const float best = candidates(cur, pre);
                        x = on ? best + bt : -INFINITY;
                        if (on) leaf_tab[(t - m - 1) * KMAX + j] = (uint16_t)pre;
                        cur ^= 1;
                    }
                    __syncthreads();
                    if (j == 0) {
                        int32_t q = tk.q_n;
                        for (int32_t t = n; t > m; --t) {
                            q = leaf_tab[(t - m - 1) * KMAX + q];
                            path[t - 1] = q;
                        }
                    }
                    __syncthreads();
                    continue;
                }
                const int32_t tmid = (m + n) / 2;
                float snap = x;
                int32_t md = 0;
                for (int32_t t = m + 1; t <= n; ++t) {
                    const float bt = ring_next(t, n);
                    dsh[cur][j] = x;
                    msh[cur][j] = md;
                    __syncthreads();
                    int32_t pre;
                    const float best = candidates(cur, pre);
                    if (t == tmid + 1) md = pre;
                    else if (t > tmid + 1) md = msh[cur][pre];
                    x = on ? best + bt : -INFINITY;
                    if (t == tmid) snap = x;
                    cur ^= 1;
                }
                ish[j] = md;
                xsh[j] = snap;
                __syncthreads();
                const int32_t qmid = clampi(ish[tk.q_n], K);
                const float amid = xsh[qmid];
                if (n - m >= 2 && sp + 2 > kSmallStack) {   // deeper than any sequence of 2^31 steps needs
                    if (j == 0) sq.status = FV_E_DEVICE;
                    return;
                }
                if (j == 0) {
                    path[tmid] = qmid;
                    if (n - m > 2) {
                        stack[sp] = SmallTask{m, tmid, tk.q_prev, qmid, tk.alpha};
                        stack[sp + 1] = SmallTask{tmid + 1, n, qmid, tk.q_n, amid};
                    } else if (n - m == 2) {
                        stack[sp] = SmallTask{m, tmid, tk.q_prev, qmid, tk.alpha};
                    }
                }
                sp += n - m > 2 ? 2 : (n - m == 2 ? 1 : 0);
                __syncthreads();
            }
        }
        qe = qp;
    }
}

extern "C" __global__ __launch_bounds__(128) void fv_small_flash128_kernel(const EngineArgs* __restrict__ table) {
    small_flash_waves<128>(table);
}

extern "C" __global__ __launch_bounds__(256) void fv_small_flash256_kernel(const EngineArgs* __restrict__ table) {
    small_flash_waves<256>(table);
}

// ---------------------------------------------------------------- preparation kernel
// Ap[i][j] = log A(i, j) on a Kp x Kp grid, -inf outside K x K (only used
// when K is not a multiple of the padding granularity).
extern "C" __global__ __launch_bounds__(kBlock) void fv_prep_dense_kernel(const float* __restrict__ log_a,
                                                                          int32_t K, int32_t Kp,
                                                                          float* __restrict__ Ap) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)Kp * Kp) return;
    const int32_t i = (int32_t)(idx / Kp), j = (int32_t)(idx - (int64_t)i * Kp);
    Ap[idx] = (i < K && j < K) ? log_a[(int64_t)i * K + j] : -INFINITY;
}

// At[j * Kp + i] = Ap[i * Kp + j]: the transposed (column-major) copy of the
// padded log A, read by the two-column items' refine.  64 x 64 tiles through
// LDS, 256 threads per tile; grid (Kp / 64, Kp / 64).
extern "C" __global__ __launch_bounds__(kBlock) void fv_transpose_dense_kernel(const float* __restrict__ Ap,
                                                                               int32_t Kp, float* __restrict__ At) {
    __shared__ float tile[64][65];
    const int32_t i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int32_t c = threadIdx.x & 63, r4 = threadIdx.x >> 6;
    for (int32_t r = r4; r < 64; r += 4) tile[r][c] = Ap[(int64_t)(i0 + r) * Kp + j0 + c];
    __syncthreads();
    for (int32_t r = r4; r < 64; r += 4) At[(int64_t)(j0 + r) * Kp + i0 + c] = tile[c][r];
}

// Per-sequence setup and the first step's row list (one block).  The
// decode covers the sequences of the caller's array whose model index is
// sa.model, in their order; their local index is their rank among them.
extern "C" __global__ __launch_bounds__(kBlock) void fv_setup_kernel(EngineArgs a, SetupArgs sa) {
    if (threadIdx.x == 0) *sa.args_out = a;
    __shared__ int64_t scan[4][kBlock];
    __shared__ int32_t s_bad;
    const int tid = threadIdx.x;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    int64_t base[4] = {0, 0, 0, 0};
    for (int32_t b0 = 0; b0 < sa.n_seqs; b0 += kBlock) {
        const int32_t b = b0 + tid;
        int64_t v[4] = {0, 0, 0, 0};
        fv_seq d{};
        int32_t pp = 1;
        const bool member = b < sa.n_seqs && (d = sa.seqs_dev[b]).model == sa.model;
        if (member) {
            const bool table = sa.emit_kind == FV_EMIT_TABLE;   // else log_b addresses observations
            if (d.T < 0 || (d.T > 0 && ((table && d.ld < sa.K) || !d.log_b || !d.path)) || !d.score) s_bad = 1;
            const int32_t T = d.T < 0 ? 0 : d.T;
            pp = sa.kind == KIND_VANILLA ? 1 : eff_parallelism(T, sa.P);
            v[0] = T;
            // root division copies: delta + link per division (dense), one beam record (beam)
            v[1] = sa.kind == KIND_ROOT ? 2 * (int64_t)(pp - 1) : (sa.kind == KIND_BROOT ? (int64_t)(pp - 1) : 0);
            v[2] = sa.kind == KIND_VANILLA ? (int64_t)T * sa.K : 0;
            v[3] = 1;
        }
        for (int k = 0; k < 4; ++k) scan[k][tid] = v[k];
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            int64_t add[4];
            for (int k = 0; k < 4; ++k) add[k] = tid >= off ? scan[k][tid - off] : 0;
            __syncthreads();
            for (int k = 0; k < 4; ++k) scan[k][tid] += add[k];
            __syncthreads();
        }
        const int64_t li = base[3] + scan[3][tid] - v[3];
        if (member && li < sa.n_local) {   // more members than the host counted: reported below
            SeqInfo si;
            si.log_b = d.log_b; si.ld = sa.emit_kind == FV_EMIT_TABLE ? d.ld : 0; si.path = d.path; si.score = d.score;
            si.T = d.T < 0 ? 0 : d.T;
            si.pp = pp;
            si.alpha_off = base[0] + scan[0][tid] - v[0];
            si.root_off = base[1] + scan[1][tid] - v[1];
            si.psi_off = base[2] + scan[2][tid] - v[2];
            si.status = FV_OK;
            si.orig = b;
            a.seqs[li] = si;
            a.keys[li] = 0ull;
            if (si.T == 0 && d.score) *d.score = 0.0f;
        }
        for (int k = 0; k < 4; ++k) base[k] += scan[k][kBlock - 1];
        __syncthreads();
    }
    if (base[0] != sa.host_sum_T || base[1] != sa.host_sum_root || base[2] != sa.host_sum_psi ||
        base[3] != sa.n_local)
        s_bad = 1;
    __syncthreads();
    const bool bad = s_bad != 0;
    const int32_t n_local = (int32_t)(base[3] < sa.n_local ? base[3] : sa.n_local);
    // task queue: every non-empty sequence's full-length pass
    int32_t n_tasks = 0;
    for (int32_t b0 = 0; b0 < n_local; b0 += kBlock) {
        const int32_t b = b0 + tid;
        int32_t has = 0;
        if (b < n_local) {
            if (bad) a.seqs[b].status = FV_E_INVALID_ARG;
            has = (!bad && a.seqs[b].T > 0) ? 1 : 0;
        }
        scan[0][tid] = has;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const int64_t add = tid >= off ? scan[0][tid - off] : 0;
            __syncthreads();
            scan[0][tid] += add;
            __syncthreads();
        }
        if (has) a.queue[n_tasks + scan[0][tid] - 1] = Task{b, sa.kind, 0, a.seqs[b].T - 1};
        n_tasks += (int32_t)scan[0][kBlock - 1];
        __syncthreads();
    }
    // longest tasks first (ties by sequence index), when they fit one LDS sort:
    // together with the round-robin admission this spreads the lengths, and
    // so the rows over time, evenly over the XCDs (any order gives the same
    // results)
    constexpr int32_t kSortMax = 4096;
    if (n_tasks > 1 && n_tasks <= kSortMax) {
        __shared__ unsigned long long skey[kSortMax];
        int32_t n2 = 1;
        while (n2 < n_tasks) n2 <<= 1;
        for (int32_t k = tid; k < n2; k += kBlock) {
            unsigned long long key = ~0ull;
            if (k < n_tasks) {
                const Task tk = a.queue[k];
                key = ((unsigned long long)(uint32_t)(0x7fffffff - (tk.n - tk.m)) << 32) | (uint32_t)tk.seq;
            }
            skey[k] = key;
        }
        __syncthreads();
        for (int32_t k = 2; k <= n2; k <<= 1) {
            for (int32_t h = k >> 1; h > 0; h >>= 1) {
                for (int32_t i = tid; i < n2; i += kBlock) {
                    const int32_t l = i ^ h;
                    if (l > i) {
                        const unsigned long long u = skey[i], v = skey[l];
                        if ((u > v) == ((i & k) == 0)) { skey[i] = v; skey[l] = u; }
                    }
                }
                __syncthreads();
            }
        }
        for (int32_t k = tid; k < n_tasks; k += kBlock) {
            const int32_t b = (int32_t)(uint32_t)skey[k];
            a.queue[k] = Task{b, sa.kind, 0, a.seqs[b].T - 1};
        }
        __syncthreads();
    }
    // local sequences the setup never reached (fewer members than the host counted)
    for (int32_t b = n_local + tid; b < sa.n_local; b += kBlock) {
        SeqInfo si{};
        si.status = FV_E_INVALID_ARG;
        si.orig = -1;
        a.seqs[b] = si;
    }
    // slot pools: pool x holds slots x, x + kXcd, ... (free stack order is irrelevant)
    for (int32_t k = tid; k < a.n_slots; k += kBlock) {
        const int32_t x = k % kXcd, i = k / kXcd;
        a.free_stack[(int64_t)x * a.pool + i] = k;
    }
    EngineState* st = a.st;
    int32_t* words = reinterpret_cast<int32_t*>(st);
    for (int32_t k = tid; k < (int32_t)(sizeof(EngineState) / 4); k += kBlock) words[k] = 0;
    for (int32_t k = tid; k < a.n_compute_blocks + 1; k += kBlock) a.arrive[k] = 0;
    __syncthreads();
    if (tid == 0) st->q_tail0 = n_tasks;
}

// Sequences whose model index is outside [0, n_models) belong to no decode.
extern "C" __global__ __launch_bounds__(kBlock) void fv_model_check_kernel(const fv_seq* seqs_dev, int32_t n_seqs,
                                                                           int32_t n_models, int32_t* status) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= n_seqs) return;
    const int32_t m = seqs_dev[b].model;
    if (m < 0 || m >= n_models) status[b] = FV_E_INVALID_ARG;
}

// Vanilla backtracking through the packed table and per-sequence status.
extern "C" __global__ __launch_bounds__(kBlock) void fv_finish_kernel(EngineArgs a, int32_t* status) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= a.n_seqs) return;
    SeqInfo& sq = a.seqs[b];
    int32_t stv = sq.status;
    if (a.st->error) stv = FV_E_DEVICE;  // kernel boundary: plain load is coherent
    if (a.sparse && stv != FV_E_DEVICE && sq.T > 0) {   // malformed CSR input outranks what it caused
        const int32_t fl = *a.csr_flag;
        if (fl & kCsrInvalid) stv = FV_E_INVALID_ARG;
        else if ((fl & kCsrWideIn) && a.method == FV_VANILLA) stv = FV_E_UNSUPPORTED;
    }
    if (a.bad_model && stv != FV_E_DEVICE && sq.T > 0 && sq.orig >= 0 && (*a.bad_model || a.bad_seq[sq.orig]))
        stv = FV_E_INVALID_ARG;
    if (stv == FV_OK && a.method == FV_VANILLA && sq.T > 1 && !a.path_done) {
        int32_t q = sq.path[sq.T - 1];
        const uint16_t* tab = a.psi16 + sq.psi_off;
        for (int32_t t = sq.T - 1; t > 0; --t) {
            const int32_t v = tab[(int64_t)t * a.K + q];
            if (a.sparse) {   // v is the slot of q's winning in-edge
                const int32_t e0 = a.in_ptr[q], e1 = a.in_ptr[q + 1];
                q = e1 > e0 ? a.in_src[min(e0 + v, e1 - 1)] : 0;
            } else {
                q = v;
            }
            sq.path[t - 1] = q;
        }
    }
    if (status && sq.orig >= 0) status[sq.orig] = stv;
}

// Beam decodes: status, and the returned score as the step-by-step float32
// re-sum of the returned path, s_0 = log pi(q_0) + log B_0(q_0),
// s_t = (s_{t-1} + log A(q_{t-1}, q_t)) + log B_t(q_t).  One wave per
// sequence: the terms are gathered 64 at a time, then added in order.
extern "C" __global__ __launch_bounds__(kBlock) void fv_beam_finish_kernel(EngineArgs a, const float* __restrict__ Ap,
                                                                           int32_t* status) {
    const int32_t b = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int32_t lane = threadIdx.x & 63;
    if (b >= a.n_seqs) return;
    SeqInfo& sq = a.seqs[b];
    int32_t stv = sq.status;
    if (a.st->error) stv = FV_E_DEVICE;  // kernel boundary: plain loads are coherent
    if (a.sparse && stv != FV_E_DEVICE && sq.T > 0 && (*a.csr_flag & kCsrInvalid)) stv = FV_E_INVALID_ARG;
    if (a.bad_model && stv != FV_E_DEVICE && sq.T > 0 && sq.orig >= 0 && (*a.bad_model || a.bad_seq[sq.orig]))
        stv = FV_E_INVALID_ARG;
    if (stv >= 0 && sq.T >= 1) {
        const int32_t K = a.K, Kp = a.Kp, T = sq.T;
        const int32_t q0 = sq.path[0];
        bool ok = q0 >= 0 && q0 < K;
        float s = -INFINITY;
        if (ok) {
            const float e = emission_of(a.emit_kind, a.emit_xy, a.emit_c2, a.emit_c0, sq.log_b, sq.ld, 0, q0);
            s = a.log_pi ? a.log_pi[q0] + e : e;
        }
        for (int32_t t0 = 1; ok && t0 < T; t0 += 64) {
            const int32_t t = t0 + lane;
            float ta = 0.0f, tb = 0.0f;
            int32_t bad = 0;
            if (t < T) {
                const int32_t qp = sq.path[t - 1], q = sq.path[t];
                if (qp < 0 || qp >= K || q < 0 || q >= K) {
                    bad = 1;
                } else {
                    if (a.sparse) {   // largest of the edges qp -> q, -inf without one
                        int32_t e0, e1;
                        sp_out_range(a.row_ptr, a.nnz, qp, e0, e1);
                        ta = -INFINITY;
                        bool found = false;
                        for (int32_t e = e0; e < e1; ++e) {
                            if (a.col[e] != q) continue;
                            if (!found || a.val[e] > ta) { ta = a.val[e]; found = true; }
                        }
                    } else {
                        ta = Ap[(int64_t)qp * Kp + q];
                    }
                    tb = emission_of(a.emit_kind, a.emit_xy, a.emit_c2, a.emit_c0, sq.log_b, sq.ld, t, q);
                }
            }
            if (__ballot(bad) != 0) { ok = false; break; }
            const int32_t cnt = min(64, T - t0);
            for (int32_t l = 0; l < cnt; ++l) {
                const float x = __shfl(ta, l, 64), y = __shfl(tb, l, 64);
                const float c = s + x;
                s = c + y;
            }
        }
        if (!ok) s = -INFINITY;
        if (lane == 0) *sq.score = s;
    }
    if (lane == 0 && status && sq.orig >= 0) status[sq.orig] = stv;
}

}  // namespace fv
