// Internal layout shared by the host API and the device kernels of the
// FLASH Viterbi library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/flashviterbi.h"

// Records the thread-local message fv_last_error() returns; returns s.
fv_status fv_set_error(fv_status s, const char* msg, ...) __attribute__((format(printf, 2, 3)));

namespace fv {

constexpr int kBlock = 256;     // threads per workgroup (4 wave64)
constexpr int kWaves = 4;
constexpr int kTileRows = 64;   // rows of a dense tile: one per lane
constexpr int kTileCols = 16;   // destination columns per dense tile
constexpr int kGroup = 16;      // predecessors per arg-max group
constexpr int kKAlign = 64;     // K is padded to a multiple of this

inline __host__ __device__ int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Kinds of rows (one row = one decoding task in flight).  KIND_BROOT and
// KIND_BSUB are FLASH-BS (beam) tasks; KIND_FSUB is the exact (all-K)
// re-decode of a beam subtask whose beam lost its known end state: it runs
// as a dense subtask and its children are beam subtasks again.
enum : int32_t { KIND_VANILLA = 0, KIND_ROOT = 1, KIND_SUB = 2, KIND_BROOT = 3, KIND_BSUB = 4, KIND_FSUB = 5 };

inline __host__ __device__ bool is_dense_sub(int32_t kind) { return kind == KIND_SUB || kind == KIND_FSUB; }
inline __host__ __device__ bool is_beam(int32_t kind) { return kind == KIND_BROOT || kind == KIND_BSUB; }

// Per-step flags of a dense row.
enum : int32_t {
    F_NEED_ARG = 1 << 0,   // psi is needed this step
    F_ANC_FIRST = 1 << 1,  // anc_t(j) = psi_t(j)
    F_ANC_CHAIN = 1 << 2,  // anc_t(j) = anc_{t-1}(psi_t(j))
    F_PSI_TABLE = 1 << 3,  // store psi_t in the vanilla table
    F_SNAP_SUB = 1 << 4,   // copy delta_t to the row's snapshot (t = t_mid)
    F_SNAP_ROOT = 1 << 5,  // copy delta_t (and anc_t) to the root's division copy aux
    F_FINAL = 1 << 6,      // t = T-1 of a full-length pass: feed the final arg max
    F_START = 1 << 7,      // sparse rows: this step computes the task's start vector
    F_LEAF_TABLE = 1 << 8, // leaf subtask: store psi_t in the slot's leaf table, row aux (= t - m)
    F_SNAP_DIV = 1 << 9,   // w-way subtask: copy delta_t (and anc_t) to the slot's division copy aux
};

// w-way subtasks.  With leaves off (K above kLeafMaxKp) and wide rows, a
// FLASH subtask [m, n] is split like the root: w' = min(kWSplit, n - m + 1)
// segments of its positions, division ends e_k = m + floor(((k+1) L - 1) / w')
// (L = n - m + 1, k < w' - 1), snapshots of delta and of the division chain
// at each e_k in its row buffer, all w' - 1 division states resolved at its
// end, and one child per segment of at least two positions.  w' = 2 is
// Alg. 1's bisection; every position is still resolved exactly once.
constexpr int32_t kWSplit = 8;
inline __host__ __device__ int32_t sub_parts(int32_t m, int32_t n, int32_t w) {
    const int32_t L = n - m + 1;
    return L < w ? L : w;
}

// Light (O(K)) operations.  L_BSPAWN does nothing: it holds a finished
// beam subtask for one step so that the scheduler, which classifies a
// step's rows while they run, reads the task's fallback flag after the
// step that wrote it.
enum : int32_t { L_INIT = 0, L_END = 1, L_FINALIZE = 2, L_BSPAWN = 3, L_LEAF_END = 4 };

// Leaf subtasks.  A FLASH subtask of at most kLeafLen steps is not bisected
// further: its forward pass keeps a small backpointer table (uint16, one row
// per step) in its slot, and its end step walks that table back from the
// known end state, resolving every position of the segment at once.  The
// anchored start makes its pointers along the path equal vanilla's, so the
// result is unchanged; the subtask tree loses its lower levels.
constexpr int32_t kLeafLen = 128;
constexpr int32_t kLeafMaxKp = 2048;   // larger K: no leaves (table too large per slot)

// Column items of two destinations per lane stage their rows' scores whole
// in LDS and refine from a transposed copy of log A: up to this Kp.
constexpr int32_t kColMaxKp = 4096;

// One vanilla decode of a dense model with K <= kSmallK runs on one wave
// instead of the persistent engine.
constexpr int32_t kSmallK = 256;
// One FLASH decode of a dense model with K <= kSmallFlashK runs on one wave too.
constexpr int32_t kSmallFlashK = 256;

// Operations of a beam row (one block each): start step, full beam step,
// end-only step of a subtask, final selection of a root.
enum : int32_t { B_INIT = 0, B_STEP = 1, B_END = 2, B_FINAL = 3 };
constexpr int32_t kBeamMaxK = 16384;   // scores of one step live in LDS
constexpr int32_t kBeamMaxB = 2048;

// Sparse models.  Vanilla backpointers of a sparse model hold the winning
// in-edge's slot within its destination's list (uint16), so a destination
// may have at most kMaxInSlot + 1 in-edges there.  A sparse beam step
// pushes the out-edges of its beam states: at most kSpCandMax candidates.
constexpr int32_t kMaxInSlot = 65535;
constexpr int32_t kSpCandMax = 4096;
enum : int32_t { kCsrInvalid = 1, kCsrWideIn = 2, kCsrBeamCands = 4 };

// A task in flight; carries what every step needs so that tiles do not
// look up the per-sequence table.
struct Row {
    int32_t seq;
    int32_t kind;
    int32_t m, n;      // segment [m, n]
    int32_t t;         // time step this row computes at the current global step
    int32_t slot;      // buffer slot
    int32_t flags;     // F_* (dense rows)
    int32_t aux;       // L_* for light rows; division index for F_SNAP_ROOT
    int32_t T, pp;     // sequence length and effective parallelism
    int64_t off;       // vanilla: backpointer table offset; root: division copy offset
    const float* log_b;
    int64_t ld;
};

struct Task {
    int32_t seq, kind, m, n;
};

struct SeqInfo {
    const float* log_b;
    int64_t ld;
    int32_t* path;
    float* score;
    int32_t T;
    int32_t pp;          // effective parallelism P'
    int64_t alpha_off;   // into alpha_at
    int64_t root_off;    // into root copies, in units (Kp floats, or one beam record)
    int64_t psi_off;     // into the vanilla table, in entries
    int32_t status;
    int32_t orig;        // index of the sequence in the caller's array
};

// XCD-partitioned control block.  Buffer slot s belongs to XCD s % kXcd;
// only blocks running on that XCD touch its row buffers, so those buffers
// are communicated through that XCD's L2.  Everything below is shared by
// all XCDs and is accessed with coherent (sc1) loads and stores.
constexpr int kXcd = 8;
constexpr int kLine = 32;  // uint32 per 128-byte line

struct EngineState {
    int32_t error;              // nonzero: watchdog or step guard fired
    int32_t steps;              // global steps executed
    int32_t max_rows;           // high-water mark of rows in flight
    int32_t q_tail0;            // tasks queued by the setup kernel
    int32_t pad0[kLine - 4];
    int32_t cnt[2][kXcd][4];    // [parity][xcd][full, light, beam, -] rows of a step
    int32_t total[2];           // rows of a step over all XCDs
    int32_t pad1[kLine - 2];
    uint32_t go[kXcd][kLine];   // barrier release flags, one line per XCD
    uint32_t xcd_blocks[kXcd][kLine];  // compute blocks per XCD (counted at start)
    int32_t claim[2][kXcd][kLine];     // [parity][xcd] next unclaimed work unit of a step
    int32_t wclaim[2][kLine];          // [parity] next unclaimed wide item of a step
    // a step's row counts of each XCD, tagged with the epoch of the barrier
    // that publishes them (see pack_counts), so that a block waiting at that
    // barrier receives them with its release flag
    unsigned long long cntw[kXcd][kLine / 2];
};

// Counts word: tag (20 bits: the publishing barrier's epoch; only the
// previous epoch's word can be stale, so the wrap is harmless) | done (no
// rows anywhere) | block rows | light rows | full rows (14 bits each; rows
// per XCD are at most the slots per XCD, kMaxPool).
constexpr uint32_t kTagMask = 0xfffffu;
constexpr int kTagShift = 43;
constexpr int32_t kMaxPool = 16383;
inline __host__ __device__ unsigned long long pack_counts(uint32_t tag, bool done, int32_t nf, int32_t nl,
                                                          int32_t nb) {
    return ((unsigned long long)(tag & kTagMask) << kTagShift) | ((unsigned long long)(done ? 1 : 0) << 42) |
           ((unsigned long long)(nb & 0x3fff) << 28) | ((unsigned long long)(nl & 0x3fff) << 14) |
           (unsigned long long)(nf & 0x3fff);
}

// Everything the persistent engine needs (one model).
struct EngineArgs {
    // model
    int32_t K, Kp;
    const float* log_pi;        // may be null
    const float* Acol;          // the same matrix as the engine's Ap: row-major, pitch Kp
    const float* At;            // its transpose (At[j * Kp + i]), Kp <= kColMaxKp; else null
    // sequences
    SeqInfo* seqs;
    int32_t n_seqs;
    int32_t method;             // FV_VANILLA / FV_FLASH / FV_BEAM
    int32_t B, Bc;              // beam width (<= K) and its padded array length
    int32_t bw;                 // parts of a beam task's step (1 for other methods)
    int32_t bw_min;             // fewest parts whose destinations fit a block's LDS
    int64_t brec;               // floats per beam record (header + state, score, anchor arrays)
    // storage
    float* slot_base;           // slots * slot_floats
    int64_t slot_floats;        // floats per slot
    int32_t n_slots;            // multiple of kXcd
    int32_t has_anc;            // slots carry anc[2] + snap
    int32_t wide;               // wide rows: every block takes a column slice of every dense row
    int32_t slab;               // local dense rows as column slabs (K = Kp = 512 or 1024)
    int32_t wsplit;             // FLASH subtasks split kWSplit ways (0: bisection)
    int32_t force_tiles;        // local dense rows as lane tiles for any row count
    int64_t div_off;            // floats from a slot's start to its division copies (w-way subtasks)
    int32_t leaf_len;           // subtasks of at most this many steps are leaves (0: none)
    int32_t beam_q;             // beam rows run four to a block (dense, one part, small K and B)
    int32_t relative_init;      // subtask starts drop the carried score (FV_FLAG_RELATIVE_INIT)
    int32_t path_done;          // the decode kernel walked the vanilla table itself (finish skips it)
    int64_t leaf_off;           // floats from a slot's start to its leaf table
    // sparse transitions (CSR out-edges and their in-edge transpose in edge
    // order); null for dense models
    int32_t sparse;
    int64_t nnz;
    const int32_t* row_ptr;     // [K+1] out-edges of each source
    const int32_t* col;         // [nnz] destination
    const float* val;           // [nnz] log A
    const int32_t* in_ptr;      // [K+1] in-edges of each destination
    const int32_t* in_src;      // [in_ptr[K]] source, non-decreasing within a destination
    const float* in_val;        // [in_ptr[K]]
    int32_t* csr_flag;          // kCsr* bits found by the transpose and the engine
    float* alpha_at;            // sum T floats
    float* root_copy;           // division copies (delta and link), units of Kp
    uint16_t* psi16;            // vanilla backpointers
    unsigned long long* keys;   // final arg max keys [n_seqs]
    // scheduling
    EngineState* st;
    uint32_t* arrive;           // [gridDim] barrier arrival flags
    Row* rows_full;             // [2][kXcd][pool] rows of a step, per XCD
    Row* rows_light;            // [2][kXcd][pool]
    Row* rows_beam;             // [2][kXcd][pool]
    int32_t pool;               // slots per XCD (= n_slots / kXcd)
    Task* queue;                // linear, capacity q_cap
    int64_t q_cap;
    int32_t* free_stack;        // [kXcd][pool]
    int32_t n_compute_blocks;   // blocks 1..n_compute_blocks compute; block 0 schedules
    int64_t spin_limit;
    int64_t max_steps;          // guard against a runaway schedule
    // emission model (sparse models only): FV_EMIT_TABLE reads each row's
    // log_b table; FV_EMIT_GAUSS2D scores the observation points that
    // log_b then addresses (float64 [T][2]) against emit_xy
    int32_t emit_kind;
    const double* emit_xy;      // [K][2] state points
    double emit_c2, emit_c0;    // log B_t(j) = (float)(c2 * d2 - c0)
    // input validation (FV_FLAG_VALIDATE): null when not requested
    const int32_t* bad_seq;     // [caller's n_seqs] nonzero: NaN or +inf in that sequence's log B
    const int32_t* bad_model;   // nonzero: NaN or +inf in this model's log A or log pi
    // measurement (fv_debug_engine_trace): per-step timestamps, or null
    unsigned long long* trace;  // [trace_steps][kTraceWords]
    int32_t trace_steps;
};

// Per-step trace words (real-time counter ticks, 100 MHz): the step's start
// as the scheduler block leaves the barrier, the scheduler's end, the first
// and last compute block's end of work, the sum of all compute blocks' ends,
// the step's row counts (full, light, block rows) packed in one word, the
// number of compute blocks that reported, and each XCD's last end.
constexpr int kTraceWords = 16;
enum { TR_START = 0, TR_SCHED = 1, TR_END_MIN = 2, TR_END_MAX = 3, TR_END_SUM = 4, TR_ROWS = 5, TR_NBLK = 6,
       TR_XCD_END = 8 };   // words 8..15: the last compute block's end on each XCD

// Arguments of the per-call setup kernel (per-sequence layout, first row list).
struct SetupArgs {
    const fv_seq* seqs_dev;
    int32_t n_seqs;
    int32_t P;
    int64_t host_sum_T;     // the host's totals, checked against the device's copies
    int64_t host_sum_root;
    int64_t host_sum_psi;
    int32_t kind;           // KIND_VANILLA, KIND_ROOT or KIND_BROOT
    int32_t K;
    int32_t model;          // this decode takes the sequences whose model index equals this
    int32_t n_local;        // the host's count of them
    int32_t emit_kind;      // FV_EMIT_TABLE: log_b is a table of ld >= K floats per step
    EngineArgs* args_out;   // the engine's copy of its arguments (workspace)
};

// Division points of the first P'-way split: e_d = floor(((d+1) T - 1) / P').
inline __host__ __device__ int64_t seg_end(int32_t T, int32_t pp, int32_t d) {
    return (((int64_t)d + 1) * T - 1) / pp;
}
// Index d of the division point equal to x, or -1 (only d <= pp-2 count).
inline __host__ __device__ int32_t div_index(int32_t T, int32_t pp, int64_t x) {
    if (x < 0) return -1;
    int64_t d = ((x + 1) * (int64_t)pp) / T - 1;
    if (d < 0 || d > pp - 2) return -1;
    return seg_end(T, pp, (int32_t)d) == x ? (int32_t)d : -1;
}
inline __host__ __device__ int32_t eff_parallelism(int32_t T, int32_t P) {
    if (T <= 1) return 1;
    int32_t pp = P < 2 ? 2 : P;
    return pp > T ? T : pp;
}

}  // namespace fv
