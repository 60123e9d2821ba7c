/*
 * flashviterbi.h -- C ABI of the MI355X (gfx950) FLASH Viterbi library.
 *
 * Problem (Sec. III-A of the FLASH Viterbi paper): an HMM with K hidden
 * states, initial scores log pi[K], transition scores log A[K][K] and
 * per-step emission scores log B_t[K] for t = 0..T-1.  Decoding returns the
 * optimal state sequence q*_0..q*_{T-1} (int32) and its log score (float32):
 *
 *   delta_0(j) = log pi_j + log B_0(j)
 *   delta_t(j) = max_i (delta_{t-1}(i) + log A(i, j)) + log B_t(j)
 *   psi_t(j)   = lowest i attaining that max
 *   q*_{T-1}   = lowest arg max_j delta_{T-1}(j),  q*_t = psi_{t+1}(q*_{t+1})
 *
 * Every value is an IEEE binary32 log-score and every candidate is one
 * float32 add rounded to nearest even; all entry points return the same path
 * and bit-identical scores as a plain sequential float32 evaluation of those
 * formulas (ties to the lowest index; log B added after the max).
 *
 * Conventions for every entry point
 *  - Array arguments are DEVICE pointers unless marked "host".  The caller
 *    owns all buffers.  The library never allocates device memory in a
 *    decode call: scratch space comes from the caller's workspace `ws` of at
 *    least fv_workspace_size() bytes (256-byte aligned).
 *  - Calls only enqueue work on `stream`; they do not synchronise it.
 *    Device buffers must stay valid until the stream has run the work.
 *  - Layouts (row-major):
 *      log_a[i*K + j]   = log A(i -> j), row = source state
 *      log_b[t*ld + j]  = log B_t(j), ld >= K
 *      log_pi[j]        (may be NULL: no initial term)
 *  - Inputs must be finite or -inf.  NaN / +inf give unspecified paths.
 *  - Host-detectable errors are returned synchronously.  Data-dependent
 *    outcomes go to the optional device array `status` (one int32 per
 *    sequence): FV_OK, FV_E_INFEASIBLE (best score is -inf; the path is
 *    filled with -1), FV_W_BEAM_FALLBACK (a beam subtask was re-decoded
 *    exactly), FV_E_WORKSPACE / FV_E_DEVICE (the decode did not run or did
 *    not finish; outputs unspecified).
 *  - One call at a time per workspace; independent workspaces may run
 *    concurrently on different streams.
 */
#ifndef FLASHVITERBI_H
#define FLASHVITERBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* fv_stream_t; /* a hipStream_t (NULL = default stream) */

typedef enum {
    FV_OK = 0,
    FV_E_INVALID_ARG = -1,
    FV_E_UNSUPPORTED = -2,
    FV_E_WORKSPACE = -3,
    FV_E_DEVICE = -4,
    FV_E_INFEASIBLE = -5,
    FV_W_BEAM_FALLBACK = 1
} fv_status;

enum { FV_DENSE = 0, FV_CSR = 1 };

/* Decode flags (bit set).  Placement of the rows in flight: by default the
 * library keeps each row on one XCD and tiles rows onto lanes (many rows,
 * log A shared through the XCD's L2), or, for large K or very few rows, uses
 * wide rows (every compute unit takes a column slice of every row and log A
 * streams from HBM once per step).  These flags force one placement; the
 * results are the same either way. */
enum { FV_FLAG_WIDE_ROWS = 1u << 0, FV_FLAG_LOCAL_ROWS = 1u << 1 };
/* Input validation.  Scores must be finite or -inf (NaN and +inf are outside
 * the contract and give unspecified paths, though never an out-of-range
 * access).  With FV_FLAG_VALIDATE the call first scans log A (or the CSR
 * scores), log pi and every sequence's log B; a sequence whose model or
 * emissions hold NaN or +inf gets status FV_E_INVALID_ARG (written
 * asynchronously, like every status). */
enum { FV_FLAG_VALIDATE = 1u << 2 };
/* FLASH schedule.  By default a subtask of at most 128 steps (dense model,
 * K <= 2048, rows on their XCD) is a leaf: it keeps a backpointer table
 * (uint16, one row of K per step, sized to the longest leaf that can occur)
 * in its row buffer and resolves all its positions at its end instead of
 * being bisected further (same result, much less recomputation).  The
 * workspace plans leaves, and sizes the row-buffer pool to the leaf-cut task
 * tree, when the default placement keeps rows on their XCD; with
 * FV_FLAG_WIDE_ROWS such a plan still decodes correctly, without leaves and
 * with subtasks waiting for row buffers.  Where there are no leaves (dense
 * wide rows with K > 2048, and CSR models), a subtask is split into up to 8
 * segments instead of two: the root's P'-way division rule applied over the
 * subtask's own span (Sec. V-A), every division state resolved at its end.
 * FV_FLAG_NO_LEAVES bisects every subtask down to the paper's minimum. */
enum { FV_FLAG_NO_LEAVES = 1u << 3 };
/* Subtask initialisation (Sec. V-B, pruning for parallel decoding).  By
 * default a subtask starting at m > 0 is anchored: its start scores are
 * (alpha + log A(q*_{m-1}, j)) + log B_m(j), alpha being the parent's score of
 * q*_{m-1} (retained pruning, Def. 3), which reproduces vanilla's float32
 * values along the path, so FLASH and FLASH-BS with B >= K return vanilla's
 * path.  FV_FLAG_RELATIVE_INIT takes the paper's displayed initialisation,
 * log A(q*_{m-1}, j) + log B_m(j) (the carried score dropped): exact in real
 * arithmetic, but in float32 rounding depends on the magnitude of the
 * running score, so paths can differ from vanilla's at near ties.  Every
 * subtask is then bisected down to the paper's minimum (no leaves: a leaf
 * would start once where the bisection restarts at each level, and the two
 * round differently).  The score returned is the root pass's maximum for
 * FLASH and the re-summed score of the decoded path for FLASH-BS; with this
 * flag the two can differ in the last bits where the path leaves vanilla's.
 * A beam of width B >= K is decoded as FLASH, so it returns FLASH's result.  Dense models only (FLASH and FLASH-BS);
 * with a CSR model the call returns FV_E_UNSUPPORTED.  Vanilla decoding
 * ignores it. */
enum { FV_FLAG_RELATIVE_INIT = 1u << 4 };
/* Kernel choices for tuning; none changes a result.  Dense rows kept on
 * their XCD normally run as column slabs (K = 512 or 1024: a block holds 64
 * columns of log A in registers), else as column items (rows' scores in LDS,
 * two destinations per lane) while an XCD holds at most 160 rows, else as
 * lane tiles (lanes = rows, log A as wave-uniform scalars).
 * FV_FLAG_STEP_ITEMS takes column items instead of slabs; FV_FLAG_STEP_TILES
 * takes lane tiles for any number of rows (they exclude each other).
 * FV_FLAG_ENGINE decodes vanilla and FLASH on a small dense model (K <= 256)
 * with the persistent engine instead of one block per sequence. */
enum { FV_FLAG_STEP_ITEMS = 1u << 5, FV_FLAG_STEP_TILES = 1u << 6, FV_FLAG_ENGINE = 1u << 7 };
enum { FV_VANILLA = 0, FV_FLASH = 1, FV_BEAM = 2 };

/* Transition model.  FV_DENSE: log_a[K*K] (device).  FV_CSR: out-edges of
 * each source, row_ptr[K+1], col[nnz] (destination), val[nnz] (device);
 * missing edges are -inf. */
typedef struct {
    int32_t kind;
    int32_t K;
    const float* log_a;
    const int32_t* row_ptr;
    const int32_t* col;
    const float* val;
    int64_t nnz;
} fv_trans;

/* One sequence of a batch (the array of these lives on the device). */
typedef struct {
    int32_t model;        /* index into the models array                  */
    int32_t T;            /* length, >= 0 (T = 0: nothing decoded, score 0) */
    const float* log_b;   /* [T][ld] emission scores                      */
    int64_t ld;
    int32_t* path;        /* [T] output                                   */
    float* score;         /* [1] output                                   */
} fv_seq;

/* Bytes of workspace a decode needs.  method: FV_VANILLA / FV_FLASH /
 * FV_BEAM.  models/n_models describe the transition models; T_host[n_seqs]
 * and model_host[n_seqs] (host; model_host may be NULL when n_models == 1)
 * give each sequence's length and model.  P and B as in the decode calls.
 * The value depends only on these arguments.  (Sizes are the memory figures
 * the library reports: Sec. VII-B's "all data structures used during
 * decoding".) */
fv_status fv_workspace_size(int32_t method, const fv_trans* models, int32_t n_models,
                            const int32_t* T_host, const int32_t* model_host, int32_t n_seqs,
                            int32_t P, int32_t B, size_t* bytes);

/* Vanilla Viterbi (Sec. III-A): full backpointer table (K x T, packed) in
 * the workspace, then backtracking.  path[T] and score[1] are device
 * outputs; status may be NULL. */
fv_status fv_decode_vanilla(const fv_trans* A, const float* log_pi, const float* log_b,
                            int64_t ld, int32_t T, int32_t* path, float* score,
                            int32_t* status, uint32_t flags, void* ws, size_t ws_bytes,
                            fv_stream_t stream);

/* FLASH Viterbi (Alg. 1 and 2; Sec. V-A/V-B): one pass over the sequence
 * keeping only the P'-1 boundary states' pointers, a P'-way split
 * P' = min(max(P,2),T), then midpoint bisection of the independent
 * segments, each started from its single known boundary state.  The
 * boundary state's float32 score is carried into the segment (retained
 * pruning, Def. 3), so the result equals fv_decode_vanilla bit for bit for
 * every P.  P <= 0 selects P automatically: the largest power of two in
 * [2, 512] with P <= T/16 for the median length T, which bounds the
 * division copies to a quarter of a vanilla backpointer table (a larger P
 * means shorter subtask trees, hence fewer engine steps and less
 * recomputation). */
fv_status fv_decode_flash(const fv_trans* A, const float* log_pi, const float* log_b,
                          int64_t ld, int32_t T, int32_t P, int32_t* path, float* score,
                          int32_t* status, uint32_t flags, void* ws, size_t ws_bytes,
                          fv_stream_t stream);

/* fv_decode_flash without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Scratch comes from a fixed
 * device array of FV_NOALLOC_SCRATCH_BYTES inside the library (one per GPU,
 * held until the process ends); the call allocates nothing and enqueues the
 * same kernels as fv_decode_flash, with the same result.  A decode needing
 * more scratch than the array holds (fv_workspace_size(FV_FLASH, ...) >
 * FV_NOALLOC_SCRATCH_BYTES; a K = 1024 sequence of T = 8000 at P = 64
 * needs about 90 MB, K = 2048 at T = 4000 about 153 MB) returns
 * FV_E_WORKSPACE with a message.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and give unspecified results; calls on one
 * stream are ordered and safe.  The engine's setup kernel re-initialises
 * every field it reads, so no state carries over between calls. */
#define FV_NOALLOC_SCRATCH_BYTES (128u << 20)
fv_status fv_decode_flash_noalloc(const fv_trans* A, const float* log_pi, const float* log_b,
                                  int64_t ld, int32_t T, int32_t P, int32_t* path, float* score,
                                  int32_t* status, uint32_t flags, fv_stream_t stream);

/* FLASH-BS (Sec. V-C): the FLASH task structure where every step keeps only
 * the B best states, ranked by (score desc, state asc).  B >= K behaves as
 * FLASH.  For B < K the result depends on P (each segment restarts its beam
 * from its boundary state), so P >= 1 is required.  A task's last step only
 * evaluates its known end state; if no beam state reaches it the task is
 * re-decoded exactly and status gets FV_W_BEAM_FALLBACK.  score is the
 * step-by-step re-sum of the returned path. */
fv_status fv_decode_beam(const fv_trans* A, const float* log_pi, const float* log_b,
                         int64_t ld, int32_t T, int32_t B, int32_t P, int32_t* path,
                         float* score, int32_t* status, uint32_t flags, void* ws,
                         size_t ws_bytes, fv_stream_t stream);

/* Many sequences, uneven lengths, one decode launch: the persistent engine,
 * or, for vanilla and FLASH decodes whose dense models all have K <= 256,
 * one block (one to four waves) per sequence running the same method (same
 * results).  models: host
 * array [n_models] (dense and CSR models may be mixed, K may differ);
 * log_pi: host array of n_models device pointers (entries may be NULL);
 * seqs_dev: device array [n_seqs]; T_host / model_host: host copies of each
 * sequence's T and model index (they lay out the workspace; model_host may
 * be NULL only when n_models == 1).  The device copies must agree: a model
 * index outside [0, n_models) or counts that differ from the host's make
 * the affected statuses FV_E_INVALID_ARG.  The launch decodes the models'
 * sequence sets one after the other, each with its own rows and buffers.
 * method FV_VANILLA / FV_FLASH / FV_BEAM with P, B as above (B >= K_m makes
 * model m's decode FLASH).  Each sequence's result equals the
 * single-sequence call's. */
fv_status fv_decode_batch(const fv_trans* models, const float* const* log_pi, int32_t n_models,
                          const fv_seq* seqs_dev, const int32_t* T_host,
                          const int32_t* model_host, int32_t n_seqs, int32_t method,
                          int32_t P, int32_t B, int32_t* status, uint32_t flags, void* ws,
                          size_t ws_bytes, fv_stream_t stream);

/* Emission model generated inside the decode (Sec. III: observations may
 * be continuous, e.g. Gaussian), replacing the log_b tables.
 * FV_EMIT_TABLE: each sequence's fv_seq.log_b table, as in every other call.
 * FV_EMIT_GAUSS2D: state j sits at the point (state_xy[2j], state_xy[2j+1])
 * (device, float64 [K][2]) and each observation is a point; a sequence's
 * fv_seq.log_b field then carries the address of its observations (device,
 * float64 [T][2], cast to const float*) and its ld is ignored.  The score is
 * evaluated in float64, every operation rounded once (no fused
 * multiply-add), then rounded to float32:
 *     dx = x_j - u_t,  dy = y_j - v_t,  d2 = dx*dx + dy*dy,
 *     log B_t(j) = (float)(c2 * d2 - c0)
 * For a Gaussian of standard deviation sigma on the distance,
 * c2 = -1 / (2 sigma^2) and c0 = ln(sigma sqrt(2 pi)).  c2 must be finite
 * and <= 0, c0 finite and >= -FLT_MAX (no score can then be +inf); with
 * finite points no score is NaN.  FV_FLAG_VALIDATE checks that every
 * coordinate (state points and observations) is finite. */
enum { FV_EMIT_TABLE = 0, FV_EMIT_GAUSS2D = 1 };
typedef struct {
    int32_t kind;
    const double* state_xy;
    double c2;
    double c0;
} fv_emission;

/* fv_decode_batch with an emission model per transition model: emissions
 * is a host array [n_models] (NULL: every model reads tables).  A
 * FV_EMIT_GAUSS2D entry requires a CSR model (FV_E_UNSUPPORTED for a dense
 * one) and K points.  Each sequence's result equals fv_decode_batch's on the
 * tables the emission model defines, bit for bit; the tables are never
 * written to memory. */
fv_status fv_decode_batch_emit(const fv_trans* models, const fv_emission* emissions,
                               const float* const* log_pi, int32_t n_models, const fv_seq* seqs_dev,
                               const int32_t* T_host, const int32_t* model_host, int32_t n_seqs,
                               int32_t method, int32_t P, int32_t B, int32_t* status, uint32_t flags,
                               void* ws, size_t ws_bytes, fv_stream_t stream);

/* Gradient of the Viterbi scores S_b (the decoded path's summed log-scores)
 * given upstream gradients grad_score[n].  No passage of the paper defines
 * this operation: it is the subgradient of the score of Sec. III-A (a sum of
 * log-scores along the decoded path) with respect to its inputs, for
 * structured-hinge training; at ties it takes the decoded path's indicator.
 *
 *   grad_log_b[b][t][j] = grad_score[b] * [j == paths[b][t]]   (t < lengths[b], else 0)
 *   grad_log_a[i][j]    = sum over b ascending of fl(grad_score[b] * c_b(i,j)),
 *                         c_b(i,j) = #{t >= 1 : (q_{b,t-1}, q_{b,t}) = (i, j)}
 *   grad_log_pi[j]      = sum over b ascending of grad_score[b] * [q_{b,0} == j]
 * paths is [n][Tmax] int32, lengths [n].  Any of the three outputs may be
 * NULL.  accumulate != 0 adds the result to the outputs' current contents
 * (old + total for the shared ones).  Deterministic: identical bits on
 * every run. */
fv_status fv_viterbi_backward(int32_t K, int32_t n_seqs, int32_t Tmax, const int32_t* lengths,
                              const int32_t* paths, const float* grad_score, float* grad_log_b,
                              float* grad_log_a, float* grad_log_pi, int32_t accumulate,
                              void* ws, size_t ws_bytes, fv_stream_t stream);

/* Workspace bytes for fv_viterbi_backward. */
fv_status fv_backward_workspace_size(int32_t K, int32_t n_seqs, int32_t Tmax, size_t* bytes);

/* score_out[b] = step-by-step float32 re-sum of paths[b] (dense model):
 * s = log pi[q0] + log B_0[q0]; s = (s + log A[q_{t-1}][q_t]) + log B_t[q_t]
 * (the path's score of Sec. III-A, added in time order; log pi NULL drops
 * the first term).  seqs_dev: device array [n_seqs] whose `path` fields are
 * read (int32 [T] each, entries in [0, K); an entry outside gives -inf) and
 * whose `score` fields are ignored; score_out: device float32 [n_seqs]. */
fv_status fv_rescore(const fv_trans* A, const float* log_pi, const fv_seq* seqs_dev,
                     int32_t n_seqs, float* score_out, fv_stream_t stream);

/* Discrete-emission HMMs: log_b[t*ld + j] = log_e[j*V + obs[t]]. */
fv_status fv_gather_emissions(int32_t K, int32_t V, const float* log_e, const int32_t* obs,
                              int32_t T, float* log_b, int64_t ld, fv_stream_t stream);

/* Measurement hook: while enabled (enable != 0, host thread-local), every
 * decode records a pair of HIP events on its stream immediately before and
 * after its decode kernel (the persistent engine, or the per-sequence
 * kernels of small dense models).  fv_profile_engine_ms waits for the last pair
 * and returns that kernel's duration in milliseconds.
 * Enable outside stream capture (it creates the events). */
fv_status fv_profile_engine(int32_t enable);
fv_status fv_profile_engine_ms(float* ms);
/* Disabling (enable == 0) waits for the last recorded pair and destroys the
 * events, so no HIP object of the library outlives the measurement. */

/* Test hook for the persistent engine's watchdog.  Nonzero max_steps or
 * spin_limit replace, for later decodes issued by this host thread, the
 * engine's bound on global steps (by default far above any valid schedule)
 * and on the iterations of each wait at its step barrier.  A decode that
 * reaches either bound stops normally on every block and reports
 * FV_E_DEVICE in every status entry.  0 restores the defaults; negative
 * values return FV_E_INVALID_ARG. */
fv_status fv_debug_engine_limits(int64_t max_steps, int64_t spin_limit);

/* Measurement hook: while set (steps > 0, host thread-local), persistent
 * engine decodes issued by this thread record, for each of their first
 * `steps` global steps, 16 words in trace[step * 16 ...] (device buffer,
 * uint64): the step's start and the scheduler's end (real-time counter,
 * 100 MHz ticks), the first and last compute block's end of work, the sum
 * of all compute blocks' ends, the rows in flight (full | light << 21 |
 * block rows << 42), the number of compute blocks that reported (word 6)
 * and, in words 8..15, the last end on each XCD.  The caller zeroes the
 * buffer except word 2 (set it to all ones) before each decode.  steps == 0
 * turns it off. */
fv_status fv_debug_engine_trace(unsigned long long* trace, int32_t steps);

const char* fv_status_str(fv_status s);
const char* fv_last_error(void);   /* thread-local message of the last failure */
int32_t fv_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FLASHVITERBI_H */
