/*
 * FLASH Viterbi -- plain CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU path.
 *
 * Arithmetic: IEEE-754 binary32, round to nearest even, one rounding per add
 * (the library's contract: float32 log-scores in, float32 score out, every
 * candidate a single float32 add).  Build with -O2 -ffp-contract=off and
 * without -ffast-math.  The float64 instantiation of vanilla exists for the
 * finite-difference gradient checks.
 *
 * Contents, each following the passage named in its header comment:
 *   fvo_vanilla      Viterbi recurrence + backtracking      (Sec. III-A)
 *   fvo_vanilla_f64  same, in double                        (Sec. III-A)
 *   fvo_vanilla_csr  same, transitions as CSR out-edges     (Sec. III-A)
 *   fvo_rescore      re-sum of one path's log score         (Sec. III-A)
 *   fvo_flash        non-recursive D&C with pruning         (Alg. 1, Alg. 2, Sec. V-A/V-B)
 *   fvo_beam         FLASH-BS dynamic beam                  (Sec. V-C)
 *   fvo_beam_csr     same, transitions as CSR out-edges     (Sec. V-C)
 *   fvo_backward     subgradient of the Viterbi score       (score is a sum of
 *                    the decoded path's log-scores, Sec. III-A)
 *   fvo_gather_emissions  log B_t[j] = log e[j, x_t]        (Sec. III, the HMM triplet)
 *   fvo_gauss_emissions   log B_t[j] of a Gaussian observation model on
 *                    points (Sec. III: continuous observations)
 *
 * Readings of points the paper leaves open (tie-breaking, where log B is
 * added, the anchored pruned initialisation, segment boundaries for P that
 * does not divide T, the beam's tie rule and end step) are stated at the
 * function that makes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FVO_OK 0
#define FVO_INVALID (-1)
#define FVO_INFEASIBLE (-5)
#define FVO_BEAM_FALLBACK 1

/* ------------------------------------------------------------------------ */
/* Vanilla Viterbi (Sec. III-A).
 *
 *   delta_0(j) = log pi_j + log B_0(j)            (log B_0(j) alone if pi is NULL)
 *   c_t(j)     = max_i  delta_{t-1}(i) + log A(i, j)
 *   psi_t(j)   = the smallest i attaining that max
 *   delta_t(j) = c_t(j) + log B_t(j)
 *   q_{T-1}    = the smallest j maximising delta_{T-1}(j)
 *   q_t        = psi_{t+1}(q_{t+1})
 *
 * Ties go to the lowest index (the paper does not say; strict ">" while
 * scanning i upward).  log B_t(j) is added after the max, so the score of the
 * decoded path equals fvo_rescore of that path bit for bit.  The value kept
 * is always the winning candidate itself.
 *
 * The predecessor scan for every destination j runs over i in increasing
 * order; j is the inner loop only so that log_a is read row by row.
 * A score of -inf at the end means no feasible path: path is filled with -1.
 */
#define DEFINE_VANILLA(NAME, REAL)                                              \
int NAME(int K, int T, const REAL* log_pi, const REAL* log_a,                   \
         const REAL* log_b, int64_t ld, int32_t* path, REAL* score)             \
{                                                                               \
    if (K < 1 || T < 1 || ld < K || !log_a || !log_b || !path || !score)        \
        return FVO_INVALID;                                                     \
    REAL* delta = (REAL*)malloc(sizeof(REAL) * (size_t)K);                      \
    REAL* best = (REAL*)malloc(sizeof(REAL) * (size_t)K);                       \
    int32_t* psi = (int32_t*)malloc(sizeof(int32_t) * (size_t)K * (size_t)T);   \
    for (int j = 0; j < K; ++j)                                                 \
        delta[j] = log_pi ? (REAL)(log_pi[j] + log_b[j]) : log_b[j];            \
    for (int t = 1; t < T; ++t) {                                               \
        int32_t* psi_t = psi + (size_t)t * K;                                   \
        for (int j = 0; j < K; ++j) {                                           \
            best[j] = (REAL)(delta[0] + log_a[j]);                              \
            psi_t[j] = 0;                                                       \
        }                                                                       \
        for (int i = 1; i < K; ++i) {                                           \
            const REAL* row = log_a + (size_t)i * K;                            \
            for (int j = 0; j < K; ++j) {                                       \
                REAL c = (REAL)(delta[i] + row[j]);                             \
                if (c > best[j]) { best[j] = c; psi_t[j] = i; }                 \
            }                                                                   \
        }                                                                       \
        const REAL* b_t = log_b + (size_t)t * ld;                               \
        for (int j = 0; j < K; ++j) delta[j] = (REAL)(best[j] + b_t[j]);        \
    }                                                                           \
    int q = 0;                                                                  \
    for (int j = 1; j < K; ++j) if (delta[j] > delta[q]) q = j;                 \
    *score = delta[q];                                                          \
    int rc = FVO_OK;                                                            \
    if (delta[q] == (REAL)-INFINITY) {                                          \
        for (int t = 0; t < T; ++t) path[t] = -1;                               \
        rc = FVO_INFEASIBLE;                                                    \
    } else {                                                                    \
        path[T - 1] = q;                                                        \
        for (int t = T - 1; t > 0; --t) path[t - 1] = psi[(size_t)t * K + path[t]]; \
    }                                                                           \
    free(delta); free(best); free(psi);                                         \
    return rc;                                                                  \
}

DEFINE_VANILLA(fvo_vanilla, float)
DEFINE_VANILLA(fvo_vanilla_f64, double)

/* Vanilla Viterbi with transitions given as CSR out-edges: row_ptr[K+1],
 * col[nnz] (destination), val[nnz] (log A(i, col)).  Missing edges are
 * log A = -inf.  Each destination's predecessors are scanned in increasing
 * source order, the first edge giving the initial value; a destination with
 * no in-edge gets -inf and psi = 0.  For any input with a finite best score
 * this decodes the same path as the dense form with -inf entries. */
int fvo_vanilla_csr(int K, int T, const float* log_pi, const int32_t* row_ptr,
                    const int32_t* col, const float* val, const float* log_b,
                    int64_t ld, int32_t* path, float* score)
{
    if (K < 1 || T < 1 || ld < K || !row_ptr || !log_b || !path || !score)
        return FVO_INVALID;
    float* delta = (float*)malloc(sizeof(float) * (size_t)K);
    float* best = (float*)malloc(sizeof(float) * (size_t)K);
    uint8_t* seen = (uint8_t*)malloc((size_t)K);
    int32_t* psi = (int32_t*)malloc(sizeof(int32_t) * (size_t)K * (size_t)T);
    for (int j = 0; j < K; ++j) delta[j] = log_pi ? log_pi[j] + log_b[j] : log_b[j];
    for (int t = 1; t < T; ++t) {
        int32_t* psi_t = psi + (size_t)t * K;
        for (int j = 0; j < K; ++j) { best[j] = -INFINITY; psi_t[j] = 0; seen[j] = 0; }
        for (int i = 0; i < K; ++i) {
            for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                int j = col[e];
                float c = delta[i] + val[e];
                if (!seen[j] || c > best[j]) { best[j] = c; psi_t[j] = i; seen[j] = 1; }
            }
        }
        const float* b_t = log_b + (size_t)t * ld;
        for (int j = 0; j < K; ++j) delta[j] = best[j] + b_t[j];
    }
    int q = 0;
    for (int j = 1; j < K; ++j) if (delta[j] > delta[q]) q = j;
    *score = delta[q];
    int rc = FVO_OK;
    if (delta[q] == -INFINITY) {
        for (int t = 0; t < T; ++t) path[t] = -1;
        rc = FVO_INFEASIBLE;
    } else {
        path[T - 1] = q;
        for (int t = T - 1; t > 0; --t) path[t - 1] = psi[(size_t)t * K + path[t]];
    }
    free(delta); free(best); free(seen); free(psi);
    return rc;
}

/* Score of one given path, summed step by step in the recurrence's order:
 * s_0 = log pi_{q0} + log B_0(q0);  s_t = (s_{t-1} + log A(q_{t-1}, q_t)) + log B_t(q_t). */
float fvo_rescore(int K, int T, const float* log_pi, const float* log_a,
                  const float* log_b, int64_t ld, const int32_t* path)
{
    float s = log_pi ? log_pi[path[0]] + log_b[path[0]] : log_b[path[0]];
    for (int t = 1; t < T; ++t) {
        float c = s + log_a[(size_t)path[t - 1] * K + path[t]];
        s = c + log_b[(size_t)t * ld + path[t]];
    }
    return s;
}

/* Emission rows of a discrete HMM: log_b[t*ld + j] = log_e[j*V + obs[t]]. */
int fvo_gather_emissions(int K, int V, const float* log_e, const int32_t* obs, int T,
                         float* log_b, int64_t ld)
{
    if (K < 1 || V < 1 || T < 0 || ld < K) return FVO_INVALID;
    for (int t = 0; t < T; ++t) {
        if (obs[t] < 0 || obs[t] >= V) return FVO_INVALID;
        for (int j = 0; j < K; ++j) log_b[(size_t)t * ld + j] = log_e[(size_t)j * V + obs[t]];
    }
    return FVO_OK;
}

/* Emission rows of a continuous-observation HMM (Sec. III names Gaussian
 * observation models): state j sits at the point (xy[2j], xy[2j+1]),
 * observation t is the point (obs[2t], obs[2t+1]), and
 *     log B_t(j) = c2 * d2 - c0,   d2 = (x_j - u_t)^2 + (y_j - v_t)^2,
 * evaluated in double, each operation rounded once (the file is built
 * without contraction), then rounded to float.  For a Gaussian of standard
 * deviation sigma on the distance, c2 = -1/(2 sigma^2) and
 * c0 = log(sigma sqrt(2 pi)). */
int fvo_gauss_emissions(int K, const double* xy, const double* obs, int T, double c2, double c0,
                        float* log_b, int64_t ld)
{
    if (K < 1 || T < 0 || ld < K) return FVO_INVALID;
    for (int t = 0; t < T; ++t) {
        const double u = obs[2 * (size_t)t], v = obs[2 * (size_t)t + 1];
        for (int j = 0; j < K; ++j) {
            const double dx = xy[2 * (size_t)j] - u;
            const double dy = xy[2 * (size_t)j + 1] - v;
            const double sx = dx * dx;
            const double sy = dy * dy;
            const double d2 = sx + sy;
            const double e = c2 * d2;
            log_b[(size_t)t * ld + j] = (float)(e - c0);
        }
    }
    return FVO_OK;
}

/* ------------------------------------------------------------------------ */
/* Shared helpers for the two divide-and-conquer oracles.                    */

/* Effective parallelism and first-level segment ends (Sec. V-A, "P-way
 * partition").  P' = min(max(P, 2), T), P' = 1 when T = 1 (P = 1 runs the
 * serial root of Alg. 2, which splits at floor((T-1)/2), i.e. P' = 2).
 * Segment d is [e_{d-1}+1, e_d] with e_d = floor(((d+1)T - 1) / P');
 * e_{P'-1} = T-1 and lengths differ by at most one. */
static int eff_parallelism(int T, int P)
{
    if (P < 1) P = 1;
    int pp = P < 2 ? 2 : P;
    if (pp > T) pp = T;
    return pp;
}

static int64_t seg_end(int T, int pp, int d) { return (((int64_t)d + 1) * T - 1) / pp; }

typedef struct {
    int m, n;           /* segment [m, n], n > m                           */
    int q_prev;         /* q*_{m-1} (ignored when m == 0)                  */
    float alpha;        /* delta_{m-1}(q*_{m-1}) (ignored when m == 0)     */
} fvo_task;

typedef struct {
    fvo_task* v;
    int head, tail, cap;
} fvo_queue;

static void q_push(fvo_queue* q, fvo_task t)
{
    if (q->tail == q->cap) {
        q->cap = q->cap ? 2 * q->cap : 64;
        q->v = (fvo_task*)realloc(q->v, sizeof(fvo_task) * (size_t)q->cap);
    }
    q->v[q->tail++] = t;
}

/* Dequeue: FIFO by default; with a seed, a uniformly random ready task (every
 * queued task's parent has finished, so any order is valid, Sec. V-A (ii)). */
static int q_pop(fvo_queue* q, uint64_t* rng, fvo_task* out)
{
    if (q->head == q->tail) return 0;
    if (rng && *rng) {
        uint64_t x = *rng;
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        *rng = x;
        int k = q->head + (int)(x % (uint64_t)(q->tail - q->head));
        fvo_task t = q->v[k];
        q->v[k] = q->v[q->head];
        q->v[q->head] = t;
    }
    *out = q->v[q->head++];
    return 1;
}

typedef struct {
    int64_t tasks;          /* decoding calls, the root included              */
    int64_t candidates;     /* delta + log A evaluations                      */
    int64_t resolved_twice; /* positions written more than once (must be 0)   */
    int64_t max_queue;      /* largest number of queued tasks                 */
} fvo_stats;

/* One max-plus step over all destinations (Alg. 2, DP loop body):
 * out[j] = max_i (in[i] + log A(i, j)) + log B(j), pre[j] = lowest arg max. */
static void dense_step(int K, const float* in, const float* log_a, const float* b_t,
                       float* out, int32_t* pre, float* best)
{
    for (int j = 0; j < K; ++j) { best[j] = in[0] + log_a[j]; pre[j] = 0; }
    for (int i = 1; i < K; ++i) {
        const float* row = log_a + (size_t)i * K;
        for (int j = 0; j < K; ++j) {
            float c = in[i] + row[j];
            if (c > best[j]) { best[j] = c; pre[j] = i; }
        }
    }
    for (int j = 0; j < K; ++j) out[j] = best[j] + b_t[j];
}

/* Transition model seen by FLASH-BS: dense log A, or CSR out-edges whose
 * missing entries are -inf (Sec. III-A's A with zero probabilities).  With
 * several edges i -> j, log A(i, j) is the largest of them. */
typedef struct {
    int K;
    const float* log_a;       /* dense [K*K], NULL for CSR */
    const int32_t* row_ptr;   /* CSR: out-edges of source i are [row_ptr[i], row_ptr[i+1]) */
    const int32_t* col;
    const float* val;
} fvo_model;

static float model_a(const fvo_model* M, int i, int j)
{
    if (M->log_a) return M->log_a[(size_t)i * M->K + j];
    float a = -INFINITY;
    for (int e = M->row_ptr[i]; e < M->row_ptr[i + 1]; ++e)
        if (M->col[e] == j && M->val[e] > a) a = M->val[e];
    return a;
}

/* sc[j] = (alpha + log A(q, j)) + b_m[j] for every j: the anchored start
 * (with relative_init the caller passes no alpha: sc[j] = log A(q, j) + b_m[j])
 * of a segment (Def. 3).  CSR: -inf except at q's out-neighbours. */
static void model_anchor_row(const fvo_model* M, int q, float alpha, int relative_init, const float* b_m,
                             float* sc)
{
    if (!M->log_a) {   /* only q's out-neighbours are finite */
        for (int j = 0; j < M->K; ++j) sc[j] = -INFINITY;
        for (int e = M->row_ptr[q]; e < M->row_ptr[q + 1]; ++e) {
            int j = M->col[e];
            float c = relative_init ? model_a(M, q, j) : alpha + model_a(M, q, j);
            sc[j] = c + b_m[j];
        }
        return;
    }
    for (int j = 0; j < M->K; ++j) {
        float c = relative_init ? model_a(M, q, j) : alpha + model_a(M, q, j);
        sc[j] = c + b_m[j];
    }
}

/* Exact step (the fallback re-decode): dense_step, or for CSR the scan of
 * vanilla_csr: sources upward, each source's edges in order, the first
 * edge giving a destination's initial value; pre[j] = 0 without in-edge. */
static void model_exact_step(const fvo_model* M, const float* in, const float* b_t, float* out,
                             int32_t* pre, float* best, uint8_t* seen)
{
    const int K = M->K;
    if (M->log_a) { dense_step(K, in, M->log_a, b_t, out, pre, best); return; }
    for (int j = 0; j < K; ++j) { best[j] = -INFINITY; pre[j] = 0; seen[j] = 0; }
    for (int i = 0; i < K; ++i) {
        for (int e = M->row_ptr[i]; e < M->row_ptr[i + 1]; ++e) {
            int j = M->col[e];
            float c = in[i] + M->val[e];
            if (!seen[j] || c > best[j]) { best[j] = c; pre[j] = i; seen[j] = 1; }
        }
    }
    for (int j = 0; j < K; ++j) out[j] = best[j] + b_t[j];
}

static float model_rescore(const fvo_model* M, int T, const float* log_pi, const float* log_b,
                           int64_t ld, const int32_t* path)
{
    float s = log_pi ? log_pi[path[0]] + log_b[path[0]] : log_b[path[0]];
    for (int t = 1; t < T; ++t) {
        float c = s + model_a(M, path[t - 1], path[t]);
        s = c + log_b[(size_t)t * ld + path[t]];
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* FLASH Viterbi (Alg. 1 + Alg. 2 with pruning, Sec. V-A and V-B).
 *
 * Root task (0, T-1): one pass over the whole sequence that keeps, for every
 * state j, MidState(j) = the state at the most recent division point on the
 * best path to j (Alg. 2's MidState, generalised to the P'-way first split),
 * and at each division point e_d (d <= P'-2) a copy of OptProb and, for
 * d >= 1, of MidState (the link back to e_{d-1}).  At the end q*_{T-1} is the
 * lowest arg max, q*_{e_{P'-2}} = MidState(q*_{T-1}) and each earlier boundary
 * state is read from the next boundary's link copy.
 *
 * Subtask (m, n), t_mid = floor((m+n)/2): initialised from the single state
 * q*_{m-1} (pruning, Sec. V-B).  The paper's displayed initialisation drops
 * the carried score (complete pruning, Def. 4); in float32 that is not exact,
 * because rounding depends on the magnitude of the running score.  This
 * oracle keeps it (retained pruning, Def. 3):
 *     OptProb_m(i) = (alpha + log A(q*_{m-1}, i)) + log B_m(i),
 * alpha = delta_{m-1}(q*_{m-1}), which reproduces vanilla's float32 values
 * along the optimal path exactly.  m = 0 starts from pi as in Alg. 2.
 * relative_init != 0 takes the paper's displayed initialisation instead,
 * OptProb_m(i) = log A(q*_{m-1}, i) + log B_m(i) (the carried score dropped);
 * its paths can differ from vanilla's where rounding decides a near tie.
 * MidState is tracked from t_mid + 1 on; q*_{t_mid} = MidState(q*_n).  The
 * anchor handed to the right child is OptProb_{t_mid}(q*_{t_mid}).
 *
 * Children (Alg. 1): (m, t_mid) and (t_mid+1, n) when n - m > 2, only
 * (m, t_mid) when n - m = 2, none otherwise.  Decoding calls = T - P' + 1.
 * shuffle_seed != 0 dequeues ready tasks in a random order.  trace (may be
 * NULL, room for 2*T ints) receives (m, n) of every subtask in decode order.
 */
int fvo_flash(int K, int T, int P, const float* log_pi, const float* log_a,
              const float* log_b, int64_t ld, int32_t* path, float* score,
              uint64_t shuffle_seed, fvo_stats* st, int32_t* trace, int relative_init)
{
    if (K < 1 || T < 1 || ld < K || !log_a || !log_b || !path || !score)
        return FVO_INVALID;
    fvo_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    int pp = eff_parallelism(T, P);

    float* opt = (float*)malloc(sizeof(float) * K);
    float* opt2 = (float*)malloc(sizeof(float) * K);
    float* best = (float*)malloc(sizeof(float) * K);
    int32_t* pre = (int32_t*)malloc(sizeof(int32_t) * K);
    int32_t* mid = (int32_t*)malloc(sizeof(int32_t) * K);
    int32_t* mid2 = (int32_t*)malloc(sizeof(int32_t) * K);
    float* snap = (float*)malloc(sizeof(float) * K);
    /* root copies at division points: OptProb for d = 0..P'-2, MidState link
     * for d = 1..P'-2 */
    float* dsnap = (float*)malloc(sizeof(float) * (size_t)K * (pp > 1 ? pp - 1 : 1));
    int32_t* link = (int32_t*)malloc(sizeof(int32_t) * (size_t)K * (pp > 1 ? pp - 1 : 1));
    uint8_t* written = (uint8_t*)calloc((size_t)T, 1);
    int64_t* e = (int64_t*)malloc(sizeof(int64_t) * pp);
    for (int d = 0; d < pp; ++d) e[d] = seg_end(T, pp, d);

    /* ---- root task ---- */
    st->tasks = 1;
    for (int j = 0; j < K; ++j) opt[j] = log_pi ? log_pi[j] + log_b[j] : log_b[j];
    int d_next = 0;                 /* next division point index to pass      */
    if (pp > 1 && e[0] == 0) { memcpy(dsnap, opt, sizeof(float) * K); d_next = 1; }
    for (int t = 1; t < T; ++t) {
        dense_step(K, opt, log_a, log_b + (size_t)t * ld, opt2, pre, best);
        st->candidates += (int64_t)K * K;
        /* t-1 is a division point: the state at it is the predecessor itself */
        int after_div = 0;
        for (int d = 0; d < pp - 1; ++d) if (e[d] == t - 1) after_div = 1;
        if (after_div) {
            for (int j = 0; j < K; ++j) mid2[j] = pre[j];
        } else if (pp > 1 && t > e[0] + 1) {
            for (int j = 0; j < K; ++j) mid2[j] = mid[pre[j]];
        }
        float* tf = opt; opt = opt2; opt2 = tf;
        int32_t* ti = mid; mid = mid2; mid2 = ti;
        if (d_next < pp - 1 && e[d_next] == t) {
            memcpy(dsnap + (size_t)d_next * K, opt, sizeof(float) * K);
            if (d_next >= 1) memcpy(link + (size_t)d_next * K, mid, sizeof(int32_t) * K);
            ++d_next;
        }
    }
    int qT = 0;
    for (int j = 1; j < K; ++j) if (opt[j] > opt[qT]) qT = j;
    *score = opt[qT];
    if (opt[qT] == -INFINITY) {
        for (int t = 0; t < T; ++t) path[t] = -1;
        free(opt); free(opt2); free(best); free(pre); free(mid); free(mid2); free(snap);
        free(dsnap); free(link); free(written); free(e);
        return FVO_INFEASIBLE;
    }
    path[T - 1] = qT;
    written[T - 1] = 1;
    float* alpha_d = (float*)malloc(sizeof(float) * pp);
    if (pp > 1) {
        int q = mid[qT];
        for (int d = pp - 2; d >= 0; --d) {
            path[e[d]] = q;
            if (written[e[d]]) st->resolved_twice++;
            written[e[d]] = 1;
            alpha_d[d] = dsnap[(size_t)d * K + q];
            if (d >= 1) q = link[(size_t)d * K + q];
        }
    }

    /* ---- InitialEnqueue: the P' first-level segments ---- */
    fvo_queue queue = {0};
    for (int d = 0; d < pp; ++d) {
        int m = d == 0 ? 0 : (int)e[d - 1] + 1, n = (int)e[d];
        if (n - m >= 1) {
            fvo_task tk = {m, n, d == 0 ? -1 : path[m - 1], d == 0 ? 0.0f : alpha_d[d - 1]};
            q_push(&queue, tk);
        }
    }
    if (queue.tail - queue.head > st->max_queue) st->max_queue = queue.tail - queue.head;

    /* ---- worker loop (Alg. 1), run serially ---- */
    uint64_t rng = shuffle_seed;
    fvo_task tk;
    while (q_pop(&queue, shuffle_seed ? &rng : NULL, &tk)) {
        int m = tk.m, n = tk.n, tmid = (m + n) / 2;
        if (trace) { trace[2 * (st->tasks - 1)] = m; trace[2 * (st->tasks - 1) + 1] = n; }
        st->tasks++;
        /* initialisation phase (pruned, anchored) */
        if (m == 0) {
            for (int i = 0; i < K; ++i) opt[i] = log_pi ? log_pi[i] + log_b[i] : log_b[i];
        } else {
            const float* row = log_a + (size_t)tk.q_prev * K;
            const float* b_m = log_b + (size_t)m * ld;
            for (int i = 0; i < K; ++i) {
                float c = relative_init ? row[i] : tk.alpha + row[i];
                opt[i] = c + b_m[i];
            }
            st->candidates += K;
        }
        if (tmid == m) memcpy(snap, opt, sizeof(float) * K);
        /* dynamic programming loop */
        for (int t = m + 1; t <= n; ++t) {
            dense_step(K, opt, log_a, log_b + (size_t)t * ld, opt2, pre, best);
            st->candidates += (int64_t)K * K;
            if (t == tmid + 1) {
                for (int j = 0; j < K; ++j) mid2[j] = pre[j];
            } else if (t > tmid + 1) {
                for (int j = 0; j < K; ++j) mid2[j] = mid[pre[j]];
            }
            float* tf = opt; opt = opt2; opt2 = tf;
            int32_t* ti = mid; mid = mid2; mid2 = ti;
            if (t == tmid) memcpy(snap, opt, sizeof(float) * K);
        }
        /* backtracking phase: the end state is already known */
        int qmid = mid[path[n]];
        path[tmid] = qmid;
        if (written[tmid]) st->resolved_twice++;
        written[tmid] = 1;
        float amid = snap[qmid];
        if (n - m > 2) {
            fvo_task l = {m, tmid, tk.q_prev, tk.alpha};
            fvo_task r = {tmid + 1, n, qmid, amid};
            q_push(&queue, l);
            q_push(&queue, r);
        } else if (n - m == 2) {
            fvo_task l = {m, tmid, tk.q_prev, tk.alpha};
            q_push(&queue, l);
        }
        if (queue.tail - queue.head > st->max_queue) st->max_queue = queue.tail - queue.head;
    }
    for (int t = 0; t < T; ++t) if (!written[t]) st->resolved_twice += 1000000; /* flag a hole */

    free(queue.v); free(alpha_d);
    free(opt); free(opt2); free(best); free(pre); free(mid); free(mid2); free(snap);
    free(dsnap); free(link); free(written); free(e);
    return FVO_OK;
}

/* ------------------------------------------------------------------------ */
/* FLASH-BS (Sec. V-C): the same task structure, with every step keeping only
 * the B best states.
 *
 * Beam entry = (State, OptProb, MidState).  At each step every destination j
 * is scored from the previous beam only:
 *     c(j) = max over beam entries b of  OptProb_b + log A(State_b, j),
 * predecessor = the lowest State attaining it, score(j) = c(j) + log B_t(j).
 * The next beam is built while the destinations are scanned in increasing j,
 * by the paper's insertion rule: below B entries insert; at B entries insert
 * only if the new score is strictly higher than the current minimum, which
 * is then evicted.  With increasing j this keeps exactly the top B by
 * (score descending, state ascending); -inf scores are never inserted.
 *
 * The beam holds at most B entries and is kept sorted by State.
 * A task's last step n evaluates only j = q*_n: q*_n is already known and
 * may have fallen out of a narrow beam.  If no beam state reaches q*_n, the
 * task is re-decoded exactly (all K states) and FVO_BEAM_FALLBACK is
 * returned.  The returned score is fvo_rescore of the returned path; the
 * root's own beam score is reported in *root_score.
 */
typedef struct { int32_t s; float v; int32_t a; } fvo_ent;

typedef struct { fvo_ent* e; int n; } fvo_beam_t;

static int ent_worse(const fvo_ent* x, const fvo_ent* y)
{   /* x ranks below y in (score desc, state asc) */
    if (x->v != y->v) return x->v < y->v;
    return x->s > y->s;
}

/* insert into a list kept in rank order (best first) of capacity B */
static void topb_insert(fvo_ent* list, int* n, int B, fvo_ent x)
{
    if (x.v == -INFINITY) return;
    if (*n == B) {
        if (!ent_worse(&list[B - 1], &x)) return;   /* not strictly better */
        --*n;
    }
    int k = *n;
    while (k > 0 && ent_worse(&list[k - 1], &x)) { list[k] = list[k - 1]; --k; }
    list[k] = x;
    ++*n;
}

static int ent_by_state(const void* a, const void* b)
{
    int32_t x = ((const fvo_ent*)a)->s, y = ((const fvo_ent*)b)->s;
    return (x > y) - (x < y);
}

/* scores[j] for all j -> beam (sorted by state), anc copied from anc[j] */
static void beam_from_scores(int K, int B, const float* sc, const int32_t* anc,
                             fvo_beam_t* out)
{
    out->n = 0;
    for (int j = 0; j < K; ++j) {
        fvo_ent x = {j, sc[j], anc ? anc[j] : -1};
        topb_insert(out->e, &out->n, B, x);
    }
    qsort(out->e, (size_t)out->n, sizeof(fvo_ent), ent_by_state);
}

/* one beam step over all destinations.  anc_mode: 0 none, 1 anc = predecessor
 * state, 2 anc = predecessor's anc.  A CSR model pushes the beam entries'
 * out-edges instead (entries in state order, each entry's edges in order,
 * a strictly larger candidate replacing a destination's current one): the
 * same maxima and predecessors as the dense scan with -inf for missing
 * edges, whose destinations never enter the beam.  c, w, seen: K-entry
 * scratch. */
static void beam_step(const fvo_model* M, int B, const fvo_beam_t* in, const float* b_t, int anc_mode,
                      fvo_beam_t* out, int64_t* cand, float* c, int32_t* w, uint8_t* seen)
{
    const int K = M->K;
    const float* log_a = M->log_a;
    out->n = 0;
    if (!log_a) {
        for (int j = 0; j < K; ++j) seen[j] = 0;
        for (int b = 0; b < in->n; ++b) {
            int s = in->e[b].s;
            for (int e = M->row_ptr[s]; e < M->row_ptr[s + 1]; ++e) {
                int j = M->col[e];
                float x = in->e[b].v + M->val[e];
                if (!seen[j] || x > c[j]) { c[j] = x; w[j] = b; seen[j] = 1; }
                ++*cand;
            }
        }
        for (int j = 0; j < K; ++j) {
            if (!seen[j]) continue;
            int b = w[j];
            fvo_ent y = {j, c[j] + b_t[j], anc_mode == 1 ? in->e[b].s : (anc_mode == 2 ? in->e[b].a : -1)};
            topb_insert(out->e, &out->n, B, y);
        }
        qsort(out->e, (size_t)out->n, sizeof(fvo_ent), ent_by_state);
        return;
    }
    for (int j = 0; j < K; ++j) {
        if (in->n == 0) break;
        float c = in->e[0].v + log_a[(size_t)in->e[0].s * K + j];
        int w = 0;
        for (int b = 1; b < in->n; ++b) {
            float x = in->e[b].v + log_a[(size_t)in->e[b].s * K + j];
            if (x > c) { c = x; w = b; }
        }
        fvo_ent y = {j, c + b_t[j], anc_mode == 1 ? in->e[w].s : (anc_mode == 2 ? in->e[w].a : -1)};
        topb_insert(out->e, &out->n, B, y);
    }
    *cand += (int64_t)K * in->n;
    qsort(out->e, (size_t)out->n, sizeof(fvo_ent), ent_by_state);
}

static const fvo_ent* beam_find(const fvo_beam_t* b, int s)
{
    for (int k = 0; k < b->n; ++k) if (b->e[k].s == s) return &b->e[k];
    return NULL;
}

static int beam_impl(const fvo_model* M, int T, int B, int P, const float* log_pi,
                     const float* log_b, int64_t ld, int32_t* path, float* score,
                     float* root_score, uint64_t shuffle_seed, fvo_stats* st, int32_t* n_fallback,
                     int relative_init)
{
    const int K = M->K;
    if (K < 1 || T < 1 || B < 1 || ld < K || !log_b || !path || !score)
        return FVO_INVALID;
    if (B > K) B = K;
    fvo_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    if (n_fallback) *n_fallback = 0;
    int pp = eff_parallelism(T, P);
    int64_t* e = (int64_t*)malloc(sizeof(int64_t) * pp);
    for (int d = 0; d < pp; ++d) e[d] = seg_end(T, pp, d);

    fvo_beam_t cur = {(fvo_ent*)malloc(sizeof(fvo_ent) * B), 0};
    fvo_beam_t nxt = {(fvo_ent*)malloc(sizeof(fvo_ent) * B), 0};
    fvo_beam_t snap = {(fvo_ent*)malloc(sizeof(fvo_ent) * B), 0};
    fvo_beam_t* rsnap = (fvo_beam_t*)malloc(sizeof(fvo_beam_t) * (pp > 1 ? pp - 1 : 1));
    for (int d = 0; d < pp - 1; ++d) { rsnap[d].e = (fvo_ent*)malloc(sizeof(fvo_ent) * B); rsnap[d].n = 0; }
    float* sc = (float*)malloc(sizeof(float) * K);
    float* cbuf = (float*)malloc(sizeof(float) * K);
    int32_t* wbuf = (int32_t*)malloc(sizeof(int32_t) * K);
    uint8_t* seen = (uint8_t*)malloc((size_t)K);
    uint8_t* written = (uint8_t*)calloc((size_t)T, 1);
    int rc = FVO_OK;

    /* ---- root ---- */
    st->tasks = 1;
    for (int j = 0; j < K; ++j) sc[j] = log_pi ? log_pi[j] + log_b[j] : log_b[j];
    beam_from_scores(K, B, sc, NULL, &cur);
    int d_next = 0;
    if (pp > 1 && e[0] == 0) {
        memcpy(rsnap[0].e, cur.e, sizeof(fvo_ent) * cur.n); rsnap[0].n = cur.n; d_next = 1;
    }
    for (int t = 1; t < T; ++t) {
        int after_div = 0;
        for (int d = 0; d < pp - 1; ++d) if (e[d] == t - 1) after_div = 1;
        int mode = after_div ? 1 : ((pp > 1 && t > e[0] + 1) ? 2 : 0);
        beam_step(M, B, &cur, log_b + (size_t)t * ld, mode, &nxt, &st->candidates, cbuf, wbuf, seen);
        fvo_beam_t tb = cur; cur = nxt; nxt = tb;
        if (d_next < pp - 1 && e[d_next] == t) {
            memcpy(rsnap[d_next].e, cur.e, sizeof(fvo_ent) * cur.n); rsnap[d_next].n = cur.n;
            ++d_next;
        }
    }
    if (cur.n == 0) {
        for (int t = 0; t < T; ++t) path[t] = -1;
        *score = -INFINITY;
        if (root_score) *root_score = -INFINITY;
        rc = FVO_INFEASIBLE;
        goto done;
    }
    {
        const fvo_ent* top = &cur.e[0];
        for (int k = 1; k < cur.n; ++k) if (ent_worse(top, &cur.e[k])) top = &cur.e[k];
        if (root_score) *root_score = top->v;
        path[T - 1] = top->s;
        written[T - 1] = 1;
        float* alpha_d = (float*)malloc(sizeof(float) * pp);
        if (pp > 1) {
            int q = top->a;
            for (int d = pp - 2; d >= 0; --d) {
                path[e[d]] = q;
                written[e[d]] = 1;
                const fvo_ent* x = beam_find(&rsnap[d], q);
                alpha_d[d] = x ? x->v : NAN;
                if (d >= 1) q = x ? x->a : -1;
            }
        }
        fvo_queue queue = {0};
        for (int d = 0; d < pp; ++d) {
            int m = d == 0 ? 0 : (int)e[d - 1] + 1, n = (int)e[d];
            if (n - m >= 1) {
                fvo_task tk = {m, n, d == 0 ? -1 : path[m - 1], d == 0 ? 0.0f : alpha_d[d - 1]};
                q_push(&queue, tk);
            }
        }
        free(alpha_d);
        uint64_t rng = shuffle_seed;
        fvo_task tk;
        float* opt = (float*)malloc(sizeof(float) * K);
        float* opt2 = (float*)malloc(sizeof(float) * K);
        float* best = (float*)malloc(sizeof(float) * K);
        int32_t* pre = (int32_t*)malloc(sizeof(int32_t) * K);
        int32_t* mid = (int32_t*)malloc(sizeof(int32_t) * K);
        int32_t* mid2 = (int32_t*)malloc(sizeof(int32_t) * K);
        while (q_pop(&queue, shuffle_seed ? &rng : NULL, &tk)) {
            int m = tk.m, n = tk.n, tmid = (m + n) / 2;
            int qn = path[n];
            st->tasks++;
            if (m == 0) {
                for (int i = 0; i < K; ++i) sc[i] = log_pi ? log_pi[i] + log_b[i] : log_b[i];
            } else {
                model_anchor_row(M, tk.q_prev, tk.alpha, relative_init, log_b + (size_t)m * ld, sc);
                st->candidates += K;
            }
            beam_from_scores(K, B, sc, NULL, &cur);
            if (tmid == m) { memcpy(snap.e, cur.e, sizeof(fvo_ent) * cur.n); snap.n = cur.n; }
            for (int t = m + 1; t < n; ++t) {
                int mode = t == tmid + 1 ? 1 : (t > tmid + 1 ? 2 : 0);
                beam_step(M, B, &cur, log_b + (size_t)t * ld, mode, &nxt, &st->candidates, cbuf, wbuf, seen);
                fvo_beam_t tb = cur; cur = nxt; nxt = tb;
                if (t == tmid) { memcpy(snap.e, cur.e, sizeof(fvo_ent) * cur.n); snap.n = cur.n; }
            }
            /* last step: only the known end state q*_n */
            int qmid = -1;
            float amid = NAN;
            int ok = 0;
            if (cur.n > 0) {
                float c = cur.e[0].v + model_a(M, cur.e[0].s, qn);
                int w = 0;
                for (int b = 1; b < cur.n; ++b) {
                    float x = cur.e[b].v + model_a(M, cur.e[b].s, qn);
                    if (x > c) { c = x; w = b; }
                }
                st->candidates += cur.n;
                if (c != -INFINITY) {
                    ok = 1;
                    qmid = (n == tmid + 1) ? cur.e[w].s : cur.e[w].a;
                    const fvo_ent* x = beam_find(&snap, qmid);
                    amid = x ? x->v : NAN;
                }
            }
            if (!ok) {
                /* exact re-decode of this task over all K states */
                rc = FVO_BEAM_FALLBACK;
                if (n_fallback) (*n_fallback)++;
                if (m == 0) {
                    for (int i = 0; i < K; ++i) opt[i] = log_pi ? log_pi[i] + log_b[i] : log_b[i];
                } else {
                    model_anchor_row(M, tk.q_prev, tk.alpha, relative_init, log_b + (size_t)m * ld, opt);
                }
                float* exsnap = sc;
                if (tmid == m) memcpy(exsnap, opt, sizeof(float) * K);
                for (int t = m + 1; t <= n; ++t) {
                    model_exact_step(M, opt, log_b + (size_t)t * ld, opt2, pre, best, seen);
                    st->candidates += (int64_t)K * K;
                    if (t == tmid + 1) for (int j = 0; j < K; ++j) mid2[j] = pre[j];
                    else if (t > tmid + 1) for (int j = 0; j < K; ++j) mid2[j] = mid[pre[j]];
                    float* tf = opt; opt = opt2; opt2 = tf;
                    int32_t* ti = mid; mid = mid2; mid2 = ti;
                    if (t == tmid) memcpy(exsnap, opt, sizeof(float) * K);
                }
                qmid = mid[qn];
                amid = exsnap[qmid];
            }
            path[tmid] = qmid;
            if (written[tmid]) st->resolved_twice++;
            written[tmid] = 1;
            if (n - m > 2) {
                fvo_task l = {m, tmid, tk.q_prev, tk.alpha};
                fvo_task r = {tmid + 1, n, qmid, amid};
                q_push(&queue, l);
                q_push(&queue, r);
            } else if (n - m == 2) {
                fvo_task l = {m, tmid, tk.q_prev, tk.alpha};
                q_push(&queue, l);
            }
            if (queue.tail - queue.head > st->max_queue) st->max_queue = queue.tail - queue.head;
        }
        free(opt); free(opt2); free(best); free(pre); free(mid); free(mid2);
        free(queue.v);
        for (int t = 0; t < T; ++t) if (!written[t]) st->resolved_twice += 1000000;
        *score = model_rescore(M, T, log_pi, log_b, ld, path);
    }
done:
    free(cur.e); free(nxt.e); free(snap.e);
    for (int d = 0; d < pp - 1; ++d) free(rsnap[d].e);
    free(rsnap); free(sc); free(cbuf); free(wbuf); free(seen); free(written); free(e);
    return rc;
}

int fvo_beam(int K, int T, int B, int P, const float* log_pi, const float* log_a,
             const float* log_b, int64_t ld, int32_t* path, float* score,
             float* root_score, uint64_t shuffle_seed, fvo_stats* st, int32_t* n_fallback,
             int relative_init)
{
    if (!log_a) return FVO_INVALID;
    fvo_model M = {K, log_a, NULL, NULL, NULL};
    return beam_impl(&M, T, B, P, log_pi, log_b, ld, path, score, root_score, shuffle_seed, st, n_fallback,
                     relative_init);
}

/* FLASH-BS on a CSR model (out-edges row_ptr[K+1], col, val; missing edges
 * -inf): the same procedure, each step pushing the beam's out-edges. */
int fvo_beam_csr(int K, int T, int B, int P, const float* log_pi, const int32_t* row_ptr,
                 const int32_t* col, const float* val, const float* log_b, int64_t ld,
                 int32_t* path, float* score, float* root_score, uint64_t shuffle_seed,
                 fvo_stats* st, int32_t* n_fallback, int relative_init)
{
    if (!row_ptr) return FVO_INVALID;
    fvo_model M = {K, NULL, row_ptr, col, val};
    return beam_impl(&M, T, B, P, log_pi, log_b, ld, path, score, root_score, shuffle_seed, st, n_fallback,
                     relative_init);
}

/* ------------------------------------------------------------------------ */
/* Backward of the Viterbi score S_b = sum of the decoded path's log-scores
 * (the path's rescore).  With the path held fixed, S_b is linear in the
 * inputs, so
 *   dS_b / d log B_b[t, j] = [j = q_{b,t}]                     (t < T_b)
 *   dS_b / d log A[i, j]   = c_b(i, j) = #{t >= 1 : (q_{b,t-1}, q_{b,t}) = (i, j)}
 *   dS_b / d log pi[j]     = [j = q_{b,0}]
 * (at a tie the decoded path's indicator is the subgradient).  With upstream
 * gradients g_b the shared parameters' gradients are summed over sequences in
 * increasing b, in float32, one term fl(g_b * c_b) per sequence:
 *   grad_log_a[i, j] = sum_b fl(g_b * c_b(i, j)).
 * accumulate != 0 adds that total to the existing value once (old + total);
 * grad_log_b is then old + g_b at the path entries.  Positions t >= T_b of
 * grad_log_b get 0 (or keep their value when accumulating).  A path entry
 * outside [0, K) (the -1 fill of an infeasible decode) contributes nothing,
 * nor does a transition that starts or ends at one. */
#define VALID_PAIR(i, j, K) ((i) >= 0 && (i) < (K) && (j) >= 0 && (j) < (K))
int fvo_backward(int K, int n, int Tmax, const int32_t* lengths, const int32_t* paths,
                 const float* grad_score, float* grad_log_b, float* grad_log_a,
                 float* grad_log_pi, int accumulate)
{
    if (K < 1 || n < 0 || Tmax < 0) return FVO_INVALID;
    for (int b = 0; b < n; ++b) if (lengths[b] < 0 || lengths[b] > Tmax) return FVO_INVALID;
    if (grad_log_b) {
        for (int b = 0; b < n; ++b) {
            for (int t = 0; t < Tmax; ++t) {
                float* row = grad_log_b + ((size_t)b * Tmax + t) * K;
                if (!accumulate) for (int j = 0; j < K; ++j) row[j] = 0.0f;
                if (t < lengths[b]) {
                    int q = paths[(size_t)b * Tmax + t];
                    if (q >= 0 && q < K) row[q] = accumulate ? row[q] + grad_score[b] : grad_score[b];
                }
            }
        }
    }
    if (grad_log_a) {
        float* total = (float*)calloc((size_t)K * K, sizeof(float));
        int32_t* cnt = (int32_t*)calloc((size_t)K * K, sizeof(int32_t));
        for (int b = 0; b < n; ++b) {
            const int32_t* q = paths + (size_t)b * Tmax;
            for (int t = 1; t < lengths[b]; ++t)
                if (VALID_PAIR(q[t - 1], q[t], K)) cnt[(size_t)q[t - 1] * K + q[t]]++;
            for (int t = 1; t < lengths[b]; ++t) {
                if (!VALID_PAIR(q[t - 1], q[t], K)) continue;
                size_t c = (size_t)q[t - 1] * K + q[t];
                if (cnt[c]) {
                    total[c] = total[c] + grad_score[b] * (float)cnt[c];
                    cnt[c] = 0;
                }
            }
        }
        for (size_t c = 0; c < (size_t)K * K; ++c)
            grad_log_a[c] = accumulate ? grad_log_a[c] + total[c] : total[c];
        free(total); free(cnt);
    }
    if (grad_log_pi) {
        float* total = (float*)calloc((size_t)K, sizeof(float));
        for (int b = 0; b < n; ++b)
            if (lengths[b] > 0) {
                int q = paths[(size_t)b * Tmax];
                if (q >= 0 && q < K) total[q] = total[q] + grad_score[b];
            }
        for (int j = 0; j < K; ++j) grad_log_pi[j] = accumulate ? grad_log_pi[j] + total[j] : total[j];
        free(total);
    }
    return FVO_OK;
}
