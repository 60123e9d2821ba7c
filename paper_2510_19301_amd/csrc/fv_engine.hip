// Persistent lock-step decoding engine for dense transition models (gfx950).
//
// One cooperative launch runs every step of every decoding task of a batch:
// vanilla passes (Sec. III-A), FLASH root passes and FLASH subtasks
// (Alg. 1 / Alg. 2).  A "row" is one task in flight; at every global step each
// row advances one time step.  Blocks 0..n_compute_blocks-1 execute the rows
// of the current step; the last block is the scheduler, which meanwhile
// builds the next step's row list (task creation, slot reuse).  One grid
// barrier separates steps.
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

__device__ __forceinline__ unsigned long long order_key(float v, int32_t j) {
    if (v == 0.0f) v = 0.0f;  // -0 and +0 compare equal; the lower index must win
    uint32_t b = __float_as_uint(v);
    uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((unsigned long long)o << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
}

__device__ __forceinline__ float* slot_delta(const EngineArgs& a, int32_t slot, int32_t parity) {
    return a.slot_base + (int64_t)slot * a.slot_floats + (int64_t)parity * a.Kp;
}
__device__ __forceinline__ int32_t* slot_anc(const EngineArgs& a, int32_t slot, int32_t parity) {
    return reinterpret_cast<int32_t*>(a.slot_base + (int64_t)slot * a.slot_floats +
                                      (int64_t)(2 + parity) * a.Kp);
}
__device__ __forceinline__ float* slot_snap(const EngineArgs& a, int32_t slot) {
    return a.slot_base + (int64_t)slot * a.slot_floats + (int64_t)4 * a.Kp;
}
__device__ __forceinline__ float* root_dsnap(const EngineArgs& a, const SeqInfo& s, int32_t d) {
    return a.root_copy + (s.root_off + d) * (int64_t)a.Kp;
}
__device__ __forceinline__ int32_t* root_link(const EngineArgs& a, const SeqInfo& s, int32_t d) {
    return reinterpret_cast<int32_t*>(a.root_copy + (s.root_off + (s.pp - 1) + d) * (int64_t)a.Kp);
}

template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- grid barrier
// Monotone arrival counter: block arrives once per step and waits until all
// blocks of this step arrived.  Bounded spin: on overrun the error flag is
// raised and every block leaves the loop.
__device__ bool grid_barrier(EngineState* st, uint32_t n_blocks, uint32_t& target,
                             int64_t spin_limit) {
    __threadfence();
    __syncthreads();
    __shared__ int s_err;
    if (threadIdx.x == 0) {
        target += n_blocks;
        __hip_atomic_fetch_add(&st->barrier, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int64_t spins = 0;
        int err = 0;
        while (__hip_atomic_load(&st->barrier, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin_limit) {
                __hip_atomic_store(&st->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                err = 1;
                break;
            }
            if ((spins & 255) == 0 &&
                __hip_atomic_load(&st->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                err = 1;
                break;
            }
        }
        if (!err) err = __hip_atomic_load(&st->error, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        s_err = err;
    }
    __syncthreads();
    return s_err == 0;
}

// ---------------------------------------------------------------- row flags
__device__ Row make_dense_row(int32_t seq, int32_t kind, int32_t m, int32_t n, int32_t t,
                              int32_t slot, int32_t T, int32_t pp) {
    Row r;
    r.seq = seq; r.kind = kind; r.m = m; r.n = n; r.t = t; r.slot = slot;
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

__device__ Row make_light_row(int32_t seq, int32_t kind, int32_t m, int32_t n, int32_t t,
                              int32_t slot, int32_t op, int32_t T, int32_t pp) {
    Row r;
    r.seq = seq; r.kind = kind; r.m = m; r.n = n; r.t = t; r.slot = slot; r.aux = op;
    int32_t f = 0;
    if (op == L_INIT) {
        if (kind == KIND_SUB && ((m + n) >> 1) == m) f |= F_SNAP_SUB;
        if (kind == KIND_ROOT && pp >= 2 && seg_end(T, pp, 0) == 0) f |= F_SNAP_ROOT;
        if (kind != KIND_SUB && T == 1) f |= F_FINAL;
    }
    r.flags = f;
    return r;
}

// ---------------------------------------------------------------- dense tile
// Partial (max, group) of 16 columns over predecessors [s0, s1) for the
// lane's row; drow = the row's delta_{t-1}, Ap = padded row-major log A.
__device__ __forceinline__ void tile_partial(const float* __restrict__ Ap, int32_t Kp, int32_t j0,
                                             const float* drow, int32_t s0, int32_t s1,
                                             float (&m)[kTileCols], int32_t (&g)[kTileCols]) {
#pragma unroll
    for (int c = 0; c < kTileCols; ++c) { m[c] = -INFINITY; g[c] = s0 / kGroup; }
    for (int32_t i0 = s0; i0 < s1; i0 += kGroup) {
        float gm[kTileCols];
#pragma unroll
        for (int c = 0; c < kTileCols; ++c) gm[c] = -INFINITY;
#pragma unroll
        for (int k = 0; k < kGroup; k += 4) {
            const float4 d = *reinterpret_cast<const float4*>(drow + i0 + k);
            const float* a0 = Ap + (int64_t)(i0 + k) * Kp + j0;
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

struct TileLds {
    float m[kWaves][kTileCols][kTileRows];
    int32_t g[kWaves][kTileCols][kTileRows];
};

__device__ void dense_tile(const EngineArgs& a, const float* __restrict__ Ap, const Row* rows,
                           int32_t nrows, int32_t tile, TileLds& lds) {
    const int32_t ncb = a.Kp / kTileCols;
    const int32_t rg = tile / ncb;
    const int32_t j0 = (tile - rg * ncb) * kTileCols;
    const int32_t lane = threadIdx.x & 63;
    const int32_t wave = threadIdx.x >> 6;
    const int32_t ridx = rg * kTileRows + lane;
    const bool valid = ridx < nrows;
    const Row r = rows[valid ? ridx : rg * kTileRows];
    const float* drow = slot_delta(a, r.slot, (r.t - 1) & 1);

    const int32_t split = a.Kp / kWaves;
    const int32_t s0 = __builtin_amdgcn_readfirstlane(wave * split);
    float m[kTileCols];
    int32_t g[kTileCols];
    tile_partial(Ap, a.Kp, __builtin_amdgcn_readfirstlane(j0), drow, s0, s0 + split, m, g);
#pragma unroll
    for (int c = 0; c < kTileCols; ++c) {
        lds.m[wave][c][lane] = m[c];
        lds.g[wave][c][lane] = g[c];
    }
    __syncthreads();

    if (valid) {
        const SeqInfo& sq = a.seqs[r.seq];
        const int32_t t = r.t;
        const float* bt = sq.log_b + (int64_t)t * sq.ld;
        float* dcur = slot_delta(a, r.slot, t & 1);
        int32_t* acur = nullptr;
        const int32_t* aprev = nullptr;
        if (a.has_anc) {
            acur = slot_anc(a, r.slot, t & 1);
            aprev = slot_anc(a, r.slot, (t - 1) & 1);
        }
        unsigned long long best_key = 0;
        const int32_t cq = wave * 4;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int32_t c = cq + cc;
            const int32_t j = j0 + c;
            if (j >= a.K) break;
            float mv = lds.m[0][c][lane];
            int32_t gi = lds.g[0][c][lane];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) {
                const float x = lds.m[w][c][lane];
                if (x > mv) { mv = x; gi = lds.g[w][c][lane]; }
            }
            float val = mv;
            int32_t psi = 0;
            if ((r.flags & F_NEED_ARG) || mv == 0.0f) {
                const int32_t src0 = gi * kGroup;
                const float* ac = a.Acol + (int64_t)src0 * a.Kp + j;   // column j, rows src0..
                const float* dp = drow + src0;
                psi = -1;
#pragma unroll
                for (int k = 0; k < kGroup; k += 4) {
                    const float4 dv = *reinterpret_cast<const float4*>(dp + k);
                    const float a0 = ac[(int64_t)k * a.Kp], a1 = ac[(int64_t)(k + 1) * a.Kp];
                    const float a2 = ac[(int64_t)(k + 2) * a.Kp], a3 = ac[(int64_t)(k + 3) * a.Kp];
                    const float x0 = dv.x + a0, x1 = dv.y + a1, x2 = dv.z + a2, x3 = dv.w + a3;
                    if (psi < 0 && x0 == mv) { psi = src0 + k; val = x0; }
                    if (psi < 0 && x1 == mv) { psi = src0 + k + 1; val = x1; }
                    if (psi < 0 && x2 == mv) { psi = src0 + k + 2; val = x2; }
                    if (psi < 0 && x3 == mv) { psi = src0 + k + 3; val = x3; }
                }
                if (psi < 0) psi = src0;  // unreachable for finite/-inf inputs
            }
            const float dnew = val + bt[j];
            dcur[j] = dnew;
            const int32_t f = r.flags;
            if (f & F_PSI_TABLE) a.psi16[sq.psi_off + (int64_t)t * a.K + j] = (uint16_t)psi;
            int32_t anc = 0;
            if (f & F_ANC_FIRST) { anc = psi; acur[j] = anc; }
            else if (f & F_ANC_CHAIN) { anc = aprev[psi]; acur[j] = anc; }
            if (f & F_SNAP_SUB) slot_snap(a, r.slot)[j] = dnew;
            if (f & F_SNAP_ROOT) {
                root_dsnap(a, sq, r.aux)[j] = dnew;
                if (r.aux >= 1) root_link(a, sq, r.aux)[j] = anc;
            }
            if (f & F_FINAL) {
                const unsigned long long k = order_key(dnew, j);
                if (k > best_key) best_key = k;
            }
        }
        if (r.flags & F_FINAL) atomicMax(&a.keys[r.seq], best_key);
    }
    __syncthreads();
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

__device__ void light_row(const EngineArgs& a, const float* __restrict__ Ap, const Row& r) {
    const int32_t lane = threadIdx.x & 63;
    SeqInfo& sq = a.seqs[r.seq];
    const int32_t K = a.K, Kp = a.Kp;
    if (r.aux == L_INIT) {
        const int32_t m = r.m;
        float* dst = slot_delta(a, r.slot, m & 1);
        float* oth = slot_delta(a, r.slot, (m + 1) & 1);
        const float* bm = sq.log_b + (int64_t)m * sq.ld;
        int32_t q = -1;
        float alpha = 0.0f;
        if (m > 0) {
            q = sq.path[m - 1];
            alpha = a.alpha_at[sq.alpha_off + m - 1];
        }
        unsigned long long best_key = 0;
        for (int32_t j = lane; j < Kp; j += 64) {
            float v = -INFINITY;
            if (j < K) {
                if (m == 0) v = a.log_pi ? a.log_pi[j] + bm[j] : bm[j];
                else if (q >= 0) { const float c = alpha + Ap[(int64_t)q * Kp + j]; v = c + bm[j]; }
                if (r.flags & F_SNAP_SUB) slot_snap(a, r.slot)[j] = v;
                if (r.flags & F_SNAP_ROOT) root_dsnap(a, sq, 0)[j] = v;
                if (r.flags & F_FINAL) {
                    const unsigned long long k = order_key(v, j);
                    if (k > best_key) best_key = k;
                }
            } else {
                oth[j] = -INFINITY;
            }
            dst[j] = v;
        }
        if (r.flags & F_FINAL) {
            for (int off = 32; off >= 1; off >>= 1) {
                const unsigned long long o = __shfl_xor(best_key, off, 64);
                if (o > best_key) best_key = o;
            }
            if (lane == 0) atomicMax(&a.keys[r.seq], best_key);
        }
    } else if (r.aux == L_END) {
        // only the known end state q*_n is evaluated at a subtask's last step
        if (ld_relaxed(&sq.status) != FV_OK) return;
        const int32_t n = r.n, tmid = (r.m + r.n) >> 1;
        const int32_t qn = sq.path[n];
        if (qn < 0) return;
        const float* dprev = slot_delta(a, r.slot, (n - 1) & 1);
        const float* ac = a.Acol + qn;  // column q*_n of log A
        float best = -INFINITY;
        int32_t arg = 0x7fffffff;
        for (int32_t i = lane; i < K; i += 64) {
            const float x = dprev[i] + ac[(int64_t)i * Kp];
            if (arg == 0x7fffffff || x > best) { best = x; arg = i; }
        }
        wave_argmax(best, arg);
        if (lane == 0) {
            const int32_t qmid = (n == tmid + 1) ? arg : slot_anc(a, r.slot, (n - 1) & 1)[arg];
            sq.path[tmid] = qmid;
            a.alpha_at[sq.alpha_off + tmid] = slot_snap(a, r.slot)[qmid];
        }
    } else {  // L_FINALIZE
        const int32_t T = sq.T;
        const unsigned long long key = a.keys[r.seq];
        int32_t qT = (int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
        if (qT < 0 || qT >= K) qT = 0;  // no key arrived: cannot happen for T >= 1
        const float sc = slot_delta(a, r.slot, (T - 1) & 1)[qT];
        if (sc == -INFINITY) {
            for (int32_t t = lane; t < T; t += 64) sq.path[t] = -1;
            if (lane == 0) {
                *sq.score = sc;
                __hip_atomic_store(&sq.status, (int32_t)FV_E_INFEASIBLE, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            return;
        }
        if (lane == 0) {
            *sq.score = sc;
            sq.path[T - 1] = qT;
            if (r.kind == KIND_ROOT && sq.pp >= 2) {
                int32_t q = slot_anc(a, r.slot, (T - 1) & 1)[qT];
                for (int32_t d = sq.pp - 2; d >= 0; --d) {
                    const int64_t e = seg_end(T, sq.pp, d);
                    sq.path[e] = q;
                    a.alpha_at[sq.alpha_off + e] = root_dsnap(a, sq, d)[q];
                    if (d >= 1) q = root_link(a, sq, d)[q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- scheduler
struct SchedLds {
    int32_t scan[4][kBlock];
    int32_t tot[4];
};

// exclusive block scan of four counters at once
__device__ void block_scan4(int32_t (&v)[4], int32_t (&tot)[4], SchedLds& lds) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) lds.scan[k][tid] = v[k];
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int32_t add[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) add[k] = tid >= off ? lds.scan[k][tid - off] : 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) lds.scan[k][tid] += add[k];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        tot[k] = lds.scan[k][kBlock - 1];
        v[k] = lds.scan[k][tid] - v[k];
    }
    __syncthreads();
}

// What a row of step s turns into at step s+1.
struct Next {
    int32_t has_full, has_light, freed, spawn;
    Row full, light;
};

__device__ int32_t root_segments(int32_t T, int32_t pp) {
    int32_t c = 0;
    for (int32_t d = 0; d < pp; ++d) {
        const int64_t m = d == 0 ? 0 : seg_end(T, pp, d - 1) + 1, n = seg_end(T, pp, d);
        if (n - m >= 1) ++c;
    }
    return c;
}

__device__ Next classify(const EngineArgs& a, const Row& r, bool from_full) {
    Next x;
    x.has_full = x.has_light = x.freed = x.spawn = 0;
    const SeqInfo& sq = a.seqs[r.seq];
    const int32_t T = sq.T, pp = sq.pp;
    if (from_full) {
        if (r.kind == KIND_SUB) {
            if (r.t + 1 < r.n) { x.has_full = 1; x.full = make_dense_row(r.seq, r.kind, r.m, r.n, r.t + 1, r.slot, T, pp); }
            else { x.has_light = 1; x.light = make_light_row(r.seq, r.kind, r.m, r.n, r.n, r.slot, L_END, T, pp); }
        } else {
            if (r.t + 1 < T) { x.has_full = 1; x.full = make_dense_row(r.seq, r.kind, r.m, r.n, r.t + 1, r.slot, T, pp); }
            else { x.has_light = 1; x.light = make_light_row(r.seq, r.kind, r.m, r.n, T, r.slot, L_FINALIZE, T, pp); }
        }
    } else if (r.aux == L_INIT) {
        if (r.kind == KIND_SUB) {
            if (r.m + 1 < r.n) { x.has_full = 1; x.full = make_dense_row(r.seq, r.kind, r.m, r.n, r.m + 1, r.slot, T, pp); }
            else { x.has_light = 1; x.light = make_light_row(r.seq, r.kind, r.m, r.n, r.n, r.slot, L_END, T, pp); }
        } else {
            if (T > 1) { x.has_full = 1; x.full = make_dense_row(r.seq, r.kind, r.m, r.n, 1, r.slot, T, pp); }
            else { x.has_light = 1; x.light = make_light_row(r.seq, r.kind, r.m, r.n, T, r.slot, L_FINALIZE, T, pp); }
        }
    } else if (r.aux == L_END) {
        x.freed = 1;
        const int32_t len = r.n - r.m;
        x.spawn = len > 2 ? 2 : (len == 2 ? 1 : 0);
    } else {  // L_FINALIZE
        x.freed = 1;
        if (r.kind == KIND_ROOT && pp >= 2) x.spawn = root_segments(T, pp);
    }
    return x;
}

__device__ void write_spawns(const EngineArgs& a, const Row& r, int64_t pos) {
    if (r.aux == L_END) {
        const int32_t tmid = (r.m + r.n) >> 1;
        const int32_t len = r.n - r.m;
        if (len >= 2) a.queue[pos++] = Task{r.seq, KIND_SUB, r.m, tmid};
        if (len > 2) a.queue[pos++] = Task{r.seq, KIND_SUB, tmid + 1, r.n};
    } else {
        const SeqInfo& sq = a.seqs[r.seq];
        const int32_t T = sq.T, pp = sq.pp;
        for (int32_t d = 0; d < pp; ++d) {
            const int64_t m = d == 0 ? 0 : seg_end(T, pp, d - 1) + 1, n = seg_end(T, pp, d);
            if (n - m >= 1) a.queue[pos++] = Task{r.seq, KIND_SUB, (int32_t)m, (int32_t)n};
        }
    }
}

__device__ void scheduler(const EngineArgs& a, int32_t s, SchedLds& lds) {
    const int cur = s & 1, nxt = cur ^ 1;
    EngineState* st = a.st;
    const int32_t nf = ld_relaxed(&st->n_full[cur]);
    const int32_t nl = ld_relaxed(&st->n_light[cur]);
    const Row* F = a.rows_full + (int64_t)cur * a.max_rows;
    const Row* L = a.rows_light + (int64_t)cur * a.max_rows;
    Row* F2 = a.rows_full + (int64_t)nxt * a.max_rows;
    Row* L2 = a.rows_light + (int64_t)nxt * a.max_rows;
    const int32_t total = nf + nl;
    const int32_t per = (total + kBlock - 1) / kBlock;
    const int32_t lo = min(total, (int32_t)threadIdx.x * per), hi = min(total, lo + per);

    int32_t cnt[4] = {0, 0, 0, 0};  // full, light, freed, spawned
    for (int32_t i = lo; i < hi; ++i) {
        const bool ff = i < nf;
        const Next x = classify(a, ff ? F[i] : L[i - nf], ff);
        cnt[0] += x.has_full; cnt[1] += x.has_light; cnt[2] += x.freed; cnt[3] += x.spawn;
    }
    int32_t tot[4];
    block_scan4(cnt, tot, lds);
    const int32_t n_free0 = ld_relaxed(&st->n_free);
    const int32_t q_tail0 = ld_relaxed(&st->q_tail);
    const int32_t q_head = ld_relaxed(&st->q_head);
    for (int32_t i = lo; i < hi; ++i) {
        const bool ff = i < nf;
        const Row r = ff ? F[i] : L[i - nf];
        const Next x = classify(a, r, ff);
        if (x.has_full) F2[cnt[0]++] = x.full;
        if (x.has_light) L2[cnt[1]++] = x.light;
        if (x.freed) a.free_stack[n_free0 + cnt[2]++] = r.slot;
        if (x.spawn) { write_spawns(a, r, (int64_t)q_tail0 + cnt[3]); cnt[3] += x.spawn; }
    }
    __threadfence_block();
    __syncthreads();
    const int32_t n_free = n_free0 + tot[2];
    const int32_t q_tail = q_tail0 + tot[3];
    const int32_t n_admit = min(n_free, q_tail - q_head);
    for (int32_t k = threadIdx.x; k < n_admit; k += kBlock) {
        const Task tk = a.queue[q_head + k];
        const int32_t slot = a.free_stack[n_free - 1 - k];
        const SeqInfo& sq = a.seqs[tk.seq];
        L2[tot[1] + k] = make_light_row(tk.seq, tk.kind, tk.m, tk.n, tk.m, slot, L_INIT, sq.T, sq.pp);
    }
    if (threadIdx.x == 0) {
        st->q_head = q_head + n_admit;
        st->q_tail = q_tail;
        st->n_free = n_free - n_admit;
        st->n_full[nxt] = tot[0];
        st->n_light[nxt] = tot[1] + n_admit;
        const int32_t inflight = tot[0] + tot[1] + n_admit;
        if (inflight > st->max_rows) st->max_rows = inflight;
    }
}

// ---------------------------------------------------------------- engine
union EngineLds {
    TileLds tile;
    SchedLds sched;
};

extern "C" __global__ __launch_bounds__(kBlock) void fv_engine_kernel(const float* __restrict__ Ap,
                                                                      EngineArgs a) {
    __shared__ EngineLds lds;
    uint32_t target = 0;
    const uint32_t n_blocks = gridDim.x;
    int32_t s = 0;
    for (;; ++s) {
        const int cur = s & 1;
        const int32_t nf = ld_relaxed(&a.st->n_full[cur]);
        const int32_t nl = ld_relaxed(&a.st->n_light[cur]);
        if (nf + nl == 0) break;
        if (s > a.max_steps) {  // schedule longer than any valid one: report, stop
            if (blockIdx.x == 0 && threadIdx.x == 0) a.st->error = 2;
            break;
        }
        if ((int32_t)blockIdx.x == a.n_compute_blocks) {
            scheduler(a, s, lds.sched);
        } else {
            const Row* F = a.rows_full + (int64_t)cur * a.max_rows;
            const Row* L = a.rows_light + (int64_t)cur * a.max_rows;
            const int32_t n_tiles = ((nf + kTileRows - 1) / kTileRows) * (a.Kp / kTileCols);
            const int32_t n_light_items = (nl + kWaves - 1) / kWaves;
            const int32_t n_items = n_tiles + n_light_items;
            for (int32_t it = blockIdx.x; it < n_items; it += a.n_compute_blocks) {
                if (it < n_tiles) {
                    dense_tile(a, Ap, F, nf, it, lds.tile);
                } else {
                    const int32_t li = (it - n_tiles) * kWaves + (threadIdx.x >> 6);
                    if (li < nl) light_row(a, Ap, L[li]);
                }
            }
        }
        if (!grid_barrier(a.st, n_blocks, target, a.spin_limit)) break;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.st->steps = s;
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

// Per-sequence setup and the first step's row list (one block).

extern "C" __global__ __launch_bounds__(kBlock) void fv_setup_kernel(EngineArgs a, SetupArgs sa) {
    __shared__ int64_t scan[3][kBlock];
    __shared__ int32_t s_bad;
    const int tid = threadIdx.x;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    int64_t base[3] = {0, 0, 0};
    int32_t n_tasks = 0;
    for (int32_t b0 = 0; b0 < sa.n_seqs; b0 += kBlock) {
        const int32_t b = b0 + tid;
        int64_t v[3] = {0, 0, 0};
        fv_seq d{};
        int32_t pp = 1;
        if (b < sa.n_seqs) {
            d = sa.seqs_dev[b];
            if (d.T < 0 || d.model != 0 || (d.T > 0 && (d.ld < sa.K || !d.log_b || !d.path)) || !d.score) s_bad = 1;
            const int32_t T = d.T < 0 ? 0 : d.T;
            pp = sa.kind == KIND_ROOT ? eff_parallelism(T, sa.P) : 1;
            v[0] = T;
            v[1] = sa.kind == KIND_ROOT ? 2 * (int64_t)(pp - 1) : 0;
            v[2] = sa.kind == KIND_VANILLA ? (int64_t)T * sa.K : 0;
        }
        for (int k = 0; k < 3; ++k) scan[k][tid] = v[k];
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            int64_t add[3];
            for (int k = 0; k < 3; ++k) add[k] = tid >= off ? scan[k][tid - off] : 0;
            __syncthreads();
            for (int k = 0; k < 3; ++k) scan[k][tid] += add[k];
            __syncthreads();
        }
        if (b < sa.n_seqs) {
            SeqInfo si;
            si.log_b = d.log_b; si.ld = d.ld; si.path = d.path; si.score = d.score;
            si.T = d.T < 0 ? 0 : d.T;
            si.pp = pp;
            si.alpha_off = base[0] + scan[0][tid] - v[0];
            si.root_off = base[1] + scan[1][tid] - v[1];
            si.psi_off = base[2] + scan[2][tid] - v[2];
            si.status = FV_OK;
            si.pad_ = 0;
            a.seqs[b] = si;
            a.keys[b] = 0ull;
            if (si.T == 0 && d.score) *d.score = 0.0f;
        }
        for (int k = 0; k < 3; ++k) base[k] += scan[k][kBlock - 1];
        __syncthreads();
    }
    if (base[0] != sa.host_sum_T || base[1] != sa.host_sum_root || base[2] != sa.host_sum_psi) s_bad = 1;
    __syncthreads();
    const bool bad = s_bad != 0;
    // task queue: every non-empty sequence's full-length pass
    for (int32_t b0 = 0; b0 < sa.n_seqs; b0 += kBlock) {
        const int32_t b = b0 + tid;
        int32_t has = 0;
        if (b < sa.n_seqs) {
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
    for (int32_t k = tid; k < a.n_slots; k += kBlock) a.free_stack[k] = a.n_slots - 1 - k;
    const int32_t n_admit = min(a.n_slots, n_tasks);
    for (int32_t k = tid; k < n_admit; k += kBlock) {
        const Task tk = a.queue[k];
        const int32_t slot = a.free_stack[a.n_slots - 1 - k];
        const SeqInfo& sq = a.seqs[tk.seq];
        a.rows_light[k] = make_light_row(tk.seq, tk.kind, tk.m, tk.n, 0, slot, L_INIT, sq.T, sq.pp);
    }
    if (tid == 0) {
        EngineState* st = a.st;
        st->barrier = 0;
        st->error = 0;
        st->n_full[0] = 0; st->n_full[1] = 0;
        st->n_light[0] = n_admit; st->n_light[1] = 0;
        st->q_head = n_admit;
        st->q_tail = n_tasks;
        st->n_free = a.n_slots - n_admit;
        st->steps = 0;
        st->max_rows = n_admit;
    }
}

// Vanilla backtracking through the packed table and per-sequence status.
extern "C" __global__ __launch_bounds__(kBlock) void fv_finish_kernel(EngineArgs a, int32_t* status) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= a.n_seqs) return;
    SeqInfo& sq = a.seqs[b];
    int32_t stv = sq.status;
    if (a.st->error) stv = FV_E_DEVICE;
    if (stv == FV_OK && a.method == FV_VANILLA && sq.T > 1) {
        int32_t q = sq.path[sq.T - 1];
        const uint16_t* tab = a.psi16 + sq.psi_off;
        for (int32_t t = sq.T - 1; t > 0; --t) {
            q = tab[(int64_t)t * a.K + q];
            sq.path[t - 1] = q;
        }
    }
    if (status) status[b] = stv;
}

}  // namespace fv
