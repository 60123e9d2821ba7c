// Backward of the Viterbi score (the decoded path's summed log-scores).
//
// With the decoded path held fixed the score is linear in the inputs (the
// recurrence of Sec. III-A evaluated along one path), so the gradients are
// path indicators and transition counts:
//   grad_log_b[b][t][j] = g_b * [j == q_{b,t}]                 (t < T_b)
//   grad_log_a[i][j]    = sum over b ascending of fl(g_b * c_b(i, j)),
//                         c_b(i, j) = #{t >= 1 : (q_{b,t-1}, q_{b,t}) = (i, j)}
//   grad_log_pi[j]      = sum over b ascending of g_b * [q_{b,0} == j]
// Shared-parameter sums run in a fixed order (one float32 term per sequence,
// sequences in increasing b), so every run gives the same bits.
//
// Kernels:
//   fill   grad_log_b one-hot rows (HBM write bound: n*Tmax*K*4 bytes)
//   dedup  one block per sequence: its transition cells i*K+j sorted in LDS,
//          run lengths = c_b(i, j)
//   fold   one block walks the sequences in order and adds fl(g_b * c) to
//          the cells of each (cells of one sequence are distinct, so the
//          threads of a block never collide; a block barrier orders b)
//   pi     one thread folds the start states in order
//   apply  out = total, or out + total when accumulating
#include "fv_internal.h"

namespace fv {

constexpr int kBwdBlock = 1024;
constexpr int32_t kBwdMaxPairs = 16384;  // transitions per sequence sorted in LDS (64 KiB)

__device__ __forceinline__ int32_t clamp_len(int32_t L, int32_t Tmax) { return L < 0 ? 0 : (L > Tmax ? Tmax : L); }

// One wave per (b, t) row of grad_log_b.
extern "C" __global__ __launch_bounds__(kBlock) void fv_bwd_fill_kernel(int32_t K, int32_t n, int32_t Tmax,
                                                                        const int32_t* __restrict__ lengths,
                                                                        const int32_t* __restrict__ paths,
                                                                        const float* __restrict__ g,
                                                                        float* __restrict__ out, int32_t accumulate,
                                                                        int32_t vec4) {
    const int64_t rows = (int64_t)n * Tmax;
    const int32_t lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t stride = ((int64_t)gridDim.x * kBlock) >> 6;
    for (int64_t r = wave0; r < rows; r += stride) {
        const int32_t b = (int32_t)(r / Tmax), t = (int32_t)(r - (int64_t)b * Tmax);
        const bool live = t < clamp_len(lengths[b], Tmax);
        const int32_t q = live ? paths[r] : -1;
        const float gb = live ? g[b] : 0.0f;
        float* row = out + r * K;
        if (accumulate) {
            if (lane == 0 && q >= 0 && q < K) row[q] = row[q] + gb;
        } else if (vec4) {
            float4* row4 = reinterpret_cast<float4*>(row);
            for (int32_t j4 = lane; j4 < K / 4; j4 += 64) {
                const int32_t j = j4 * 4;
                float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (q == j) v.x = gb;
                if (q == j + 1) v.y = gb;
                if (q == j + 2) v.z = gb;
                if (q == j + 3) v.w = gb;
                row4[j4] = v;
            }
        } else {
            for (int32_t j = lane; j < K; j += 64) row[j] = (j == q) ? gb : 0.0f;
        }
    }
}

// Per sequence: the distinct transition cells and their counts, in cell order.
extern "C" __global__ __launch_bounds__(kBwdBlock) void fv_bwd_dedup_kernel(int32_t K, int32_t Tmax,
                                                                            const int32_t* __restrict__ lengths,
                                                                            const int32_t* __restrict__ paths,
                                                                            uint32_t* __restrict__ ent_key,
                                                                            int32_t* __restrict__ ent_cnt,
                                                                            int32_t* __restrict__ n_ent) {
    __shared__ uint32_t keys[kBwdMaxPairs];
    __shared__ int32_t wsum[kBwdBlock / 64];
    __shared__ int32_t s_base;
    const int32_t b = blockIdx.x, tid = threadIdx.x;
    const int32_t T = clamp_len(lengths[b], Tmax);
    const int32_t np = T > 1 ? T - 1 : 0;
    int32_t pw = 1;
    while (pw < np) pw <<= 1;
    const int32_t* q = paths + (int64_t)b * Tmax;
    const uint32_t kNone = 0xFFFFFFFFu;  // above every cell (K*K < 2^32 - 1)
    for (int32_t k = tid; k < pw; k += kBwdBlock) {
        uint32_t key = kNone;
        if (k < np) {
            const int32_t i = q[k], j = q[k + 1];
            if (i >= 0 && i < K && j >= 0 && j < K) key = (uint32_t)i * (uint32_t)K + (uint32_t)j;
        }
        keys[k] = key;
    }
    __syncthreads();
    // bitonic sort, ascending
    for (int32_t size = 2; size <= pw; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t k = tid; k < pw; k += kBwdBlock) {
                const int32_t p = k ^ stride;
                if (p > k) {
                    const uint32_t x = keys[k], y = keys[p];
                    const bool up = (k & size) == 0;
                    if ((x > y) == up) { keys[k] = y; keys[p] = x; }
                }
            }
            __syncthreads();
        }
    }
    // run starts -> compacted (cell, count) in cell order
    if (tid == 0) s_base = 0;
    __syncthreads();
    const int32_t lane = tid & 63, wv = tid >> 6;
    for (int32_t k0 = 0; k0 < pw; k0 += kBwdBlock) {
        const int32_t k = k0 + tid;
        const uint32_t key = k < pw ? keys[k] : kNone;
        const bool start = key != kNone && (k == 0 || keys[k - 1] != key);
        int32_t cnt = 0;
        if (start) {
            int32_t e = k + 1;
            while (e < pw && keys[e] == key) ++e;
            cnt = e - k;
        }
        // block-wide exclusive scan of the start flags
        const unsigned long long m = __ballot(start);
        const int32_t before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int32_t off = s_base;
        for (int32_t w = 0; w < wv; ++w) off += wsum[w];
        if (start) {
            const int64_t o = (int64_t)b * Tmax + off + before;
            ent_key[o] = key;
            ent_cnt[o] = cnt;
        }
        __syncthreads();
        if (tid == 0) {
            int32_t tot = 0;
            for (int32_t w = 0; w < kBwdBlock / 64; ++w) tot += wsum[w];
            s_base += tot;
        }
        __syncthreads();
    }
    if (tid == 0) n_ent[b] = s_base;
}

extern "C" __global__ __launch_bounds__(kBlock) void fv_bwd_zero_kernel(float* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0.0f;
}

extern "C" __global__ __launch_bounds__(kBwdBlock) void fv_bwd_fold_kernel(int32_t n, int32_t Tmax,
                                                                           const float* __restrict__ g,
                                                                           const uint32_t* __restrict__ ent_key,
                                                                           const int32_t* __restrict__ ent_cnt,
                                                                           const int32_t* __restrict__ n_ent,
                                                                           float* __restrict__ total) {
    for (int32_t b = 0; b < n; ++b) {
        const float gb = g[b];
        const int32_t ne = n_ent[b];
        const int64_t o = (int64_t)b * Tmax;
        for (int32_t u = threadIdx.x; u < ne; u += kBwdBlock) {
            const uint32_t c = ent_key[o + u];
            const float term = gb * (float)ent_cnt[o + u];
            total[c] = total[c] + term;
        }
        __syncthreads();
    }
}

extern "C" __global__ void fv_bwd_pi_kernel(int32_t K, int32_t n, int32_t Tmax, const int32_t* __restrict__ lengths,
                                            const int32_t* __restrict__ paths, const float* __restrict__ g,
                                            float* __restrict__ total) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int32_t b = 0; b < n; ++b) {
        if (clamp_len(lengths[b], Tmax) < 1) continue;
        const int32_t q = paths[(int64_t)b * Tmax];
        if (q >= 0 && q < K) total[q] = total[q] + g[b];
    }
}

extern "C" __global__ __launch_bounds__(kBlock) void fv_bwd_apply_kernel(const float* __restrict__ total,
                                                                         float* __restrict__ out, int64_t n,
                                                                         int32_t accumulate) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = accumulate ? out[i] + total[i] : total[i];
}

}  // namespace fv

using namespace fv;

namespace {

struct BwdLayout {
    size_t total_a = 0, total_pi = 0, key = 0, cnt = 0, nent = 0, bytes = 0;
};

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

fv_status plan_bwd(int32_t K, int32_t n, int32_t Tmax, BwdLayout& L) {
    if (K < 1 || K > 65535 || n < 0 || Tmax < 0)
        return fv_set_error(FV_E_INVALID_ARG, "fv_viterbi_backward: need 1 <= K <= 65535, n >= 0, Tmax >= 0");
    if (Tmax > kBwdMaxPairs + 1)
        return fv_set_error(FV_E_UNSUPPORTED, "fv_viterbi_backward: Tmax above 16385 is not supported");
    size_t cur = 0;
    L.total_a = cur; cur = up256(cur + (size_t)K * K * 4);
    L.total_pi = cur; cur = up256(cur + (size_t)K * 4);
    L.key = cur; cur = up256(cur + (size_t)n * Tmax * 4);
    L.cnt = cur; cur = up256(cur + (size_t)n * Tmax * 4);
    L.nent = cur; cur = up256(cur + (size_t)n * 4);
    L.bytes = cur;
    return FV_OK;
}

int32_t grid_for(int64_t items, int64_t per_block) {
    int64_t g = (items + per_block - 1) / per_block;
    return (int32_t)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace

extern "C" fv_status fv_backward_workspace_size(int32_t K, int32_t n_seqs, int32_t Tmax, size_t* bytes) {
    if (!bytes) return fv_set_error(FV_E_INVALID_ARG, "fv_backward_workspace_size: bytes is NULL");
    BwdLayout L;
    fv_status s = plan_bwd(K, n_seqs, Tmax, L);
    if (s != FV_OK) return s;
    *bytes = L.bytes;
    return FV_OK;
}

extern "C" fv_status fv_viterbi_backward(int32_t K, int32_t n, int32_t Tmax, const int32_t* lengths,
                                         const int32_t* paths, const float* grad_score, float* grad_log_b,
                                         float* grad_log_a, float* grad_log_pi, int32_t accumulate, void* ws,
                                         size_t ws_bytes, fv_stream_t stream) {
    BwdLayout L;
    fv_status s = plan_bwd(K, n, Tmax, L);
    if (s != FV_OK) return s;
    const bool any = n > 0 && Tmax > 0;
    if (any && (!lengths || !paths || !grad_score))
        return fv_set_error(FV_E_INVALID_ARG, "fv_viterbi_backward: lengths, paths and grad_score are required");
    if ((grad_log_a || grad_log_pi) && (!ws || ws_bytes < L.bytes))
        return fv_set_error(FV_E_WORKSPACE, "fv_viterbi_backward: workspace of %zu bytes needed", L.bytes);
    if (ws && (reinterpret_cast<uintptr_t>(ws) & 255))
        return fv_set_error(FV_E_INVALID_ARG, "fv_viterbi_backward: workspace must be 256-byte aligned");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);

    if (grad_log_b && any) {
        const int32_t vec4 = (K % 4 == 0) && (reinterpret_cast<uintptr_t>(grad_log_b) % 16 == 0);
        const int64_t rows = (int64_t)n * Tmax;
        hipLaunchKernelGGL(fv_bwd_fill_kernel, dim3(grid_for(rows, kBlock / 64)), dim3(kBlock), 0, st, K, n, Tmax,
                           lengths, paths, grad_score, grad_log_b, accumulate, vec4);
    }
    if (grad_log_a) {
        float* total = reinterpret_cast<float*>(w + L.total_a);
        const int64_t cells = (int64_t)K * K;
        hipLaunchKernelGGL(fv_bwd_zero_kernel, dim3(grid_for(cells, kBlock)), dim3(kBlock), 0, st, total, cells);
        if (any) {
            uint32_t* key = reinterpret_cast<uint32_t*>(w + L.key);
            int32_t* cnt = reinterpret_cast<int32_t*>(w + L.cnt);
            int32_t* nent = reinterpret_cast<int32_t*>(w + L.nent);
            hipLaunchKernelGGL(fv_bwd_dedup_kernel, dim3(n), dim3(kBwdBlock), 0, st, K, Tmax, lengths, paths, key,
                               cnt, nent);
            hipLaunchKernelGGL(fv_bwd_fold_kernel, dim3(1), dim3(kBwdBlock), 0, st, n, Tmax, grad_score, key, cnt,
                               nent, total);
        }
        hipLaunchKernelGGL(fv_bwd_apply_kernel, dim3(grid_for(cells, kBlock)), dim3(kBlock), 0, st, total,
                           grad_log_a, cells, accumulate);
    }
    if (grad_log_pi) {
        float* total = reinterpret_cast<float*>(w + L.total_pi);
        hipLaunchKernelGGL(fv_bwd_zero_kernel, dim3(1), dim3(kBlock), 0, st, total, (int64_t)K);
        if (any)
            hipLaunchKernelGGL(fv_bwd_pi_kernel, dim3(1), dim3(64), 0, st, K, n, Tmax, lengths, paths, grad_score,
                               total);
        hipLaunchKernelGGL(fv_bwd_apply_kernel, dim3(grid_for(K, kBlock)), dim3(kBlock), 0, st, total, grad_log_pi,
                           (int64_t)K, accumulate);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fv_set_error(FV_E_DEVICE, "fv_viterbi_backward: launch failed");
    return FV_OK;
}
