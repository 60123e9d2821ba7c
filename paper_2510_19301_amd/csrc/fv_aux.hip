// Auxiliary kernels: emission gather for discrete HMMs and path re-scoring.
#include "fv_internal.h"

namespace fv {

// log_b[t*ld + j] = log_e[j*V + obs[t]]  (the HMM's emission matrix indexed by
// the observed symbol, Sec. III).  A symbol outside [0, V) is an impossible
// observation: its row is -inf.  One block per time step.
extern "C" __global__ __launch_bounds__(kBlock) void fv_gather_kernel(int32_t K, int32_t V,
                                                                      const float* __restrict__ log_e,
                                                                      const int32_t* __restrict__ obs,
                                                                      float* __restrict__ log_b, int64_t ld) {
    const int32_t t = blockIdx.x;
    const int32_t x = obs[t];
    const bool ok = x >= 0 && x < V;
    for (int32_t j = threadIdx.x; j < K; j += kBlock)
        log_b[(int64_t)t * ld + j] = ok ? log_e[(int64_t)j * V + x] : -INFINITY;
}

// Step-by-step float32 re-sum of a given path (the decoded path's score):
// s_0 = log pi[q0] + log B_0[q0];  s_t = (s_{t-1} + log A[q_{t-1}][q_t]) + log B_t[q_t].
// One thread per sequence (the sum is sequential by definition).
extern "C" __global__ __launch_bounds__(kBlock) void fv_rescore_kernel(const float* __restrict__ log_a, int32_t K,
                                                                       const float* __restrict__ log_pi,
                                                                       const fv_seq* __restrict__ seqs,
                                                                       int32_t n, float* __restrict__ out) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= n) return;
    const fv_seq s = seqs[b];
    if (s.T <= 0) { out[b] = 0.0f; return; }
    int32_t q = s.path[0];
    if (q < 0 || q >= K) { out[b] = -INFINITY; return; }
    float v = log_pi ? log_pi[q] + s.log_b[q] : s.log_b[q];
    for (int32_t t = 1; t < s.T; ++t) {
        const int32_t q2 = s.path[t];
        if (q2 < 0 || q2 >= K) { v = -INFINITY; break; }
        const float c = v + log_a[(int64_t)q * K + q2];
        v = c + s.log_b[(int64_t)t * s.ld + q2];
        q = q2;
    }
    out[b] = v;
}

// ---- input validation (FV_FLAG_VALIDATE): every score must be finite or -inf

extern "C" __global__ __launch_bounds__(kBlock) void fv_fill_i32_kernel(int32_t* __restrict__ p, int64_t n,
                                                                        int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}

// NaN and +inf fail "x < +inf"; -inf and finite values pass.
__device__ __forceinline__ bool bad_score(float x) { return !(x < INFINITY); }

// *flag = 1 if any of p[0..n) is NaN or +inf (p may be null: nothing to check).
extern "C" __global__ __launch_bounds__(kBlock) void fv_validate_array_kernel(const float* __restrict__ p, int64_t n,
                                                                              int32_t* __restrict__ flag) {
    if (!p) return;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        bad |= bad_score(p[i]);
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1);
}

// bad_seq[b] = 1 if sequence b (of model `model`) has a NaN or +inf among its
// emission scores log_b[t*ld + j], t < T, j < K.  Blocks take sequences.
extern "C" __global__ __launch_bounds__(kBlock) void fv_validate_seqs_kernel(const fv_seq* __restrict__ seqs,
                                                                             int32_t n_seqs, int32_t model,
                                                                             int32_t K, int32_t* __restrict__ bad_seq) {
    for (int32_t b = blockIdx.x; b < n_seqs; b += gridDim.x) {
        const fv_seq d = seqs[b];
        if (d.model != model || d.T <= 0 || !d.log_b || d.ld < K) continue;
        bool bad = false;
        const int64_t n = (int64_t)d.T * K;
        for (int64_t i = threadIdx.x; i < n; i += kBlock) {
            const int64_t t = i / K, j = i - t * K;
            bad |= bad_score(d.log_b[t * d.ld + j]);
        }
        if (__syncthreads_or(bad) && threadIdx.x == 0) bad_seq[b] = 1;
    }
}

// Observation points of the Gaussian emission model must be finite.
__device__ __forceinline__ bool bad_point(double x) { return !__builtin_isfinite(x); }

// *flag = 1 if any of p[0..n) (float64 coordinates) is NaN or infinite.
extern "C" __global__ __launch_bounds__(kBlock) void fv_validate_points_kernel(const double* __restrict__ p, int64_t n,
                                                                               int32_t* __restrict__ flag) {
    if (!p) return;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        bad |= bad_point(p[i]);
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1);
}

// bad_seq[b] = 1 if sequence b (of model `model`) has a NaN or infinite
// coordinate among its observations (float64 [T][2] at its log_b field).
extern "C" __global__ __launch_bounds__(kBlock) void fv_validate_obs_kernel(const fv_seq* __restrict__ seqs,
                                                                            int32_t n_seqs, int32_t model,
                                                                            int32_t* __restrict__ bad_seq) {
    for (int32_t b = blockIdx.x; b < n_seqs; b += gridDim.x) {
        const fv_seq d = seqs[b];
        if (d.model != model || d.T <= 0 || !d.log_b) continue;
        const double* o = reinterpret_cast<const double*>(d.log_b);
        bool bad = false;
        for (int64_t i = threadIdx.x; i < 2 * (int64_t)d.T; i += kBlock) bad |= bad_point(o[i]);
        if (__syncthreads_or(bad) && threadIdx.x == 0) bad_seq[b] = 1;
    }
}

}  // namespace fv

using namespace fv;

extern "C" fv_status fv_gather_emissions(int32_t K, int32_t V, const float* log_e, const int32_t* obs,
                                         int32_t T, float* log_b, int64_t ld, fv_stream_t stream) {
    if (K < 1 || V < 1 || T < 0 || ld < K || (T > 0 && (!log_e || !obs || !log_b))) return FV_E_INVALID_ARG;
    if (T == 0) return FV_OK;
    hipLaunchKernelGGL(fv_gather_kernel, dim3(T), dim3(kBlock), 0, reinterpret_cast<hipStream_t>(stream), K, V,
                       log_e, obs, log_b, ld);
    return hipGetLastError() == hipSuccess ? FV_OK : FV_E_DEVICE;
}

extern "C" fv_status fv_rescore(const fv_trans* A, const float* log_pi, const fv_seq* seqs_dev, int32_t n_seqs,
                                float* score_out, fv_stream_t stream) {
    if (!A || A->kind != FV_DENSE || A->K < 1 || !A->log_a || n_seqs < 0 || (n_seqs > 0 && (!seqs_dev || !score_out)))
        return FV_E_INVALID_ARG;
    if (n_seqs == 0) return FV_OK;
    hipLaunchKernelGGL(fv_rescore_kernel, dim3((n_seqs + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), A->log_a, A->K, log_pi, seqs_dev, n_seqs, score_out);
    return hipGetLastError() == hipSuccess ? FV_OK : FV_E_DEVICE;
}
