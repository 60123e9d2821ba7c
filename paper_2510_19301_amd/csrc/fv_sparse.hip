// Sparse transition models: the in-edge transpose of a CSR model.
//
// The recurrence (Sec. III-A) maximises over the predecessors i of each
// destination j; with transitions given as CSR out-edges (a missing edge is
// log A = -inf) the predecessors of j are its in-edges.  Each decode builds
// them in the workspace, ordered within a destination by edge position in
// the CSR arrays, which is (source, position in the source's list) order:
// scanning them in order takes the lowest predecessor on ties, as the dense
// scan over i does.
//
// Steps: in-degrees (atomic counts), their prefix sum, an unordered scatter
// of edge ids, then each edge's rank among its destination's edges (a count
// of the smaller edge ids in the segment, so the result does not depend on
// the scatter order) gives its final place.  Malformed CSR arrays never
// cause an out-of-range access: edges whose destination lies outside
// [0, K) are dropped, sources come from a clamped search of row_ptr, and
// flag bits report what was wrong (kCsrInvalid, kCsrWideIn).
#include "fv_internal.h"

namespace fv {

extern "C" __global__ __launch_bounds__(kBlock) void fv_csr_zero_kernel(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0;
}

// row_ptr must start at 0, never decrease and end at nnz
extern "C" __global__ __launch_bounds__(kBlock) void fv_csr_check_kernel(int32_t K, int64_t nnz,
                                                                         const int32_t* __restrict__ row_ptr,
                                                                         int32_t* __restrict__ flag) {
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i <= K; i += gridDim.x * kBlock) {
        const int32_t v = row_ptr[i];
        bool bad = v < 0 || (int64_t)v > nnz;
        if (i == 0) bad |= v != 0;
        if (i == K) bad |= (int64_t)v != nnz;
        if (i < K) bad |= row_ptr[i + 1] < v;
        if (bad) atomicOr(flag, kCsrInvalid);
    }
}

// in-degree of every destination
extern "C" __global__ __launch_bounds__(kBlock) void fv_csr_count_kernel(int32_t K, int64_t nnz,
                                                                         const int32_t* __restrict__ col,
                                                                         int32_t* __restrict__ deg) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
        const int32_t j = col[e];
        if (j >= 0 && j < K) atomicAdd(&deg[j], 1);
    }
}

// in_ptr = exclusive prefix sum of deg, in_ptr[K] = the total (one block)
extern "C" __global__ __launch_bounds__(1024) void fv_csr_scan_kernel(int32_t K, const int32_t* __restrict__ deg,
                                                                     int32_t* __restrict__ in_ptr,
                                                                     int32_t* __restrict__ flag) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t s_carry;
    const int32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < K; base += 1024 * 8) {
        int32_t v[8], local = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t i = base + tid * 8 + k;
            v[k] = i < K ? deg[i] : 0;
            if (v[k] > kMaxInSlot + 1) atomicOr(flag, kCsrWideIn);
            local += v[k];
        }
        int32_t x = local;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        int32_t before = s_carry, all = 0;
        for (int u = 0; u < 16; ++u) {
            if (u < w) before += wsum[u];
            all += wsum[u];
        }
        before += x - local;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t i = base + tid * 8 + k;
            if (i < K) in_ptr[i] = before;
            before += v[k];
        }
        __syncthreads();
        if (tid == 0) s_carry += all;
        __syncthreads();
    }
    if (tid == 0) in_ptr[K] = s_carry;
}

// unordered placement of the edge ids into their destination's segment
extern "C" __global__ __launch_bounds__(kBlock) void fv_csr_scatter_kernel(int32_t K, int64_t nnz,
                                                                           const int32_t* __restrict__ col,
                                                                           const int32_t* __restrict__ in_ptr,
                                                                           int32_t* __restrict__ cursor,
                                                                           int32_t* __restrict__ eid) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
        const int32_t j = col[e];
        if (j < 0 || j >= K) continue;
        eid[in_ptr[j] + atomicAdd(&cursor[j], 1)] = (int32_t)e;
    }
}

// source of edge e: the i with row_ptr[i] <= e < row_ptr[i+1] (clamped to [0, K))
__device__ __forceinline__ int32_t edge_source(const int32_t* row_ptr, int32_t K, int32_t e) {
    int32_t lo = 0, hi = K + 1;   // first index with row_ptr > e
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (row_ptr[mid] <= e) lo = mid + 1; else hi = mid;
    }
    const int32_t i = lo - 1;
    return i < 0 ? 0 : (i >= K ? K - 1 : i);
}

// final order: an edge's rank among its segment's edge ids
extern "C" __global__ __launch_bounds__(kBlock) void fv_csr_place_kernel(int32_t K,
                                                                         const int32_t* __restrict__ row_ptr,
                                                                         const int32_t* __restrict__ col,
                                                                         const float* __restrict__ val,
                                                                         const int32_t* __restrict__ in_ptr,
                                                                         const int32_t* __restrict__ eid,
                                                                         int32_t* __restrict__ in_src,
                                                                         float* __restrict__ in_val) {
    const int32_t n_in = in_ptr[K];
    for (int32_t p = blockIdx.x * kBlock + threadIdx.x; p < n_in; p += gridDim.x * kBlock) {
        const int32_t e = eid[p];
        const int32_t j = col[e];
        const int32_t lo = in_ptr[j], hi = in_ptr[j + 1];
        int32_t rank = 0;
        for (int32_t q = lo; q < hi; ++q) rank += eid[q] < e;
        in_src[lo + rank] = edge_source(row_ptr, K, e);
        in_val[lo + rank] = val[e];
    }
}

}  // namespace fv
