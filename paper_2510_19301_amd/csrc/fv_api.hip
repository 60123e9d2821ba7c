// Host side of the C ABI: argument checks, workspace layout, launches.
#include <stdarg.h>
#include <stdio.h>
#include <float.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "fv_internal.h"

namespace fv {
extern "C" __global__ void fv_engine_kernel(const EngineArgs* __restrict__ table, int32_t n_models);
extern "C" __global__ void fv_small_vanilla32_kernel(const EngineArgs* __restrict__ table);
extern "C" __global__ void fv_small_vanilla64_kernel(const EngineArgs* __restrict__ table);
extern "C" __global__ void fv_small_vanilla128_kernel(const EngineArgs* __restrict__ table);
extern "C" __global__ void fv_small_vanilla256_kernel(const EngineArgs* __restrict__ table);
extern "C" __global__ void fv_small_flash32_kernel(const EngineArgs* __restrict__ table);
extern "C" __global__ void fv_small_flash64_kernel(const EngineArgs* __restrict__ table);
extern "C" __global__ void fv_small_flash128_kernel(const EngineArgs* __restrict__ table);
extern "C" __global__ void fv_small_flash256_kernel(const EngineArgs* __restrict__ table);
extern "C" __global__ void fv_fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v);
extern "C" __global__ void fv_validate_array_kernel(const float* __restrict__ p, int64_t n, int32_t* __restrict__ flag);
extern "C" __global__ void fv_validate_points_kernel(const double* __restrict__ p, int64_t n, int32_t* flag);
extern "C" __global__ void fv_validate_obs_kernel(const fv_seq* __restrict__ seqs, int32_t n_seqs, int32_t model,
                                                  int32_t* __restrict__ bad_seq);
extern "C" __global__ void fv_validate_seqs_kernel(const fv_seq* __restrict__ seqs, int32_t n_seqs, int32_t model,
                                                   int32_t K, int32_t* __restrict__ bad_seq);
extern "C" __global__ void fv_model_check_kernel(const fv_seq* seqs_dev, int32_t n_seqs, int32_t n_models,
                                                 int32_t* status);
extern "C" __global__ void fv_prep_dense_kernel(const float* __restrict__ log_a, int32_t K, int32_t Kp,
                                                float* __restrict__ Ap);
extern "C" __global__ void fv_transpose_dense_kernel(const float* __restrict__ Ap, int32_t Kp, float* __restrict__ At);
extern "C" __global__ void fv_setup_kernel(EngineArgs a, SetupArgs sa);
extern "C" __global__ void fv_finish_kernel(EngineArgs a, int32_t* status);
extern "C" __global__ void fv_beam_finish_kernel(EngineArgs a, const float* __restrict__ Ap, int32_t* status);
extern "C" __global__ void fv_csr_zero_kernel(int32_t* __restrict__ p, int64_t n);
extern "C" __global__ void fv_csr_check_kernel(int32_t K, int64_t nnz, const int32_t* __restrict__ row_ptr,
                                               int32_t* __restrict__ flag);
extern "C" __global__ void fv_csr_count_kernel(int32_t K, int64_t nnz, const int32_t* __restrict__ col,
                                               int32_t* __restrict__ deg);
extern "C" __global__ void fv_csr_scan_kernel(int32_t K, const int32_t* __restrict__ deg, int32_t* __restrict__ in_ptr,
                                              int32_t* __restrict__ flag);
extern "C" __global__ void fv_csr_scatter_kernel(int32_t K, int64_t nnz, const int32_t* __restrict__ col,
                                                 const int32_t* __restrict__ in_ptr, int32_t* __restrict__ cursor,
                                                 int32_t* __restrict__ eid);
extern "C" __global__ void fv_csr_place_kernel(int32_t K, const int32_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col, const float* __restrict__ val,
                                               const int32_t* __restrict__ in_ptr, const int32_t* __restrict__ eid,
                                               int32_t* __restrict__ in_src, float* __restrict__ in_val);
}  // namespace fv

using namespace fv;

static thread_local std::string g_last_error;
static thread_local bool g_prof_on = false;
static thread_local hipEvent_t g_prof_ev[2] = {nullptr, nullptr};
static thread_local bool g_prof_recorded = false;
// test hook (fv_debug_engine_limits): nonzero values replace the engine's
// step and barrier-wait limits for decodes issued by this host thread
static thread_local int64_t g_dbg_max_steps = 0;
static thread_local int64_t g_dbg_spin_limit = 0;
static thread_local unsigned long long* g_dbg_trace = nullptr;
static thread_local int32_t g_dbg_trace_steps = 0;

static fv_status fail(fv_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static fv_status fail(fv_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

fv_status fv_set_error(fv_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(FV_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

// Fixed device scratch of fv_decode_flash_noalloc: every GPU the library
// runs on holds one copy until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, once per
// device, and is kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[FV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kMaxDenseK = 65535;   // packed uint16 backpointers
constexpr int32_t kMaxSparseK = 1 << 30;
constexpr int64_t kMaxNnz = 0x7fffffffLL;
constexpr int32_t kMaxBlocks = 4096;    // engine grid size limit (arrival flags)
constexpr int kEngineBlock = 1024;      // engine threads per block (one block per CU)

struct Region {
    size_t off = 0, bytes = 0;
};

struct DenseLayout {
    int32_t method = 0, K = 0, Kp = 0, n_seqs = 0, n_slots = 0, pool = 0;
    int64_t sum_T = 0, sum_root = 0, sum_psi = 0, n_tasks = 0, slot_floats = 0;
    int32_t has_anc = 0;
    int32_t B = 0, Bc = 0;       // beam width and padded length (beam decodes)
    int32_t bw = 1;              // parts of a beam task's step
    int64_t brec = 0;            // floats per beam record
    int64_t q_cap = 0;
    int32_t sparse = 0;
    int64_t nnz = 0;
    int32_t leaves = 0;          // slots carry a leaf backpointer table
    int32_t wsplit = 0;          // FLASH subtasks split kWSplit ways (slots carry division copies)
    int64_t div_off = 0;         // their offset in a slot, in floats
    int32_t leaf_len = 0;        // the longest leaf that can occur (table rows per slot)
    int64_t leaf_off = 0;        // its offset in a slot, in floats
    int64_t leaf_tasks = 0;      // task-tree nodes when leaves end the bisection (slot sizing)
    Region Ap, At, seq1, seqinfo, keys, args, state, arrive, rows_full, rows_light, rows_beam, queue, free_stack,
        slots, alpha, root, psi, csr_flag, csr_ptr, csr_deg, csr_eid, csr_src, csr_val;
    size_t total = 0;
};

// Nodes of the bisection tree of a subtask with `pos` positions whose
// subtasks of at most leaf_len positions are leaves (children follow
// Alg. 1: [m, tmid] and, when the segment has more than 3 positions,
// [tmid + 1, n]).  Depends only on the length; memoised.
bool use_wide_rows(uint32_t flags, int32_t K, int32_t n_seqs, bool sparse);

int64_t leaf_tree_nodes(int32_t pos, int32_t leaf_len, std::map<int32_t, int64_t>& memo) {
    if (pos <= leaf_len) return 1;
    auto it = memo.find(pos);
    if (it != memo.end()) return it->second;
    const int32_t len = pos - 1;
    int64_t c = 1;
    if (len >= 2) c += leaf_tree_nodes(len / 2 + 1, leaf_len, memo);
    if (len > 2) c += leaf_tree_nodes(len - len / 2, leaf_len, memo);
    memo[pos] = c;
    return c;
}

size_t put(size_t& cur, Region& r, size_t bytes) {
    r.off = (cur + kAlign - 1) / kAlign * kAlign;
    r.bytes = bytes;
    cur = r.off + bytes;
    return r.off;
}

// Workspace layout of a dense decode.  Depends only on the arguments, so
// fv_workspace_size and the decode calls agree.  method FV_BEAM means a
// beam narrower than K (a beam of width >= K is planned as FV_FLASH).
fv_status plan_dense(int32_t method, const fv_trans* A, const int32_t* T_host, int32_t n_seqs, int32_t P, int32_t B,
                     bool single, DenseLayout& L) {
    L = DenseLayout{};
    L.method = method;
    const int32_t K = A->K;
    const bool sparse = A->kind == FV_CSR;
    L.sparse = sparse ? 1 : 0;
    L.nnz = sparse ? A->nnz : 0;
    const bool beam = method == FV_BEAM;
    if (beam && sparse) {
        // one block per task step: the beam states' out-edges are pushed
        if (B < 1 || B >= K) return fail(FV_E_INVALID_ARG, "beam width must be in [1, K)");
        if (B > kBeamMaxB) return fail(FV_E_UNSUPPORTED, "beam width %d exceeds %d", B, kBeamMaxB);
        L.B = B;
        L.Bc = (int32_t)round_up(B, 64);
        L.brec = 64 + 3 * (int64_t)L.Bc;
        L.bw = 1;
    } else if (beam) {
        if (K > kBeamMaxK) return fail(FV_E_UNSUPPORTED, "beam decoding supports K <= %d (got %d)", kBeamMaxK, K);
        if (B < 1 || B >= K) return fail(FV_E_INVALID_ARG, "beam width must be in [1, K)");
        if (B > kBeamMaxB) return fail(FV_E_UNSUPPORTED, "beam width %d exceeds %d", B, kBeamMaxB);
        L.B = B;
        L.Bc = (int32_t)round_up(B, 64);
        L.brec = 64 + 3 * (int64_t)L.Bc;
        // parts per step: at most 4096 destinations per part, at most 8192
        // candidates to merge; a batch that fills the device by itself keeps
        // one part per task, a small one spreads each task over up to 32
        // blocks (about 256 destinations per part)
        const int32_t Kp = (int32_t)round_up(K, kKAlign);
        int32_t W = n_seqs >= 64 ? 1 : std::min<int32_t>(32, std::min<int32_t>(Kp / 256, 8192 / B));
        W = std::max<int32_t>(W, (Kp + 4095) / 4096);
        W = std::max<int32_t>(1, std::min<int32_t>(W, K));
        if (W * B > 8192 || (K + W - 1) / W > 4096)
            return fail(FV_E_UNSUPPORTED, "beam width %d is too large for K=%d", B, K);
        L.bw = W;
    }
    L.K = K;
    L.Kp = (int32_t)round_up(K, kKAlign);
    L.n_seqs = n_seqs;
    int64_t nonempty = 0;
    for (int32_t b = 0; b < n_seqs; ++b) {
        const int32_t T = T_host[b];
        if (T < 0) return fail(FV_E_INVALID_ARG, "sequence %d has negative length %d", b, T);
        L.sum_T += T;
        if (T == 0) continue;
        ++nonempty;
        if (method == FV_VANILLA) {
            L.sum_psi += (int64_t)T * K;
            L.n_tasks += 1;
        } else {
            const int32_t pp = eff_parallelism(T, P);
            L.sum_root += (beam ? 1 : 2) * (int64_t)(pp - 1);
            L.n_tasks += T - pp + 1;
        }
    }
    L.has_anc = method != FV_VANILLA;
    // FLASH on a dense model of moderate K placed on local rows (the default
    // placement; wide rows run without leaves): leaf subtasks, their tables
    // sized to the longest leaf that can occur, the slot pool to the
    // leaf-cut tree
    L.leaves = method == FV_FLASH && !sparse && L.Kp <= kLeafMaxKp && !use_wide_rows(0, K, n_seqs, sparse);
    if (L.leaves) {
        std::map<int32_t, int64_t> memo;
        for (int32_t b = 0; b < n_seqs; ++b) {
            const int32_t T = T_host[b];
            if (T <= 1) continue;
            const int32_t pp = eff_parallelism(T, P);
            L.leaf_tasks += 1;
            for (int32_t d = 0; d < pp; ++d) {
                const int64_t m = d == 0 ? 0 : seg_end(T, pp, d - 1) + 1, n = seg_end(T, pp, d);
                if (n - m < 1) continue;
                const int32_t pos = (int32_t)(n - m + 1);
                L.leaf_len = std::max(L.leaf_len, std::min(pos, kLeafLen));
                L.leaf_tasks += leaf_tree_nodes(pos, kLeafLen, memo);
            }
        }
        if (L.leaf_len < 2) L.leaves = 0;
    }
    // dense rows: delta[2] (+ anc[2] + snapshot); beam rows: three beam
    // records, and room for a dense row should the task need its exact re-decode
    L.slot_floats = (int64_t)L.Kp * (method == FV_VANILLA ? 2 : 5);
    L.leaf_off = 5 * (int64_t)L.Kp;
    if (L.leaves) L.slot_floats += (int64_t)L.leaf_len * L.Kp / 2;
    // FLASH without leaf tables (dense above the leaf limit on wide rows, the
    // default placement there; sparse models): w-way subtasks, their
    // division copies (kWSplit - 1 delta rows and kWSplit - 2 link rows) in
    // each slot
    L.wsplit = (method == FV_FLASH &&
                (sparse || (L.Kp > kLeafMaxKp && use_wide_rows(0, K, n_seqs, sparse)))) ? kWSplit : 0;
    if (L.wsplit) {
        L.div_off = L.slot_floats;
        L.slot_floats += (int64_t)(2 * kWSplit - 3) * L.Kp;
    }
    if (beam) L.slot_floats = std::max<int64_t>(L.slot_floats, (2 * (int64_t)L.bw + 1) * L.brec);
    // a beam subtask may be queued twice (its exact re-decode)
    L.q_cap = std::max<int64_t>(1, beam ? 2 * L.n_tasks : L.n_tasks);
    const int64_t slot_bytes = L.slot_floats * 4;
    int64_t slots;
    if (method == FV_VANILLA) {
        slots = nonempty;
    } else {
        // rows in flight: every root at once, then as many subtasks as a
        // bounded budget of row buffers allows (parallelism vs memory)
        const int64_t budget = (int64_t)(L.leaves ? 512 : 128) << 20;
        const int64_t cap = std::max<int64_t>(256, std::min<int64_t>(4096, budget / slot_bytes));
        const int64_t tasks = L.leaves ? L.leaf_tasks : L.n_tasks;
        slots = std::min<int64_t>(tasks, std::max<int64_t>(std::min<int64_t>(nonempty, 1 << 16), cap));
        if (L.wsplit) {
            // w-way slots carry 2w - 3 division rows: keep the pool within
            // three quarters of the backpointer table a vanilla decode of the
            // same batch would hold (2 bytes per state and step), so that a
            // small batch at large K does not need more memory than vanilla
            const int64_t psi_bytes = L.sum_T * (int64_t)K * 2;
            slots = std::min<int64_t>(slots, std::max<int64_t>(2 * kXcd, (psi_bytes / 4 * 3) / slot_bytes));
        }
    }
    if (slots < 1) slots = 1;
    slots = round_up(slots, kXcd);  // equal slot pools, one per XCD
    if (slots > (1 << 26)) return fail(FV_E_UNSUPPORTED, "too many concurrent sequences");
    L.n_slots = (int32_t)slots;
    L.pool = L.n_slots / kXcd;
    if (L.pool > kMaxPool) return fail(FV_E_UNSUPPORTED, "too many rows in flight per XCD (%d)", L.pool);
    size_t cur = 0;
    put(cur, L.Ap, (!sparse && L.Kp != K) ? (size_t)L.Kp * L.Kp * 4 : 0);  // padded dense copy only when needed
    // transposed copy for the two-column items of moderate K
    put(cur, L.At, (!sparse && L.Kp <= kColMaxKp) ? (size_t)L.Kp * L.Kp * 4 : 0);
    put(cur, L.seq1, single ? sizeof(fv_seq) : 0);
    put(cur, L.seqinfo, (size_t)std::max(n_seqs, 1) * sizeof(SeqInfo));
    put(cur, L.keys, (size_t)std::max(n_seqs, 1) * 8);
    put(cur, L.args, sizeof(EngineArgs));
    put(cur, L.state, sizeof(EngineState));
    put(cur, L.arrive, (size_t)kMaxBlocks * 4);
    put(cur, L.rows_full, (size_t)2 * L.n_slots * sizeof(Row));
    put(cur, L.rows_light, (size_t)2 * L.n_slots * sizeof(Row));
    put(cur, L.rows_beam, (size_t)2 * L.n_slots * sizeof(Row));   // block rows: beam tasks and finalizes
    put(cur, L.queue, (size_t)L.q_cap * sizeof(Task));
    put(cur, L.free_stack, (size_t)L.n_slots * 4);
    put(cur, L.slots, (size_t)L.n_slots * slot_bytes);
    put(cur, L.alpha, method != FV_VANILLA ? (size_t)L.sum_T * 4 : 0);
    put(cur, L.root, (size_t)L.sum_root * (beam ? L.brec : L.Kp) * 4);
    put(cur, L.psi, (size_t)L.sum_psi * 2);
    // sparse models: the in-edge transpose (pointers, sources, scores) and its scratch
    const size_t nn = sparse ? (size_t)std::max<int64_t>(L.nnz, 1) : 0;
    put(cur, L.csr_flag, sparse ? 4 : 0);
    put(cur, L.csr_ptr, sparse ? ((size_t)K + 1) * 4 : 0);
    put(cur, L.csr_deg, sparse ? (size_t)K * 4 : 0);
    put(cur, L.csr_eid, nn * 4);
    put(cur, L.csr_src, nn * 4);
    put(cur, L.csr_val, nn * 4);
    L.total = (cur + kAlign - 1) / kAlign * kAlign;
    return FV_OK;
}

fv_status check_model(const fv_trans* A) {
    if (!A) return fail(FV_E_INVALID_ARG, "null transition model");
    if (A->K < 1) return fail(FV_E_INVALID_ARG, "K must be >= 1 (got %d)", A->K);
    if (A->kind == FV_DENSE) {
        if (A->K > kMaxDenseK) return fail(FV_E_UNSUPPORTED, "K=%d exceeds %d", A->K, kMaxDenseK);
        if (!A->log_a) return fail(FV_E_INVALID_ARG, "null log_a");
        return FV_OK;
    }
    if (A->kind != FV_CSR) return fail(FV_E_INVALID_ARG, "unknown transition model kind %d", A->kind);
    if (A->K > kMaxSparseK) return fail(FV_E_UNSUPPORTED, "K=%d exceeds %d", A->K, kMaxSparseK);
    if (A->nnz < 0) return fail(FV_E_INVALID_ARG, "nnz < 0");
    if (A->nnz > kMaxNnz) return fail(FV_E_UNSUPPORTED, "nnz=%lld exceeds %lld", (long long)A->nnz, (long long)kMaxNnz);
    if (!A->row_ptr || (A->nnz > 0 && (!A->col || !A->val))) return fail(FV_E_INVALID_ARG, "null CSR array");
    return FV_OK;
}

unsigned grid_for(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 8192));
}

// In-edge transpose of a CSR model into the workspace (see fv_sparse.hip).
void launch_transpose(const fv_trans* A, const DenseLayout& L, char* w, hipStream_t stream) {
    auto at = [&](const Region& r) { return reinterpret_cast<int32_t*>(w + r.off); };
    const int32_t K = A->K;
    const int64_t nnz = A->nnz;
    int32_t* flag = at(L.csr_flag);
    int32_t* deg = at(L.csr_deg);
    int32_t* in_ptr = at(L.csr_ptr);
    hipLaunchKernelGGL(fv_csr_zero_kernel, dim3(1), dim3(kBlock), 0, stream, flag, (int64_t)1);
    hipLaunchKernelGGL(fv_csr_zero_kernel, dim3(grid_for(K)), dim3(kBlock), 0, stream, deg, (int64_t)K);
    hipLaunchKernelGGL(fv_csr_check_kernel, dim3(grid_for((int64_t)K + 1)), dim3(kBlock), 0, stream, K, nnz,
                       A->row_ptr, flag);
    hipLaunchKernelGGL(fv_csr_count_kernel, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, K, nnz, A->col, deg);
    hipLaunchKernelGGL(fv_csr_scan_kernel, dim3(1), dim3(1024), 0, stream, K, deg, in_ptr, flag);
    hipLaunchKernelGGL(fv_csr_zero_kernel, dim3(grid_for(K)), dim3(kBlock), 0, stream, deg, (int64_t)K);
    hipLaunchKernelGGL(fv_csr_scatter_kernel, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, K, nnz, A->col,
                       in_ptr, deg, at(L.csr_eid));
    hipLaunchKernelGGL(fv_csr_place_kernel, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, K, A->row_ptr, A->col,
                       A->val, in_ptr, at(L.csr_eid), at(L.csr_src), reinterpret_cast<float*>(at(L.csr_val)));
}

struct DeviceInfo {
    int cus = 0;
    int engine_blocks_per_cu = 0;
};

// Queried once per device and cached: a decode call then does no property
// or occupancy query between the caller's events and its launches.
constexpr int kMaxDevices = 64;
std::mutex g_dev_mutex;
DeviceInfo g_dev_info[kMaxDevices];
bool g_dev_known[kMaxDevices] = {};

void* g_scratch_ptr[kMaxDevices] = {};

fv_status scratch_address(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FV_E_DEVICE, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FV_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FV_OK;
}

fv_status device_info(DeviceInfo& di) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FV_E_DEVICE, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    if (!g_dev_known[dev]) {
        hipDeviceProp_t p;
        HIP_TRY(hipGetDeviceProperties(&p, dev));
        DeviceInfo d;
        d.cus = p.multiProcessorCount;
        int nb = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fv_engine_kernel),
                                                             kEngineBlock, 0));
        d.engine_blocks_per_cu = nb;
        if (nb < 1) return fail(FV_E_DEVICE, "engine kernel cannot be resident");
        g_dev_info[dev] = d;
        g_dev_known[dev] = true;
    }
    di = g_dev_info[dev];
    return FV_OK;
}

__global__ void write_seq_kernel(fv_seq* dst, fv_seq v) { *dst = v; }

// Row placement (see FV_FLAG_WIDE_ROWS): wide rows when log A cannot be
// shared through L2 (large K) or when too few rows exist to fill lane tiles.
bool use_wide_rows(uint32_t flags, int32_t K, int32_t n_seqs, bool sparse) {
    if (sparse) return false;
    if (flags & FV_FLAG_WIDE_ROWS) return true;
    if (flags & FV_FLAG_LOCAL_ROWS) return false;
    return K >= 4096 || (K >= 1024 && n_seqs <= 4);
}

// FLASH parallelism when the caller passes P <= 0.  The engine's time is
// about (number of global steps) x (fixed cost per step) + work / rate:
// a larger P shortens the subtask trees (fewer steps after the root pass,
// less recomputation), and costs (P'-1) division copies of 2K values per
// sequence.  The choice keeps those copies at most a quarter of what a
// vanilla backpointer table would need (2 bytes per state and step), i.e.
// P' <= T/16 for the median length, as a power of two in [2, 512].
int32_t auto_parallelism(const int32_t* T_host, int32_t n_seqs) {
    std::vector<int32_t> t;
    for (int32_t b = 0; b < n_seqs; ++b)
        if (T_host[b] > 0) t.push_back(T_host[b]);
    if (t.empty()) return 2;
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    const int32_t med = t[t.size() / 2];
    int32_t P = 2;
    while (P < 512 && 2 * P * 16 <= med) P *= 2;
    return P;
}

// Beam widths of at least K keep every state: that is FLASH decoding.
int32_t effective_method(int32_t method, const fv_trans* A, int32_t B) {
    return (method == FV_BEAM && A && B >= A->K) ? FV_FLASH : method;
}

// Workspace of a batch: the engine's table of per-model argument blocks,
// then one region per model that has sequences (its own plan).
struct BatchPlan {
    Region table;
    Region valid;                   // validation flags: [n_seqs] per sequence, then one per planned decode
    std::vector<int32_t> model;     // model index of each planned decode
    std::vector<int32_t> method;    // its effective method
    std::vector<DenseLayout> L;
    std::vector<size_t> base;       // byte offset of its region
    size_t total = 0;
};

fv_status plan_batch(int32_t method, const fv_trans* models, int32_t n_models, const int32_t* T_host,
                     const int32_t* model_host, int32_t n_seqs, int32_t P, int32_t B, bool single, BatchPlan& bp) {
    bp = BatchPlan{};
    if (!models || n_models < 1) return fail(FV_E_INVALID_ARG, "need at least one transition model");
    if (n_models > 1 && n_seqs > 0 && !model_host)
        return fail(FV_E_INVALID_ARG, "model_host is required when n_models > 1");
    for (int32_t m = 0; m < n_models; ++m) {
        fv_status rc = check_model(&models[m]);
        if (rc != FV_OK) return fail(rc, "model %d: %s", m, g_last_error.c_str());
    }
    std::vector<std::vector<int32_t>> lens(n_models);
    for (int32_t b = 0; b < n_seqs; ++b) {
        const int32_t mi = model_host ? model_host[b] : 0;
        if (mi < 0 || mi >= n_models) return fail(FV_E_INVALID_ARG, "sequence %d has model %d", b, mi);
        lens[mi].push_back(T_host[b]);
    }
    int32_t n_plans = 0;
    for (int32_t m = 0; m < n_models; ++m) n_plans += !lens[m].empty();
    size_t cur = 0;
    put(cur, bp.table, (size_t)std::max(n_plans, 1) * sizeof(EngineArgs));
    put(cur, bp.valid, ((size_t)std::max(n_seqs, 0) + std::max(n_plans, 1)) * 4);
    for (int32_t m = 0; m < n_models; ++m) {
        if (lens[m].empty()) continue;
        const int32_t eff = effective_method(method, &models[m], B);
        DenseLayout L;
        fv_status rc = plan_dense(eff, &models[m], lens[m].data(), (int32_t)lens[m].size(), P, B, single, L);
        if (rc != FV_OK) return n_models > 1 ? fail(rc, "model %d: %s", m, g_last_error.c_str()) : rc;
        const size_t base = (cur + kAlign - 1) / kAlign * kAlign;
        bp.model.push_back(m);
        bp.method.push_back(eff);
        bp.L.push_back(L);
        bp.base.push_back(base);
        cur = base + L.total;
    }
    bp.total = (cur + kAlign - 1) / kAlign * kAlign;
    return FV_OK;
}

fv_status check_flags(uint32_t flags, int32_t method, const fv_trans* models, int32_t n_models) {
    if ((flags & FV_FLAG_WIDE_ROWS) && (flags & FV_FLAG_LOCAL_ROWS))
        return fail(FV_E_INVALID_ARG, "FV_FLAG_WIDE_ROWS and FV_FLAG_LOCAL_ROWS exclude each other");
    if (flags & ~(uint32_t)(FV_FLAG_WIDE_ROWS | FV_FLAG_LOCAL_ROWS | FV_FLAG_VALIDATE | FV_FLAG_NO_LEAVES |
                            FV_FLAG_RELATIVE_INIT | FV_FLAG_STEP_ITEMS | FV_FLAG_STEP_TILES | FV_FLAG_ENGINE))
        return fail(FV_E_INVALID_ARG, "unknown flags 0x%x", flags);
    if ((flags & FV_FLAG_STEP_ITEMS) && (flags & FV_FLAG_STEP_TILES))
        return fail(FV_E_INVALID_ARG, "FV_FLAG_STEP_ITEMS and FV_FLAG_STEP_TILES exclude each other");
    if ((flags & FV_FLAG_RELATIVE_INIT) && method != FV_VANILLA)
        for (int32_t m = 0; models && m < n_models; ++m)
            if (models[m].kind == FV_CSR)
                return fail(FV_E_UNSUPPORTED, "FV_FLAG_RELATIVE_INIT applies to dense models only");
    if (flags & FV_FLAG_WIDE_ROWS)
        for (int32_t m = 0; models && m < n_models; ++m)
            if (models[m].kind == FV_CSR) return fail(FV_E_INVALID_ARG, "FV_FLAG_WIDE_ROWS applies to dense models only");
    return FV_OK;
}

// Decodes every sequence of seqs_dev (or the one sequence `single`) with
// its model: per model, the preparation kernels and the setup kernel, then
// one persistent engine launch for all models, then the finish kernels.
// Emission descriptors (NULL: tables for every model).
fv_status check_emissions(const fv_emission* emits, const fv_trans* models, int32_t n_models) {
    for (int32_t m = 0; emits && models && m < n_models; ++m) {
        const fv_emission& e = emits[m];
        if (e.kind == FV_EMIT_TABLE) continue;
        if (e.kind != FV_EMIT_GAUSS2D) return fail(FV_E_INVALID_ARG, "model %d: unknown emission kind %d", m, e.kind);
        if (models[m].kind != FV_CSR)
            return fail(FV_E_UNSUPPORTED, "model %d: generated emissions apply to CSR models only", m);
        if (!e.state_xy) return fail(FV_E_INVALID_ARG, "model %d: null state points", m);
        if (!std::isfinite(e.c2) || e.c2 > 0.0 || !std::isfinite(e.c0) || e.c0 < -(double)FLT_MAX)
            return fail(FV_E_INVALID_ARG, "model %d: emission coefficients need finite c2 <= 0 and finite c0 >= -FLT_MAX",
                        m);
    }
    return FV_OK;
}

fv_status run_batch(int32_t method, const fv_trans* models, const float* const* log_pi, int32_t n_models,
                    const fv_seq* seqs_dev, const int32_t* T_host, const int32_t* model_host, int32_t n_seqs,
                    int32_t P, int32_t B, const fv_seq* single, int32_t* status, uint32_t flags, void* ws,
                    size_t ws_bytes, hipStream_t stream, const fv_emission* emits = nullptr) {
    fv_status rc = check_flags(flags, method, models, n_models);
    if (rc != FV_OK) return rc;
    rc = check_emissions(emits, models, n_models);
    if (rc != FV_OK) return rc;
    BatchPlan bp;
    rc = plan_batch(method, models, n_models, T_host, model_host, n_seqs, P, B, single != nullptr, bp);
    if (rc != FV_OK) return rc;
    if (!ws || ws_bytes < bp.total)
        return fail(FV_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required", ws_bytes, bp.total);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return fail(FV_E_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
    if (bp.L.empty()) return FV_OK;   // no sequences
    DeviceInfo di;
    rc = device_info(di);
    if (rc != FV_OK) return rc;
    const int32_t n_compute = std::min(di.cus, kMaxBlocks) - 1;
    if (n_compute < kXcd) return fail(FV_E_UNSUPPORTED, "device has too few compute units");

    char* const w0 = static_cast<char*>(ws);
    EngineArgs* table = reinterpret_cast<EngineArgs*>(w0 + bp.table.off);
    const bool validate = (flags & FV_FLAG_VALIDATE) != 0;
    const int32_t n_desc = single ? 1 : n_seqs;   // descriptors the sequence flags index
    int32_t* bad_seq = reinterpret_cast<int32_t*>(w0 + bp.valid.off);
    int32_t* bad_model = bad_seq + n_desc;
    if (validate) {
        const int64_t n_flags = (int64_t)n_desc + (int64_t)bp.L.size();
        hipLaunchKernelGGL(fv_fill_i32_kernel, dim3(grid_for(n_flags)), dim3(kBlock), 0, stream, bad_seq, n_flags, 0);
    }
    std::vector<EngineArgs> args(bp.L.size());
    std::vector<const float*> aps(bp.L.size());
    for (size_t p = 0; p < bp.L.size(); ++p) {
        const DenseLayout& L = bp.L[p];
        const fv_trans* A = &models[bp.model[p]];
        const fv_emission emit = emits ? emits[bp.model[p]] : fv_emission{FV_EMIT_TABLE, nullptr, 0.0, 0.0};
        const int32_t meth = bp.method[p];
        const int32_t n_local = L.n_seqs;
        const bool sparse = A->kind == FV_CSR;
        char* w = w0 + bp.base[p];
        auto at = [&](const Region& r) { return static_cast<void*>(w + r.off); };
        const fv_seq* sd = seqs_dev;
        if (single) {
            hipLaunchKernelGGL(write_seq_kernel, dim3(1), dim3(1), 0, stream, static_cast<fv_seq*>(at(L.seq1)), *single);
            sd = static_cast<const fv_seq*>(at(L.seq1));
        }
        const float* Ap = sparse ? nullptr : A->log_a;
        if (sparse) launch_transpose(A, L, w, stream);
        if (!sparse && L.Kp != A->K) {
            float* pad = static_cast<float*>(at(L.Ap));
            const int64_t cells = (int64_t)L.Kp * L.Kp;
            hipLaunchKernelGGL(fv_prep_dense_kernel, dim3((unsigned)((cells + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                               stream, A->log_a, A->K, L.Kp, pad);
            Ap = pad;
        }
        aps[p] = Ap;
        const bool wide = use_wide_rows(flags, A->K, n_local, sparse);
        float* At = nullptr;
        if (L.At.bytes && !wide) {   // wide rows never use it
            At = static_cast<float*>(at(L.At));
            hipLaunchKernelGGL(fv_transpose_dense_kernel, dim3(L.Kp / 64, L.Kp / 64), dim3(kBlock), 0, stream, Ap,
                               L.Kp, At);
        }
        if (validate) {
            const int64_t kk = (int64_t)A->K;
            if (sparse) {
                if (A->nnz > 0)
                    hipLaunchKernelGGL(fv_validate_array_kernel, dim3(grid_for(A->nnz)), dim3(kBlock), 0, stream,
                                       A->val, A->nnz, bad_model + p);
            } else {
                hipLaunchKernelGGL(fv_validate_array_kernel, dim3(grid_for(kk * kk)), dim3(kBlock), 0, stream,
                                   A->log_a, kk * kk, bad_model + p);
            }
            const float* pi = log_pi ? log_pi[bp.model[p]] : nullptr;
            if (pi)
                hipLaunchKernelGGL(fv_validate_array_kernel, dim3(grid_for(kk)), dim3(kBlock), 0, stream, pi, kk,
                                   bad_model + p);
            if (emit.kind == FV_EMIT_GAUSS2D) {
                hipLaunchKernelGGL(fv_validate_points_kernel, dim3(grid_for(2 * kk)), dim3(kBlock), 0, stream,
                                   emit.state_xy, 2 * kk, bad_model + p);
                hipLaunchKernelGGL(fv_validate_obs_kernel, dim3((unsigned)std::min(n_desc, 4096)), dim3(kBlock), 0,
                                   stream, sd, n_desc, single ? 0 : bp.model[p], bad_seq);
            } else {
                hipLaunchKernelGGL(fv_validate_seqs_kernel, dim3((unsigned)std::min(n_desc, 4096)), dim3(kBlock), 0,
                                   stream, sd, n_desc, single ? 0 : bp.model[p], A->K, bad_seq);
            }
        }
        EngineArgs& a = args[p];
        a = EngineArgs{};
        a.K = A->K;
        a.Kp = L.Kp;
        a.log_pi = log_pi ? log_pi[bp.model[p]] : nullptr;
        a.Acol = Ap;
        a.At = At;
        a.seqs = static_cast<SeqInfo*>(at(L.seqinfo));
        a.n_seqs = n_local;
        a.method = meth;
        a.slot_base = static_cast<float*>(at(L.slots));
        a.slot_floats = L.slot_floats;
        a.n_slots = L.n_slots;
        a.has_anc = L.has_anc;
        a.wide = wide ? 1 : 0;
        a.slab = (!wide && !sparse && At && A->K == L.Kp && (L.Kp == 512 || L.Kp == 1024) &&
                  !(flags & (FV_FLAG_STEP_ITEMS | FV_FLAG_STEP_TILES))) ? 1 : 0;
        a.force_tiles = (flags & FV_FLAG_STEP_TILES) ? 1 : 0;
        // leaves are exact only with anchored starts: the paper's displayed
        // start restarts every bisection level, and so does the decode
        a.leaf_len = (L.leaves && !a.wide && !(flags & (FV_FLAG_NO_LEAVES | FV_FLAG_RELATIVE_INIT))) ? L.leaf_len
                                                                                                      : 0;
        a.relative_init = (flags & FV_FLAG_RELATIVE_INIT) ? 1 : 0;
        // w-way subtasks on wide rows and sparse rows; the paper's bisection under
        // FV_FLAG_NO_LEAVES, and under the relative start (whose result
        // depends on the schedule)
        a.wsplit = (L.wsplit && (wide || sparse) && !(flags & (FV_FLAG_NO_LEAVES | FV_FLAG_RELATIVE_INIT))) ? L.wsplit
                                                                                                           : 0;
        a.div_off = L.div_off;
        a.beam_q = (meth == FV_BEAM && !sparse && L.bw == 1 && L.Kp <= 2048 && L.B <= 256) ? 1 : 0;
        a.leaf_off = L.leaf_off;
        if (sparse) {
            a.sparse = 1;
            a.nnz = A->nnz;
            a.row_ptr = A->row_ptr;
            a.col = A->col;
            a.val = A->val;
            a.in_ptr = static_cast<const int32_t*>(at(L.csr_ptr));
            a.in_src = static_cast<const int32_t*>(at(L.csr_src));
            a.in_val = static_cast<const float*>(at(L.csr_val));
            a.csr_flag = static_cast<int32_t*>(at(L.csr_flag));
        }
        a.emit_kind = emit.kind;
        a.emit_xy = emit.state_xy;
        a.emit_c2 = emit.c2;
        a.emit_c0 = emit.c0;
        a.alpha_at = static_cast<float*>(at(L.alpha));
        a.root_copy = static_cast<float*>(at(L.root));
        a.psi16 = static_cast<uint16_t*>(at(L.psi));
        a.keys = static_cast<unsigned long long*>(at(L.keys));
        a.st = static_cast<EngineState*>(at(L.state));
        a.arrive = static_cast<uint32_t*>(at(L.arrive));
        a.rows_full = static_cast<Row*>(at(L.rows_full));
        a.rows_light = static_cast<Row*>(at(L.rows_light));
        a.rows_beam = static_cast<Row*>(at(L.rows_beam));
        a.B = L.B;
        a.Bc = L.Bc;
        a.brec = L.brec;
        a.bw = L.bw;
        a.bw_min = std::min<int32_t>(L.bw, std::max<int32_t>(1, (L.Kp + 4095) / 4096));
        a.pool = L.pool;
        a.queue = static_cast<Task*>(at(L.queue));
        a.q_cap = L.q_cap;
        a.free_stack = static_cast<int32_t*>(at(L.free_stack));
        // one engine block per CU: block 0 schedules, the others compute
        a.n_compute_blocks = n_compute;
        a.spin_limit = g_dbg_spin_limit ? g_dbg_spin_limit : (int64_t)1 << 24;
        // beam: exact re-decodes add at most one pass per subtask
        a.max_steps = g_dbg_max_steps ? g_dbg_max_steps : (meth == FV_BEAM ? 16 : 8) * (L.sum_T + L.n_tasks) + 4096;
        if (validate) {
            a.bad_seq = bad_seq;
            a.bad_model = bad_model + p;
        }
        if (g_dbg_trace && p == 0) {   // the first model's steps only
            a.trace = g_dbg_trace;
            a.trace_steps = g_dbg_trace_steps;
        }

        SetupArgs sa{};
        sa.seqs_dev = sd;
        sa.n_seqs = single ? 1 : n_seqs;
        sa.P = P;
        sa.host_sum_T = L.sum_T;
        sa.host_sum_root = L.sum_root;
        sa.host_sum_psi = L.sum_psi;
        sa.kind = meth == FV_VANILLA ? KIND_VANILLA : (meth == FV_BEAM ? KIND_BROOT : KIND_ROOT);
        sa.K = A->K;
        sa.model = single ? 0 : bp.model[p];
        sa.n_local = n_local;
        sa.emit_kind = emit.kind;
        sa.args_out = table + p;
        hipLaunchKernelGGL(fv_setup_kernel, dim3(1), dim3(kBlock), 0, stream, a, sa);
    }
    if (status && !single && n_models > 1)
        hipLaunchKernelGGL(fv_model_check_kernel, dim3((n_seqs + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                           seqs_dev, n_seqs, n_models, status);

    const EngineArgs* table_dev = table;
    int32_t n_tab = (int32_t)bp.L.size();
    void* kargs[] = {&table_dev, &n_tab};
    if (g_prof_on) HIP_TRY(hipEventRecord(g_prof_ev[0], stream));
    // vanilla or FLASH decodes whose models are all small and dense: one wave per sequence, one
    // launch per model, no persistent engine
    bool small = !(flags & FV_FLAG_ENGINE);
    for (size_t p = 0; p < bp.L.size(); ++p) {
        const int32_t Kp_ = bp.L[p].K;
        small = small && models[bp.model[p]].kind == FV_DENSE &&
                ((bp.method[p] == FV_VANILLA && Kp_ <= kSmallK) || (bp.method[p] == FV_FLASH && Kp_ <= kSmallFlashK));
    }
    if (small) {
        for (size_t p = 0; p < bp.L.size(); ++p) {
            const int32_t Ks = bp.L[p].K;
            const dim3 grid(std::max(1, bp.L[p].n_seqs));
            const dim3 block(Ks <= 64 ? 64 : (Ks <= 128 ? 128 : 256));
            if (bp.method[p] == FV_VANILLA)
                hipLaunchKernelGGL(Ks <= 32 ? fv_small_vanilla32_kernel
                                            : (Ks <= 64 ? fv_small_vanilla64_kernel
                                                        : (Ks <= 128 ? fv_small_vanilla128_kernel
                                                                     : fv_small_vanilla256_kernel)),
                                   grid, block, 0, stream, table_dev + p);
            else
                hipLaunchKernelGGL(Ks <= 32 ? fv_small_flash32_kernel
                                            : (Ks <= 64 ? fv_small_flash64_kernel
                                                        : (Ks <= 128 ? fv_small_flash128_kernel
                                                                     : fv_small_flash256_kernel)),
                                   grid, block, 0, stream, table_dev + p);
        }
    }
    else
        HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(fv_engine_kernel), dim3(n_compute + 1),
                                           dim3(kEngineBlock), kargs, 0, stream));
    if (g_prof_on) {
        HIP_TRY(hipEventRecord(g_prof_ev[1], stream));
        g_prof_recorded = true;
    }
    for (size_t p = 0; p < bp.L.size(); ++p) {
        const int32_t n_local = bp.L[p].n_seqs;
        if (bp.method[p] == FV_BEAM)
            hipLaunchKernelGGL(fv_beam_finish_kernel, dim3((n_local + kWaves - 1) / kWaves), dim3(kBlock), 0, stream,
                               args[p], aps[p], status);
        else
        {
            args[p].path_done = small ? 1 : 0;   // the one-wave vanilla kernel walks its own table
            hipLaunchKernelGGL(fv_finish_kernel, dim3((n_local + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                               args[p], status);
        }
    }
    HIP_TRY(hipGetLastError());
    return FV_OK;
}

}  // namespace

extern "C" {

int32_t fv_abi_version(void) { return 1; }

const char* fv_last_error(void) { return g_last_error.c_str(); }

const char* fv_status_str(fv_status s) {
    switch (s) {
        case FV_OK: return "FV_OK";
        case FV_E_INVALID_ARG: return "FV_E_INVALID_ARG: invalid argument";
        case FV_E_UNSUPPORTED: return "FV_E_UNSUPPORTED: size or model kind beyond the library's limits";
        case FV_E_WORKSPACE: return "FV_E_WORKSPACE: workspace too small";
        case FV_E_DEVICE: return "FV_E_DEVICE: HIP launch/runtime failure or engine watchdog";
        case FV_E_INFEASIBLE: return "FV_E_INFEASIBLE: best score is -inf";
        case FV_W_BEAM_FALLBACK: return "FV_W_BEAM_FALLBACK: a beam subtask was re-decoded exactly";
    }
    return "unknown fv_status";
}

fv_status fv_profile_engine(int32_t enable) {
    if (enable && !g_prof_ev[0]) {
        HIP_TRY(hipEventCreate(&g_prof_ev[0]));
        HIP_TRY(hipEventCreate(&g_prof_ev[1]));
    }
    if (!enable && g_prof_ev[0]) {
        // the events are released here, not left to process teardown: wait
        // for the last recorded pair, then destroy both
        hipError_t e0 = hipEventSynchronize(g_prof_ev[1]);
        hipError_t e1 = hipEventDestroy(g_prof_ev[0]);
        hipError_t e2 = hipEventDestroy(g_prof_ev[1]);
        g_prof_ev[0] = g_prof_ev[1] = nullptr;
        g_prof_on = false;
        g_prof_recorded = false;
        for (hipError_t e : {e0, e1, e2})
            if (e != hipSuccess) return fail(FV_E_DEVICE, "profiling events: %s", hipGetErrorString(e));
        return FV_OK;
    }
    g_prof_on = enable != 0;
    g_prof_recorded = false;
    return FV_OK;
}

fv_status fv_debug_engine_trace(unsigned long long* trace, int32_t steps) {
    if (steps < 0 || (steps > 0 && !trace)) return fail(FV_E_INVALID_ARG, "bad trace buffer");
    g_dbg_trace = steps > 0 ? trace : nullptr;
    g_dbg_trace_steps = steps;
    return FV_OK;
}

fv_status fv_debug_engine_limits(int64_t max_steps, int64_t spin_limit) {
    if (max_steps < 0 || spin_limit < 0) return fail(FV_E_INVALID_ARG, "limits must be >= 0");
    g_dbg_max_steps = max_steps;
    g_dbg_spin_limit = spin_limit;
    return FV_OK;
}

fv_status fv_profile_engine_ms(float* ms) {
    if (!ms) return fail(FV_E_INVALID_ARG, "null ms");
    if (!g_prof_recorded) return fail(FV_E_INVALID_ARG, "no engine launch recorded since profiling was enabled");
    HIP_TRY(hipEventSynchronize(g_prof_ev[1]));
    HIP_TRY(hipEventElapsedTime(ms, g_prof_ev[0], g_prof_ev[1]));
    return FV_OK;
}


fv_status fv_workspace_size(int32_t method, const fv_trans* models, int32_t n_models,
                            const int32_t* T_host, const int32_t* model_host, int32_t n_seqs,
                            int32_t P, int32_t B, size_t* bytes) {
    if (!bytes) return fail(FV_E_INVALID_ARG, "null bytes");
    if (n_seqs < 0 || (n_seqs > 0 && !T_host)) return fail(FV_E_INVALID_ARG, "bad sequence list");
    if (method != FV_VANILLA && method != FV_FLASH && method != FV_BEAM)
        return fail(FV_E_INVALID_ARG, "unknown method %d", method);
    if (method == FV_BEAM && (B < 1 || P < 1)) return fail(FV_E_INVALID_ARG, "beam decoding needs B >= 1 and P >= 1");
    if (method == FV_FLASH && P <= 0) P = auto_parallelism(T_host, n_seqs);
    BatchPlan bp;
    // single-sequence calls reserve room for their device descriptor too
    fv_status rc = plan_batch(method, models, n_models, T_host, model_host, n_seqs, P, B, n_seqs == 1, bp);
    if (rc != FV_OK) return rc;
    *bytes = bp.total;
    return FV_OK;
}

static fv_status decode_one(int32_t method, const fv_trans* A, const float* log_pi, const float* log_b, int64_t ld,
                            int32_t T, int32_t P, int32_t B, int32_t* path, float* score, int32_t* status,
                            uint32_t flags, void* ws, size_t ws_bytes, fv_stream_t stream) {
    if (T < 1) return fail(FV_E_INVALID_ARG, "T must be >= 1 (got %d)", T);
    if (!A || !log_b || !path || !score) return fail(FV_E_INVALID_ARG, "null argument");
    if (ld < A->K) return fail(FV_E_INVALID_ARG, "ld=%lld < K=%d", (long long)ld, A->K);
    fv_seq s{0, T, log_b, ld, path, score};
    const float* pis[1] = {log_pi};
    return run_batch(method, A, pis, 1, nullptr, &T, nullptr, 1, P, B, &s, status, flags, ws, ws_bytes,
                     reinterpret_cast<hipStream_t>(stream));
}

fv_status fv_decode_vanilla(const fv_trans* A, const float* log_pi, const float* log_b, int64_t ld,
                            int32_t T, int32_t* path, float* score, int32_t* status, uint32_t flags,
                            void* ws, size_t ws_bytes, fv_stream_t stream) {
    return decode_one(FV_VANILLA, A, log_pi, log_b, ld, T, 1, 0, path, score, status, flags, ws, ws_bytes, stream);
}

fv_status fv_decode_flash(const fv_trans* A, const float* log_pi, const float* log_b, int64_t ld,
                          int32_t T, int32_t P, int32_t* path, float* score, int32_t* status,
                          uint32_t flags, void* ws, size_t ws_bytes, fv_stream_t stream) {
    if (P <= 0 && T >= 1) P = auto_parallelism(&T, 1);
    return decode_one(FV_FLASH, A, log_pi, log_b, ld, T, P, 0, path, score, status, flags, ws, ws_bytes, stream);
}

fv_status fv_decode_flash_noalloc(const fv_trans* A, const float* log_pi, const float* log_b, int64_t ld,
                                  int32_t T, int32_t P, int32_t* path, float* score, int32_t* status,
                                  uint32_t flags, fv_stream_t stream) {
    if (T < 1) return fail(FV_E_INVALID_ARG, "T must be >= 1 (got %d)", T);
    if (P <= 0) P = auto_parallelism(&T, 1);
    size_t need = 0;
    fv_status rc = fv_workspace_size(FV_FLASH, A, 1, &T, nullptr, 1, P, 0, &need);
    if (rc != FV_OK) return rc;
    if (need > (size_t)FV_NOALLOC_SCRATCH_BYTES)
        return fail(FV_E_WORKSPACE,
                    "fv_decode_flash_noalloc: this decode needs %zu bytes of scratch; the fixed scratch holds %zu "
                    "(use fv_decode_flash with a workspace)",
                    need, (size_t)FV_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != FV_OK) return rc;
    return decode_one(FV_FLASH, A, log_pi, log_b, ld, T, P, 0, path, score, status, flags, ws,
                      (size_t)FV_NOALLOC_SCRATCH_BYTES, stream);
}

fv_status fv_decode_beam(const fv_trans* A, const float* log_pi, const float* log_b, int64_t ld, int32_t T,
                         int32_t B, int32_t P, int32_t* path, float* score, int32_t* status, uint32_t flags,
                         void* ws, size_t ws_bytes, fv_stream_t stream) {
    if (B < 1 || P < 1) return fail(FV_E_INVALID_ARG, "beam decoding needs B >= 1 and P >= 1");
    return decode_one(FV_BEAM, A, log_pi, log_b, ld, T, P, B, path, score, status, flags, ws, ws_bytes, stream);
}

fv_status fv_decode_batch(const fv_trans* models, const float* const* log_pi, int32_t n_models,
                          const fv_seq* seqs_dev, const int32_t* T_host, const int32_t* model_host,
                          int32_t n_seqs, int32_t method, int32_t P, int32_t B, int32_t* status,
                          uint32_t flags, void* ws, size_t ws_bytes, fv_stream_t stream) {
    if (n_seqs < 0) return fail(FV_E_INVALID_ARG, "n_seqs < 0");
    if (n_seqs > 0 && (!seqs_dev || !T_host)) return fail(FV_E_INVALID_ARG, "null sequence list");
    if (method != FV_VANILLA && method != FV_FLASH && method != FV_BEAM)
        return fail(FV_E_INVALID_ARG, "unknown method %d", method);
    if (method == FV_BEAM && (B < 1 || P < 1)) return fail(FV_E_INVALID_ARG, "beam decoding needs B >= 1 and P >= 1");
    if (method == FV_FLASH && P <= 0) P = auto_parallelism(T_host, n_seqs);
    return run_batch(method, models, log_pi, n_models, seqs_dev, T_host, model_host, n_seqs, P, B, nullptr, status,
                     flags, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

fv_status fv_decode_batch_emit(const fv_trans* models, const fv_emission* emissions, const float* const* log_pi,
                               int32_t n_models, const fv_seq* seqs_dev, const int32_t* T_host,
                               const int32_t* model_host, int32_t n_seqs, int32_t method, int32_t P, int32_t B,
                               int32_t* status, uint32_t flags, void* ws, size_t ws_bytes, fv_stream_t stream) {
    if (n_seqs < 0) return fail(FV_E_INVALID_ARG, "n_seqs < 0");
    if (n_seqs > 0 && (!seqs_dev || !T_host)) return fail(FV_E_INVALID_ARG, "null sequence list");
    if (method != FV_VANILLA && method != FV_FLASH && method != FV_BEAM)
        return fail(FV_E_INVALID_ARG, "unknown method %d", method);
    if (method == FV_BEAM && (B < 1 || P < 1)) return fail(FV_E_INVALID_ARG, "beam decoding needs B >= 1 and P >= 1");
    if (method == FV_FLASH && P <= 0) P = auto_parallelism(T_host, n_seqs);
    return run_batch(method, models, log_pi, n_models, seqs_dev, T_host, model_host, n_seqs, P, B, nullptr, status,
                     flags, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream), emissions);
}

}  // extern "C"
