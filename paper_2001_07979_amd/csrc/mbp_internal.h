// Internal declarations shared by the C-ABI layer (capi.cpp) and the HIP
// kernels (decode.hip) of the MBP decoder library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mbp.h"

namespace mbp {

// Frames per interleaved group: one frame per lane of a 64-wide wavefront.
constexpr int kLanes = 64;

// Largest check degree the batched decode's sum-product rule handles (its
// unrolled slot count: 34 slots keep the sum-product persistent kernel at 2
// waves per SIMD; 64 would need all 256 registers, 1 wave).
constexpr int kBatchedSpaMaxDeg = 34;

// Largest number of matrices the independent-decoder coupling handles: the
// flooding variable pass finds an edge's matrix from three boundaries.
constexpr int kIndepMaxU = 4;

// Extra zero entries after the device edge-index arrays, so kernels can read
// indices in fixed blocks (up to 64 + 32 entries) past the end.
constexpr int kIndexPad = 128;

// Packing of d_var_rt: the table row (below 64 * 65 / 2 = 2080) in the low
// kRtShift bits, the check above them.
constexpr int kRtShift = 12;
constexpr int64_t kRtMaxChecks = int64_t(1) << (32 - kRtShift);

// Per-kernel timing totals (see mbp_profile_get).
enum KernelId {
    kCheckNode = 0,
    kVarNode = 1,
    kSyndrome = 2,
    kStaging = 3,
    kFirst = 4,   // the first iteration in closed form
    kSecond = 5,  // the check pass after it, which rebuilds the old messages
    kNumKernels = 6
};

struct KernelStat {
    int64_t launches = 0;
    double total_ms = 0.0;
};

// Records the last error of the calling thread and returns `code`.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

}  // namespace mbp

struct mbp_ctx {
    int32_t device = 0;
    int32_t num_cus = 0;
    // Decode workspace: one device allocation, grown on demand.
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // Per-group "still running" masks the kernels write to host-visible
    // pinned memory, so the host can stop launching iterations early.
    uint64_t *status_host = nullptr;
    uint64_t *status_dev = nullptr;
    int32_t status_cap = 0;
    std::vector<hipEvent_t> poll_events;
    // Profiling.
    int32_t profiling = 0;  // bit k: time launches of kernel id k
    mbp::KernelStat stats[mbp::kNumKernels];
    std::vector<hipEvent_t> timing_events;
    int32_t live_codes = 0;  // codes, plans and queues of the context not yet destroyed
    // set by mbp_ctx_destroy while codes or plans of the context are still
    // alive: the GPU resources are gone and the last of their destroy calls
    // frees the struct
    bool closed = false;
};

// A serving queue: frames submitted as batches wait until a flush decodes
// everything pending in one batched launch; each flush owns its workspace and
// an event until poll or wait sees it complete.
struct mbp_queue {
    mbp_ctx *ctx = nullptr;
    mbp_params params{};
    mbp_tuning tuning{};
    std::vector<mbp_batch> pending;
    int64_t pending_frames = 0;
    struct Flight {
        void *ws = nullptr;
        hipEvent_t done = nullptr;
        int32_t *err_dev = nullptr;
        int64_t frames = 0;
    };
    std::vector<Flight> flights;  // oldest first
    int64_t done_frames = 0;
};

struct mbp_plan {
    mbp_ctx *ctx = nullptr;
    void *ws = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t *err_dev = nullptr;
};

// A run of consecutive variables whose degrees fit dv slots of the variable
// pass (variables [i0, i1)).
struct mbp_var_class {
    int32_t i0, i1, dv;
};

struct mbp_code {
    mbp_ctx *ctx = nullptr;
    int32_t n = 0, u = 0, M = 0;
    int64_t E = 0;
    std::vector<int32_t> m;
    std::vector<int64_t> e_off;  // [u + 1] first stacked edge of each matrix
    int32_t max_check_deg = 0, max_var_deg = 0;
    int32_t max_var_deg_matrix = 0;  // largest degree of a variable within one matrix
    // Device edge layouts of the stacked graph [H_1; ...; H_u]:
    // edges in check-major order (matrix, row, column); for each variable its
    // edges in the same order.
    int32_t *d_row_ptr = nullptr;   // [M + 1]
    int32_t *d_row_mat = nullptr;   // [M] matrix of each stacked check
    int32_t *d_mat_off = nullptr;   // [u + 1] first stacked check of each matrix
    int32_t *d_col = nullptr;       // [E]
    int32_t *d_var_ptr = nullptr;   // [n + 1]
    int32_t *d_var_edge = nullptr;  // [E]
    // var_edge again, with bit 31 set on an entry whose edge starts the next
    // matrix's edges in its variable's list (not on a variable's first entry)
    int32_t *d_var_edge_f = nullptr;  // [E]
    // position in var_edge of the first edge of matrix l at variable i, at
    // [l * n + i] for l = 0..u (row u: one past the variable's last edge)
    int32_t *d_var_mptr = nullptr;  // [(u + 1) n]
    // per variable, the slots of its edge list that start the next matrix's
    // edges (bit j: slot j), and the variables split into degree classes
    uint64_t *d_var_runs = nullptr;  // [n]
    // var_edge again, each entry as (check << kRtShift) | (row of the
    // first-iteration magnitude table) for its edge: the table has one row
    // per slot of every check degree the code has (degrees ascending, slot j
    // of degree d at first_row(d) + j), first_rows rows in all, and
    // d_first_rowdj gives each row's (d << 8) | j. Null when the code has
    // kRtMaxChecks checks or more.
    uint32_t *d_var_rt = nullptr;       // [E + kIndexPad]
    uint32_t *d_first_rowdj = nullptr;  // [first_rows]
    int32_t first_rows = 0;
    std::vector<mbp_var_class> var_classes;
};

namespace mbp {

// Implemented in decode.hip; arguments are validated by capi.cpp. The
// channel is either llr (y and e null) or Bob's bits y with error rates e
// (llr null).
int decode_impl(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes,
                const void *llr, const uint8_t *y, const double *e, const uint8_t *synd, uint8_t *bits_out,
                int32_t *iters_out, uint8_t *ok_out, void *llr_out, hipStream_t stream);
// Implemented in syndrome.hip; arguments are validated by capi.cpp.
int syndrome_impl(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, const uint8_t *x, uint8_t *z,
                  hipStream_t stream);
// The allocation-free variant (syndrome.hip): its bit words live in a fixed
// device array of kNoallocWords words, whose address scratch_setup looks up
// once per device (with that device current).
constexpr size_t kNoallocWords = size_t(1) << 21;  // 16 MiB
int scratch_setup(int device);
int syndrome_noalloc_impl(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, const uint8_t *x, uint8_t *z,
                          hipStream_t stream);
int llr_impl(mbp_ctx *ctx, int32_t nframes, int32_t n, const uint8_t *y, const double *e,
             int32_t dtype, void *llr_out, hipStream_t stream);
int peg_build_impl(mbp_ctx *ctx, int32_t n, int32_t m, int32_t u, const int32_t *var_deg, const uint64_t *seeds,
                   int32_t max_depth, int32_t *row_ptr, int32_t *col_idx);

// Batched persistent decode (batched.hip).
mbp_tuning default_tuning();
int check_tuning(const mbp_tuning &tu);
uint64_t batched_workspace_bytes(int32_t nb, const mbp_batch *b, const mbp_tuning &tu);
int batched_decode(mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu,
                   hipStream_t stream);
// Uploads the descriptors into ws (a workspace of batched_workspace_bytes)
// and enqueues the whole batched decode on stream, without waiting; *err_dev
// receives the grid-barrier error flag's address in ws (nonzero: timed out).
int batched_launch(mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu,
                   void *ws, hipStream_t stream, int32_t **err_dev);
int batched_plan_capture(mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu,
                         void *ws, hipGraphExec_t *exec, int32_t **err_dev);

// Unrolled normalized min-sum (unrolled.hip).
uint64_t unrolled_workspace_bytes(const mbp_code *code, int32_t nframes, int32_t K, int32_t ckpt);
int unrolled_forward(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, int32_t K, int32_t ckpt,
                     double clip, const float *llr, const uint8_t *synd, const float *alpha,
                     float *llr_out, void *ws, hipStream_t stream);
int unrolled_backward(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, int32_t K, int32_t ckpt,
                      double clip, const float *llr, const uint8_t *synd, const float *alpha,
                      const float *grad_out, float *grad_llr, float *grad_alpha, void *ws,
                      hipStream_t stream);

}  // namespace mbp
