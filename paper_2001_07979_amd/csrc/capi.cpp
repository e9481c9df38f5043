// C-ABI entry points of the MBP decoder: argument validation, error
// reporting, contexts and the device edge layouts of uploaded codes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mbp_internal.h"

namespace mbp {

static thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? MBP_ENOMEM : MBP_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace mbp

using mbp::fail;
using mbp::hip_fail;

#define HIP_OR_RETURN(expr)                              \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_fail(_e, #expr); \
    } while (0)

extern "C" {

const char *mbp_last_error(void) { return mbp::g_last_error.c_str(); }

int32_t mbp_version(void) { return 1; }

int mbp_ctx_create(int32_t device, mbp_ctx **out) {
    if (!out) return fail(MBP_EINVAL, "mbp_ctx_create: out is NULL");
    *out = nullptr;
    int count = 0;
    HIP_OR_RETURN(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(MBP_EINVAL, "mbp_ctx_create: device " + std::to_string(device) +
                                    " out of range (have " + std::to_string(count) + ")");
    HIP_OR_RETURN(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_OR_RETURN(hipGetDeviceProperties(&prop, device));
    mbp_ctx *ctx = new (std::nothrow) mbp_ctx();
    if (!ctx) return fail(MBP_ENOMEM, "mbp_ctx_create: out of host memory");
    ctx->device = device;
    ctx->num_cus = prop.multiProcessorCount;
    *out = ctx;
    return MBP_OK;
}

void mbp_ctx_destroy(mbp_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
    for (hipEvent_t e : ctx->poll_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->timing_events) (void)hipEventDestroy(e);
    delete ctx;
}

int mbp_code_create(mbp_ctx *ctx, int32_t n, int32_t u, const int32_t *m,
                    const int32_t *const *row_ptr, const int32_t *const *col_idx,
                    mbp_code **out) {
    if (!out) return fail(MBP_EINVAL, "mbp_code_create: out is NULL");
    *out = nullptr;
    if (!ctx) return fail(MBP_EINVAL, "mbp_code_create: ctx is NULL");
    if (n < 1 || n > (1 << 30)) return fail(MBP_EINVAL, "mbp_code_create: n must be in [1, 2^30]");
    if (u < 1 || u > 64) return fail(MBP_EINVAL, "mbp_code_create: u must be in [1, 64]");
    if (!m || !row_ptr || !col_idx) return fail(MBP_EINVAL, "mbp_code_create: null array");
    int64_t M = 0, E = 0;
    for (int32_t l = 0; l < u; ++l) {
        if (m[l] < 1) return fail(MBP_EINVAL, "mbp_code_create: m[" + std::to_string(l) + "] < 1");
        if (!row_ptr[l] || !col_idx[l]) return fail(MBP_EINVAL, "mbp_code_create: null CSR array");
        if (row_ptr[l][0] != 0) return fail(MBP_EINVAL, "mbp_code_create: row_ptr must start at 0");
        M += m[l];
        for (int32_t j = 0; j < m[l]; ++j) {
            int32_t d = row_ptr[l][j + 1] - row_ptr[l][j];
            if (d < 2)
                return fail(MBP_EINVAL, "mbp_code_create: check " + std::to_string(j) + " of matrix " +
                                            std::to_string(l) + " has fewer than two edges");
        }
        E += row_ptr[l][m[l]];
    }
    if (M >= (int64_t(1) << 31) || E >= (int64_t(1) << 31))
        return fail(MBP_EINVAL, "mbp_code_create: stacked graph too large (M, E < 2^31)");

    std::vector<int32_t> h_row_ptr(M + 1), h_col(E), var_cnt(n + 1, 0);
    int32_t maxcd = 0;
    int64_t r = 0, e = 0;
    for (int32_t l = 0; l < u; ++l) {
        const int32_t *rp = row_ptr[l], *ci = col_idx[l];
        for (int32_t j = 0; j < m[l]; ++j, ++r) {
            h_row_ptr[r] = (int32_t)e;
            int32_t prev = -1;
            for (int32_t k = rp[j]; k < rp[j + 1]; ++k) {
                int32_t v = ci[k];
                if (v < 0 || v >= n)
                    return fail(MBP_EINVAL, "mbp_code_create: column out of range in matrix " +
                                                std::to_string(l));
                if (v <= prev)
                    return fail(MBP_EINVAL, "mbp_code_create: columns must ascend strictly within a row "
                                            "(matrix " + std::to_string(l) + ", row " + std::to_string(j) + ")");
                prev = v;
                h_col[e++] = v;
                var_cnt[v + 1]++;
            }
            maxcd = std::max(maxcd, rp[j + 1] - rp[j]);
        }
    }
    h_row_ptr[M] = (int32_t)E;
    if (maxcd > 64)
        return fail(MBP_EUNSUPPORTED, "mbp_code_create: largest check degree " + std::to_string(maxcd) +
                                          " exceeds 64");
    int32_t maxvd = 0;
    for (int32_t i = 0; i < n; ++i) maxvd = std::max(maxvd, var_cnt[i + 1]);
    for (int32_t i = 0; i < n; ++i) var_cnt[i + 1] += var_cnt[i];
    std::vector<int32_t> h_var_edge(E), fill(var_cnt.begin(), var_cnt.end() - 1);
    for (int64_t k = 0; k < E; ++k) h_var_edge[fill[h_col[k]]++] = (int32_t)k;

    mbp_code *code = new (std::nothrow) mbp_code();
    if (!code) return fail(MBP_ENOMEM, "mbp_code_create: out of host memory");
    code->ctx = ctx;
    code->n = n;
    code->u = u;
    code->M = (int32_t)M;
    code->E = E;
    code->m.assign(m, m + u);
    code->max_check_deg = maxcd;
    code->max_var_deg = maxvd;
    auto cleanup = [&](int rc) {
        (void)hipFree(code->d_row_ptr);
        (void)hipFree(code->d_col);
        (void)hipFree(code->d_var_ptr);
        (void)hipFree(code->d_var_edge);
        delete code;
        return rc;
    };
    hipError_t he;
    if ((he = hipSetDevice(ctx->device)) != hipSuccess) return cleanup(hip_fail(he, "hipSetDevice"));
    if ((he = hipMalloc(&code->d_row_ptr, sizeof(int32_t) * (M + 1))) != hipSuccess ||
        (he = hipMalloc(&code->d_col, sizeof(int32_t) * (E + mbp::kIndexPad))) != hipSuccess ||
        (he = hipMalloc(&code->d_var_ptr, sizeof(int32_t) * (n + 1))) != hipSuccess ||
        (he = hipMalloc(&code->d_var_edge, sizeof(int32_t) * (E + mbp::kIndexPad))) != hipSuccess)
        return cleanup(hip_fail(he, "mbp_code_create: hipMalloc"));
    // the kernels read edge indices in fixed-size blocks that may run past the
    // last edge; the padding holds valid (zero) indices
    h_col.resize(E + mbp::kIndexPad, 0);
    h_var_edge.resize(E + mbp::kIndexPad, 0);
    if ((he = hipMemcpy(code->d_row_ptr, h_row_ptr.data(), sizeof(int32_t) * (M + 1),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_col, h_col.data(), sizeof(int32_t) * (E + mbp::kIndexPad),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_var_ptr, var_cnt.data(), sizeof(int32_t) * (n + 1),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_var_edge, h_var_edge.data(), sizeof(int32_t) * (E + mbp::kIndexPad),
                        hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(hip_fail(he, "mbp_code_create: hipMemcpy"));
    ctx->live_codes++;
    *out = code;
    return MBP_OK;
}

void mbp_code_destroy(mbp_code *code) {
    if (!code) return;
    (void)hipSetDevice(code->ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(code->d_row_ptr);
    (void)hipFree(code->d_col);
    (void)hipFree(code->d_var_ptr);
    (void)hipFree(code->d_var_edge);
    code->ctx->live_codes--;
    delete code;
}

int mbp_code_info(const mbp_code *code, int32_t *n, int32_t *u, int32_t *M, int64_t *E,
                  int32_t *max_check_deg, int32_t *max_var_deg) {
    if (!code) return fail(MBP_EINVAL, "mbp_code_info: code is NULL");
    if (n) *n = code->n;
    if (u) *u = code->u;
    if (M) *M = code->M;
    if (E) *E = code->E;
    if (max_check_deg) *max_check_deg = code->max_check_deg;
    if (max_var_deg) *max_var_deg = code->max_var_deg;
    return MBP_OK;
}

int mbp_llr_from_bits(mbp_ctx *ctx, int32_t nframes, int32_t n, const uint8_t *y,
                      const double *e, int32_t dtype, void *llr_out, void *stream) {
    if (!ctx) return fail(MBP_EINVAL, "mbp_llr_from_bits: ctx is NULL");
    if (nframes < 0 || n < 1) return fail(MBP_EINVAL, "mbp_llr_from_bits: bad sizes");
    if (dtype != MBP_F32 && dtype != MBP_F64)
        return fail(MBP_EINVAL, "mbp_llr_from_bits: dtype must be MBP_F32 or MBP_F64");
    if (nframes == 0) return MBP_OK;
    if (!y || !e || !llr_out) return fail(MBP_EINVAL, "mbp_llr_from_bits: null pointer");
    return mbp::llr_impl(ctx, nframes, n, y, e, dtype, llr_out, (hipStream_t)stream);
}

int mbp_decode(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes,
               const void *llr, const uint8_t *synd, uint8_t *bits_out, int32_t *iters_out,
               uint8_t *ok_out, void *llr_out, void *stream) {
    if (!ctx || !code || !p) return fail(MBP_EINVAL, "mbp_decode: null ctx, code or params");
    if (code->ctx != ctx) return fail(MBP_EINVAL, "mbp_decode: code belongs to another context");
    if (p->algo != MBP_ALGO_SPA && p->algo != MBP_ALGO_NMS)
        return fail(MBP_EINVAL, "mbp_decode: unknown algo");
    if (p->dtype != MBP_F32 && p->dtype != MBP_F64) return fail(MBP_EINVAL, "mbp_decode: unknown dtype");
    if (p->max_iter < 1 || p->max_iter > 10000)
        return fail(MBP_EINVAL, "mbp_decode: max_iter must be in [1, 10000]");
    if (p->early_exit != 0 && p->early_exit != 1)
        return fail(MBP_EINVAL, "mbp_decode: early_exit must be 0 or 1");
    if (!std::isfinite(p->llr_clip) || p->llr_clip <= 0.0)
        return fail(MBP_EINVAL, "mbp_decode: llr_clip must be finite and > 0");
    if (p->algo == MBP_ALGO_SPA && p->llr_clip > 30.0)
        return fail(MBP_EINVAL, "mbp_decode: llr_clip must be <= 30 for sum-product");
    if (p->algo == MBP_ALGO_NMS && (!std::isfinite(p->alpha) || p->alpha <= 0.0))
        return fail(MBP_EINVAL, "mbp_decode: alpha must be finite and > 0");
    if (nframes < 0) return fail(MBP_EINVAL, "mbp_decode: nframes < 0");
    if (nframes > 65535 * mbp::kLanes)
        return fail(MBP_EINVAL, "mbp_decode: at most 65535 * 64 frames per call");
    if (nframes == 0) return MBP_OK;
    if (!llr || !synd || !bits_out || !iters_out || !ok_out)
        return fail(MBP_EINVAL, "mbp_decode: null buffer");
    return mbp::decode_impl(ctx, code, p, nframes, llr, synd, bits_out, iters_out, ok_out, llr_out,
                            (hipStream_t)stream);
}

int mbp_profile_enable(mbp_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(MBP_EINVAL, "mbp_profile_enable: ctx is NULL");
    ctx->profiling = enable != 0;
    return MBP_OK;
}

int mbp_profile_reset(mbp_ctx *ctx) {
    if (!ctx) return fail(MBP_EINVAL, "mbp_profile_reset: ctx is NULL");
    for (auto &s : ctx->stats) s = mbp::KernelStat();
    return MBP_OK;
}

int mbp_profile_get(const mbp_ctx *ctx, int32_t which, int64_t *launches, double *total_ms) {
    if (!ctx) return fail(MBP_EINVAL, "mbp_profile_get: ctx is NULL");
    if (which < 0 || which >= mbp::kNumKernels) return fail(MBP_EINVAL, "mbp_profile_get: bad kernel id");
    if (launches) *launches = ctx->stats[which].launches;
    if (total_ms) *total_ms = ctx->stats[which].total_ms;
    return MBP_OK;
}

}  // extern "C"
