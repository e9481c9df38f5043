// C-ABI entry points of the MBP decoder: argument validation, error
// reporting, contexts and the device edge layouts of uploaded codes.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
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

namespace {

// Checks shared by mbp_decode and mbp_decode_from_bits; `f` names the call.
int check_decode(const char *f, mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes) {
    const std::string fn(f);
    if (!ctx || !code || !p) return fail(MBP_EINVAL, fn + ": null ctx, code or params");
    if (code->ctx != ctx) return fail(MBP_EINVAL, fn + ": code belongs to another context");
    if (p->algo != MBP_ALGO_SPA && p->algo != MBP_ALGO_NMS) return fail(MBP_EINVAL, fn + ": unknown algo");
    if (p->dtype != MBP_F32 && p->dtype != MBP_F64) return fail(MBP_EINVAL, fn + ": unknown dtype");
    if (p->max_iter < 1 || p->max_iter > 10000) return fail(MBP_EINVAL, fn + ": max_iter must be in [1, 10000]");
    if (p->early_exit != 0 && p->early_exit != 1) return fail(MBP_EINVAL, fn + ": early_exit must be 0 or 1");
    if (p->compact != 0 && p->compact != 1) return fail(MBP_EINVAL, fn + ": compact must be 0 or 1");
    if (p->schedule != MBP_FLOODING && p->schedule != MBP_MATRIX_SERIAL)
        return fail(MBP_EINVAL, fn + ": unknown schedule");
    if (p->coupling != MBP_JOINT && p->coupling != MBP_INDEPENDENT)
        return fail(MBP_EINVAL, fn + ": unknown coupling");
    if (p->msg_dtype != MBP_MSG_F32 && p->msg_dtype != MBP_MSG_F16)
        return fail(MBP_EINVAL, fn + ": unknown msg_dtype");
    if (p->msg_dtype == MBP_MSG_F16 &&
        (p->dtype != MBP_F32 || p->schedule != MBP_FLOODING || p->coupling != MBP_JOINT))
        return fail(MBP_EUNSUPPORTED, fn + ": binary16 messages need dtype F32, the flooding schedule and the "
                                           "joint coupling");
    if (p->coupling == MBP_INDEPENDENT && code->u > mbp::kIndepMaxU)
        return fail(MBP_EUNSUPPORTED, fn + ": independent decoders take codes of at most " +
                                          std::to_string(mbp::kIndepMaxU) + " matrices");
    if (!std::isfinite(p->llr_clip) || p->llr_clip <= 0.0)
        return fail(MBP_EINVAL, fn + ": llr_clip must be finite and > 0");
    if (p->algo == MBP_ALGO_SPA && p->llr_clip > 30.0)
        return fail(MBP_EINVAL, fn + ": llr_clip must be <= 30 for sum-product");
    if (p->algo == MBP_ALGO_NMS && (!std::isfinite(p->alpha) || p->alpha <= 0.0))
        return fail(MBP_EINVAL, fn + ": alpha must be finite and > 0");
    if (nframes < 0) return fail(MBP_EINVAL, fn + ": nframes < 0");
    if (nframes > 65535 * mbp::kLanes) return fail(MBP_EINVAL, fn + ": at most 65535 * 64 frames per call");
    return MBP_OK;
}

}  // namespace

extern "C" {

const char *mbp_last_error(void) { return mbp::g_last_error.c_str(); }

int32_t mbp_version(void) { return 3; }

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
    // the allocation-free calls' fixed scratch: its address on this device
    if (int rc = mbp::scratch_setup(device); rc != MBP_OK) return rc;
    mbp_ctx *ctx = new (std::nothrow) mbp_ctx();
    if (!ctx) return fail(MBP_ENOMEM, "mbp_ctx_create: out of host memory");
    ctx->device = device;
    ctx->num_cus = prop.multiProcessorCount;
    *out = ctx;
    return MBP_OK;
}

void mbp_ctx_destroy(mbp_ctx *ctx) {
    if (!ctx || ctx->closed) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
    for (hipEvent_t e : ctx->poll_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->timing_events) (void)hipEventDestroy(e);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    ctx->status_host = nullptr;
    ctx->status_dev = nullptr;
    ctx->status_cap = 0;
    ctx->poll_events.clear();
    ctx->timing_events.clear();
    // codes still alive keep the struct (their destroy reads its device and
    // count); the last of them frees it
    if (ctx->live_codes > 0)
        ctx->closed = true;
    else
        delete ctx;
}

int mbp_code_create(mbp_ctx *ctx, int32_t n, int32_t u, const int32_t *m,
                    const int32_t *const *row_ptr, const int32_t *const *col_idx,
                    mbp_code **out) {
    if (!out) return fail(MBP_EINVAL, "mbp_code_create: out is NULL");
    *out = nullptr;
    if (!ctx) return fail(MBP_EINVAL, "mbp_code_create: ctx is NULL");
    // the FP32 check pass addresses a variable's 64-frame row (256 bytes)
    // with a 32-bit signed byte offset
    if (n < 1 || n > (1 << 23)) return fail(MBP_EINVAL, "mbp_code_create: n must be in [1, 2^23]");
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

    std::vector<int32_t> h_row_ptr(M + 1), h_row_mat(M), h_col(E), var_cnt(n + 1, 0), h_mat_off(u + 1, 0);
    for (int32_t l = 0; l < u; ++l) h_mat_off[l + 1] = h_mat_off[l] + m[l];
    int32_t maxcd = 0;
    int64_t r = 0, e = 0;
    for (int32_t l = 0; l < u; ++l) {
        const int32_t *rp = row_ptr[l], *ci = col_idx[l];
        for (int32_t j = 0; j < m[l]; ++j, ++r) {
            h_row_ptr[r] = (int32_t)e;
            h_row_mat[r] = l;
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
    if (maxvd > 64)
        return fail(MBP_EUNSUPPORTED, "mbp_code_create: largest variable degree over all matrices " +
                                          std::to_string(maxvd) + " exceeds 64");
    for (int32_t i = 0; i < n; ++i) var_cnt[i + 1] += var_cnt[i];
    std::vector<int32_t> h_var_edge(E), fill(var_cnt.begin(), var_cnt.end() - 1);
    for (int64_t k = 0; k < E; ++k) h_var_edge[fill[h_col[k]]++] = (int32_t)k;
    // each variable's edges ascend, so its edges of one matrix are one run:
    // mark where each run after the first starts, and where every matrix's
    // run starts (empty runs included)
    std::vector<int32_t> edge_mat(E);
    for (int64_t rr = 0; rr < M; ++rr)
        for (int32_t k = h_row_ptr[rr]; k < h_row_ptr[rr + 1]; ++k) edge_mat[k] = h_row_mat[rr];
    std::vector<int32_t> h_var_edge_f(h_var_edge), h_var_mptr(static_cast<size_t>(u + 1) * n);
    int32_t maxvdm = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t k = var_cnt[i];
        for (int32_t l = 0; l < u; ++l) {
            h_var_mptr[static_cast<size_t>(l) * n + i] = k;
            const int32_t k0 = k;
            while (k < var_cnt[i + 1] && edge_mat[h_var_edge[k]] == l) {
                if (k == k0 && k > var_cnt[i]) h_var_edge_f[k] |= static_cast<int32_t>(0x80000000u);
                ++k;
            }
            maxvdm = std::max(maxvdm, k - k0);
        }
        h_var_mptr[static_cast<size_t>(u) * n + i] = var_cnt[i + 1];
    }

    // the run starts as a bitmask per variable (degrees are at most 64)
    std::vector<uint64_t> h_var_runs(n, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = var_cnt[i]; k < var_cnt[i + 1]; ++k)
            if (h_var_edge_f[k] < 0) h_var_runs[i] |= 1ull << (k - var_cnt[i]);
    // degree classes: runs of consecutive variables by the slot count their
    // degree needs; runs of fewer than 2048 variables merge into a neighbour
    // (taking the larger count), and a code with many runs gets one class
    auto cap_of = [](int32_t d) {
        for (int32_t c : {8, 12, 16, 32})
            if (d <= c) return c;
        return 64;
    };
    std::vector<mbp_var_class> classes;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t c = cap_of(var_cnt[i + 1] - var_cnt[i]);
        if (classes.empty() || classes.back().dv != c)
            classes.push_back({i, i + 1, c});
        else
            classes.back().i1 = i + 1;
        if (classes.size() > 64) break;
    }
    if (classes.size() > 64) {
        classes.assign(1, mbp_var_class{0, n, cap_of(maxvd)});
    } else {
        for (bool merged = true; merged && classes.size() > 1;) {
            merged = false;
            for (size_t k = 0; k < classes.size(); ++k) {
                if (classes[k].i1 - classes[k].i0 >= 2048) continue;
                const size_t o = k > 0 ? k - 1 : k + 1;  // the neighbour it joins
                const size_t lo = std::min(k, o), hi = std::max(k, o);
                classes[lo] = {classes[lo].i0, classes[hi].i1, std::max(classes[lo].dv, classes[hi].dv)};
                classes.erase(classes.begin() + static_cast<std::ptrdiff_t>(hi));
                merged = true;
                break;
            }
            // neighbours that now share a slot count become one class
            for (size_t k = 1; k < classes.size();) {
                if (classes[k].dv == classes[k - 1].dv) {
                    classes[k - 1].i1 = classes[k].i1;
                    classes.erase(classes.begin() + static_cast<std::ptrdiff_t>(k));
                } else {
                    ++k;
                }
            }
        }
        if (classes.size() > 6) classes.assign(1, mbp_var_class{0, n, cap_of(maxvd)});
    }

    mbp_code *code = new (std::nothrow) mbp_code();
    if (!code) return fail(MBP_ENOMEM, "mbp_code_create: out of host memory");
    code->var_classes = classes;
    code->ctx = ctx;
    code->n = n;
    code->u = u;
    code->M = (int32_t)M;
    code->E = E;
    code->m.assign(m, m + u);
    code->e_off.resize(u + 1);
    for (int32_t l = 0; l <= u; ++l) code->e_off[l] = h_row_ptr[h_mat_off[l]];
    code->max_check_deg = maxcd;
    code->max_var_deg = maxvd;
    code->max_var_deg_matrix = maxvdm;
    auto cleanup = [&](int rc) {
        (void)hipFree(code->d_row_ptr);
        (void)hipFree(code->d_row_mat);
        (void)hipFree(code->d_mat_off);
        (void)hipFree(code->d_col);
        (void)hipFree(code->d_var_ptr);
        (void)hipFree(code->d_var_edge);
        (void)hipFree(code->d_var_edge_f);
        (void)hipFree(code->d_var_mptr);
        (void)hipFree(code->d_var_runs);
        (void)hipFree(code->d_var_rt);
        (void)hipFree(code->d_first_rowdj);
        delete code;
        return rc;
    };
    hipError_t he;
    if ((he = hipSetDevice(ctx->device)) != hipSuccess) return cleanup(hip_fail(he, "hipSetDevice"));
    if ((he = hipMalloc(&code->d_row_ptr, sizeof(int32_t) * (M + 1))) != hipSuccess ||
        (he = hipMalloc(&code->d_row_mat, sizeof(int32_t) * M)) != hipSuccess ||
        (he = hipMalloc(&code->d_mat_off, sizeof(int32_t) * (u + 1))) != hipSuccess ||
        (he = hipMalloc(&code->d_col, sizeof(int32_t) * (E + mbp::kIndexPad))) != hipSuccess ||
        (he = hipMalloc(&code->d_var_ptr, sizeof(int32_t) * (n + 1))) != hipSuccess ||
        (he = hipMalloc(&code->d_var_edge, sizeof(int32_t) * (E + mbp::kIndexPad))) != hipSuccess ||
        (he = hipMalloc(&code->d_var_edge_f, sizeof(int32_t) * (E + mbp::kIndexPad))) != hipSuccess ||
        (he = hipMalloc(&code->d_var_mptr, sizeof(int32_t) * (u + 1) * n)) != hipSuccess ||
        (he = hipMalloc(&code->d_var_runs, sizeof(uint64_t) * n)) != hipSuccess)
        return cleanup(hip_fail(he, "mbp_code_create: hipMalloc"));
    // each variable edge's check and its row of the first-iteration
    // magnitude table: one row per slot of every check degree present
    if (M < mbp::kRtMaxChecks) {
        std::vector<int32_t> first_row(65, -1);
        std::vector<uint32_t> rowdj;
        std::vector<char> present(65, 0);
        for (int64_t rr = 0; rr < M; ++rr) present[h_row_ptr[rr + 1] - h_row_ptr[rr]] = 1;
        for (int32_t d = 1; d <= 64; ++d) {
            if (!present[d]) continue;
            first_row[d] = static_cast<int32_t>(rowdj.size());
            for (int32_t j = 0; j < d; ++j) rowdj.push_back(static_cast<uint32_t>(d << 8 | j));
        }
        std::vector<uint32_t> h_var_rt(E + mbp::kIndexPad, 0);
        std::vector<int32_t> edge_row(E);
        for (int64_t rr = 0; rr < M; ++rr)
            for (int32_t k = h_row_ptr[rr]; k < h_row_ptr[rr + 1]; ++k) edge_row[k] = static_cast<int32_t>(rr);
        for (int64_t k = 0; k < E; ++k) {
            const int32_t ek = h_var_edge[k], rr = edge_row[ek];
            const int32_t d = h_row_ptr[rr + 1] - h_row_ptr[rr], j = ek - h_row_ptr[rr];
            h_var_rt[k] = (static_cast<uint32_t>(rr) << mbp::kRtShift) | static_cast<uint32_t>(first_row[d] + j);
        }
        code->first_rows = static_cast<int32_t>(rowdj.size());
        if ((he = hipMalloc(&code->d_var_rt, sizeof(uint32_t) * (E + mbp::kIndexPad))) != hipSuccess ||
            (he = hipMemcpy(code->d_var_rt, h_var_rt.data(), sizeof(uint32_t) * (E + mbp::kIndexPad),
                            hipMemcpyHostToDevice)) != hipSuccess ||
            (he = hipMalloc(&code->d_first_rowdj, sizeof(uint32_t) * rowdj.size())) != hipSuccess ||
            (he = hipMemcpy(code->d_first_rowdj, rowdj.data(), sizeof(uint32_t) * rowdj.size(),
                            hipMemcpyHostToDevice)) != hipSuccess)
            return cleanup(hip_fail(he, "mbp_code_create: first-iteration rows"));
    }
    // the kernels read edge indices in fixed-size blocks that may run past the
    // last edge; the padding holds valid (zero) indices
    h_col.resize(E + mbp::kIndexPad, 0);
    h_var_edge.resize(E + mbp::kIndexPad, 0);
    h_var_edge_f.resize(E + mbp::kIndexPad, 0);
    if ((he = hipMemcpy(code->d_row_ptr, h_row_ptr.data(), sizeof(int32_t) * (M + 1),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_row_mat, h_row_mat.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (he = hipMemcpy(code->d_mat_off, h_mat_off.data(), sizeof(int32_t) * (u + 1),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_col, h_col.data(), sizeof(int32_t) * (E + mbp::kIndexPad),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_var_ptr, var_cnt.data(), sizeof(int32_t) * (n + 1),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_var_edge, h_var_edge.data(), sizeof(int32_t) * (E + mbp::kIndexPad),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_var_edge_f, h_var_edge_f.data(), sizeof(int32_t) * (E + mbp::kIndexPad),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_var_mptr, h_var_mptr.data(), sizeof(int32_t) * (u + 1) * n,
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(code->d_var_runs, h_var_runs.data(), sizeof(uint64_t) * n, hipMemcpyHostToDevice)) !=
            hipSuccess)
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
    (void)hipFree(code->d_row_mat);
    (void)hipFree(code->d_mat_off);
    (void)hipFree(code->d_col);
    (void)hipFree(code->d_var_ptr);
    (void)hipFree(code->d_var_edge);
    (void)hipFree(code->d_var_edge_f);
    (void)hipFree(code->d_var_mptr);
    (void)hipFree(code->d_var_runs);
    (void)hipFree(code->d_var_rt);
    (void)hipFree(code->d_first_rowdj);
    mbp_ctx *ctx = code->ctx;
    delete code;
    if (--ctx->live_codes == 0 && ctx->closed) delete ctx;
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

int mbp_syndrome(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, const uint8_t *x, uint8_t *synd_out,
                 void *stream) {
    if (!ctx || !code) return fail(MBP_EINVAL, "mbp_syndrome: null ctx or code");
    if (code->ctx != ctx) return fail(MBP_EINVAL, "mbp_syndrome: code belongs to another context");
    if (nframes < 0) return fail(MBP_EINVAL, "mbp_syndrome: nframes < 0");
    if (nframes > 65535 * mbp::kLanes) return fail(MBP_EINVAL, "mbp_syndrome: at most 65535 * 64 frames per call");
    if (nframes == 0) return MBP_OK;
    if (!x || !synd_out) return fail(MBP_EINVAL, "mbp_syndrome: null buffer");
    return mbp::syndrome_impl(ctx, code, nframes, x, synd_out, (hipStream_t)stream);
}

int mbp_syndrome_noalloc(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, const uint8_t *x,
                         uint8_t *synd_out, void *stream) {
    if (!ctx || !code) return fail(MBP_EINVAL, "mbp_syndrome_noalloc: null ctx or code");
    if (code->ctx != ctx) return fail(MBP_EINVAL, "mbp_syndrome_noalloc: code belongs to another context");
    if (nframes < 0) return fail(MBP_EINVAL, "mbp_syndrome_noalloc: nframes < 0");
    if (nframes > 65535 * mbp::kLanes)
        return fail(MBP_EINVAL, "mbp_syndrome_noalloc: at most 65535 * 64 frames per call");
    if (nframes == 0) return MBP_OK;
    if (!x || !synd_out) return fail(MBP_EINVAL, "mbp_syndrome_noalloc: null buffer");
    return mbp::syndrome_noalloc_impl(ctx, code, nframes, x, synd_out, (hipStream_t)stream);
}

int mbp_peg_build(mbp_ctx *ctx, int32_t n, int32_t m, int32_t u, const int32_t *var_deg, const uint64_t *seeds,
                  int32_t max_depth, int32_t *row_ptr, int32_t *col_idx) {
    if (!ctx) return fail(MBP_EINVAL, "mbp_peg_build: null ctx");
    if (n < 1 || m < 1 || u < 1) return fail(MBP_EINVAL, "mbp_peg_build: n, m and u must be >= 1");
    if (!var_deg || !seeds || !row_ptr || !col_idx) return fail(MBP_EINVAL, "mbp_peg_build: null buffer");
    int64_t E = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (var_deg[i] < 1 || var_deg[i] > m || var_deg[i] > 1024)
            return fail(MBP_EINVAL, "mbp_peg_build: variable degrees must be in [1, min(m, 1024)]");
        if (i > 0 && var_deg[i] < var_deg[i - 1])
            return fail(MBP_EINVAL, "mbp_peg_build: variable degrees must be non-decreasing");
        E += var_deg[i];
    }
    if (E >= INT32_MAX / 2) return fail(MBP_EINVAL, "mbp_peg_build: too many edges");
    return mbp::peg_build_impl(ctx, n, m, u, var_deg, seeds, max_depth, row_ptr, col_idx);
}

int mbp_decode(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes,
               const void *llr, const uint8_t *synd, uint8_t *bits_out, int32_t *iters_out,
               uint8_t *ok_out, void *llr_out, void *stream) {
    int rc = check_decode("mbp_decode", ctx, code, p, nframes);
    if (rc != MBP_OK || nframes == 0) return rc;
    if (!llr || !synd || !bits_out || !iters_out || !ok_out)
        return fail(MBP_EINVAL, "mbp_decode: null buffer");
    return mbp::decode_impl(ctx, code, p, nframes, llr, nullptr, nullptr, synd, bits_out, iters_out, ok_out,
                            llr_out, (hipStream_t)stream);
}

int mbp_decode_from_bits(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes,
                         const uint8_t *y, const double *e, const uint8_t *synd, uint8_t *bits_out,
                         int32_t *iters_out, uint8_t *ok_out, void *llr_out, void *stream) {
    int rc = check_decode("mbp_decode_from_bits", ctx, code, p, nframes);
    if (rc != MBP_OK || nframes == 0) return rc;
    if (!y || !e || !synd || !bits_out || !iters_out || !ok_out)
        return fail(MBP_EINVAL, "mbp_decode_from_bits: null buffer");
    return mbp::decode_impl(ctx, code, p, nframes, nullptr, y, e, synd, bits_out, iters_out, ok_out, llr_out,
                            (hipStream_t)stream);
}

static int check_unrolled(const char *fn, const mbp_code *code, int32_t nframes, int32_t K,
                          int32_t ckpt) {
    if (!code) return fail(MBP_EINVAL, std::string(fn) + ": code is NULL");
    if (nframes < 1 || nframes > 65535 * mbp::kLanes)
        return fail(MBP_EINVAL, std::string(fn) + ": nframes must be in [1, 65535 * 64]");
    if (K < 1 || K > 1000) return fail(MBP_EINVAL, std::string(fn) + ": K must be in [1, 1000]");
    if (ckpt < 1 || ckpt > K) return fail(MBP_EINVAL, std::string(fn) + ": ckpt_every must be in [1, K]");
    return MBP_OK;
}

int mbp_unrolled_workspace_bytes(const mbp_code *code, int32_t nframes, int32_t K,
                                 int32_t ckpt_every, uint64_t *bytes) {
    int rc = check_unrolled("mbp_unrolled_workspace_bytes", code, nframes, K, ckpt_every);
    if (rc != MBP_OK) return rc;
    if (!bytes) return fail(MBP_EINVAL, "mbp_unrolled_workspace_bytes: bytes is NULL");
    *bytes = mbp::unrolled_workspace_bytes(code, nframes, K, ckpt_every);
    return MBP_OK;
}

static int check_unrolled_call(const char *fn, mbp_ctx *ctx, const mbp_code *code, int32_t nframes,
                               int32_t K, int32_t ckpt, double clip, void *ws, uint64_t ws_bytes) {
    if (!ctx) return fail(MBP_EINVAL, std::string(fn) + ": ctx is NULL");
    int rc = check_unrolled(fn, code, nframes, K, ckpt);
    if (rc != MBP_OK) return rc;
    if (code->ctx != ctx) return fail(MBP_EINVAL, std::string(fn) + ": code belongs to another context");
    if (!std::isfinite(clip) || clip <= 0.0)
        return fail(MBP_EINVAL, std::string(fn) + ": llr_clip must be finite and > 0");
    if (!ws || ws_bytes < mbp::unrolled_workspace_bytes(code, nframes, K, ckpt))
        return fail(MBP_EINVAL, std::string(fn) + ": workspace missing or smaller than "
                                                  "mbp_unrolled_workspace_bytes");
    return MBP_OK;
}

int mbp_nms_unrolled_fwd(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, int32_t K,
                         int32_t ckpt_every, double llr_clip, const float *llr, const uint8_t *synd,
                         const float *alpha, float *llr_out, void *workspace,
                         uint64_t workspace_bytes, void *stream) {
    int rc = check_unrolled_call("mbp_nms_unrolled_fwd", ctx, code, nframes, K, ckpt_every, llr_clip,
                                 workspace, workspace_bytes);
    if (rc != MBP_OK) return rc;
    if (!llr || !synd || !alpha || !llr_out) return fail(MBP_EINVAL, "mbp_nms_unrolled_fwd: null buffer");
    return mbp::unrolled_forward(ctx, code, nframes, K, ckpt_every, llr_clip, llr, synd, alpha, llr_out,
                                 workspace, (hipStream_t)stream);
}

int mbp_nms_unrolled_bwd(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, int32_t K,
                         int32_t ckpt_every, double llr_clip, const float *llr, const uint8_t *synd,
                         const float *alpha, const float *grad_out, float *grad_llr,
                         float *grad_alpha, void *workspace, uint64_t workspace_bytes,
                         void *stream) {
    int rc = check_unrolled_call("mbp_nms_unrolled_bwd", ctx, code, nframes, K, ckpt_every, llr_clip,
                                 workspace, workspace_bytes);
    if (rc != MBP_OK) return rc;
    if (!llr || !synd || !alpha || !grad_out || !grad_llr || !grad_alpha)
        return fail(MBP_EINVAL, "mbp_nms_unrolled_bwd: null buffer");
    return mbp::unrolled_backward(ctx, code, nframes, K, ckpt_every, llr_clip, llr, synd, alpha, grad_out,
                                  grad_llr, grad_alpha, workspace, (hipStream_t)stream);
}

int mbp_tuning_default(mbp_tuning *out) {
    if (!out) return fail(MBP_EINVAL, "mbp_tuning_default: out is NULL");
    *out = mbp::default_tuning();
    return MBP_OK;
}

// Parameters of a batched decode (FP32, flooding; min-sum or sum-product).
static int check_batched_params(const char *fn, const mbp_params *p) {
    const std::string f(fn);
    if (p->algo != MBP_ALGO_NMS && p->algo != MBP_ALGO_SPA) return fail(MBP_EINVAL, f + ": unknown algo");
    if (p->dtype != MBP_F32) return fail(MBP_EUNSUPPORTED, f + ": the batched decode runs in FP32 only");
    if (p->schedule != MBP_FLOODING)
        return fail(MBP_EUNSUPPORTED, f + ": the batched decode runs the flooding schedule only");
    if (p->coupling != MBP_JOINT)
        return fail(MBP_EUNSUPPORTED, f + ": the batched decode runs the joint (stacked) graph only");
    if (p->msg_dtype != MBP_MSG_F32)
        return fail(MBP_EUNSUPPORTED, f + ": the batched decode stores FP32 messages only");
    if (p->max_iter < 1 || p->max_iter > 10000) return fail(MBP_EINVAL, f + ": max_iter must be in [1, 10000]");
    if (p->early_exit != 0 && p->early_exit != 1) return fail(MBP_EINVAL, f + ": early_exit must be 0 or 1");
    if (!std::isfinite(p->llr_clip) || p->llr_clip <= 0.0)
        return fail(MBP_EINVAL, f + ": llr_clip must be finite and > 0");
    if (p->algo == MBP_ALGO_SPA && p->llr_clip > 30.0)
        return fail(MBP_EINVAL, f + ": llr_clip must be <= 30 for sum-product");
    if (p->algo == MBP_ALGO_NMS && (!std::isfinite(p->alpha) || p->alpha <= 0.0))
        return fail(MBP_EINVAL, f + ": alpha must be finite and > 0");
    return MBP_OK;
}

static int check_batches(const char *fn, mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p,
                         const mbp_tuning *tu) {
    const std::string f(fn);
    if (!ctx || !p) return fail(MBP_EINVAL, f + ": null ctx or params");
    if (nb < 1 || !b) return fail(MBP_EINVAL, f + ": need at least one batch");
    if (int rc = check_batched_params(fn, p); rc != MBP_OK) return rc;
    int64_t groups = 0;
    for (int32_t i = 0; i < nb; ++i) {
        const mbp_batch &x = b[i];
        if (!x.code || x.code->ctx != ctx) return fail(MBP_EINVAL, f + ": batch code missing or of another context");
        if (p->algo == MBP_ALGO_SPA && x.code->max_check_deg > mbp::kBatchedSpaMaxDeg)
            return fail(MBP_EUNSUPPORTED, f + ": the batched sum-product rule takes check degrees up to " +
                                              std::to_string(mbp::kBatchedSpaMaxDeg));
        if (x.nframes < 1 || x.nframes > 65535 * mbp::kLanes)
            return fail(MBP_EINVAL, f + ": batch nframes must be in [1, 65535 * 64]");
        if (!x.llr || !x.synd || !x.bits_out || !x.iters_out || !x.ok_out)
            return fail(MBP_EINVAL, f + ": null batch buffer");
        groups += (x.nframes + mbp::kLanes - 1) / mbp::kLanes;
    }
    if (groups > (1 << 24)) return fail(MBP_EINVAL, f + ": too many frame groups");
    if (tu) return mbp::check_tuning(*tu);
    return MBP_OK;
}

int mbp_decode_batched(mbp_ctx *ctx, int32_t nbatches, const mbp_batch *batches, const mbp_params *p,
                       const mbp_tuning *tuning, void *stream) {
    int rc = check_batches("mbp_decode_batched", ctx, nbatches, batches, p, tuning);
    if (rc != MBP_OK) return rc;
    return mbp::batched_decode(ctx, nbatches, batches, p, tuning ? *tuning : mbp::default_tuning(),
                               (hipStream_t)stream);
}

int mbp_plan_create(mbp_ctx *ctx, int32_t nbatches, const mbp_batch *batches, const mbp_params *p,
                    const mbp_tuning *tuning, mbp_plan **out) {
    if (!out) return fail(MBP_EINVAL, "mbp_plan_create: out is NULL");
    *out = nullptr;
    int rc = check_batches("mbp_plan_create", ctx, nbatches, batches, p, tuning);
    if (rc != MBP_OK) return rc;
    const mbp_tuning tu = tuning ? *tuning : mbp::default_tuning();
    mbp_plan *plan = new (std::nothrow) mbp_plan();
    if (!plan) return fail(MBP_ENOMEM, "mbp_plan_create: out of host memory");
    plan->ctx = ctx;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMalloc(&plan->ws, mbp::batched_workspace_bytes(nbatches, batches, tu));
    if (e != hipSuccess) {
        delete plan;
        return hip_fail(e, "mbp_plan_create: workspace");
    }
    rc = mbp::batched_plan_capture(ctx, nbatches, batches, p, tu, plan->ws, &plan->exec, &plan->err_dev);
    if (rc != MBP_OK) {
        (void)hipFree(plan->ws);
        delete plan;
        return rc;
    }
    ctx->live_codes++;  // a plan, like a code, keeps the context record
    *out = plan;
    return MBP_OK;
}

int mbp_plan_launch(mbp_plan *plan, void *stream) {
    if (!plan) return fail(MBP_EINVAL, "mbp_plan_launch: plan is NULL");
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    return e == hipSuccess ? MBP_OK : hip_fail(e, "hipGraphLaunch");
}

int mbp_plan_wait(mbp_plan *plan, void *stream) {
    if (!plan) return fail(MBP_EINVAL, "mbp_plan_wait: plan is NULL");
    int32_t flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, plan->err_dev, sizeof(flag), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mbp_plan_wait");
    if (flag) return fail(MBP_EDEVICE, "mbp_plan_wait: a grid barrier timed out");
    return MBP_OK;
}

void mbp_plan_destroy(mbp_plan *plan) {
    if (!plan) return;
    (void)hipSetDevice(plan->ctx->device);
    (void)hipDeviceSynchronize();
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    (void)hipFree(plan->ws);
    mbp_ctx *ctx = plan->ctx;
    delete plan;
    if (--ctx->live_codes == 0 && ctx->closed) delete ctx;
}

int mbp_queue_create(mbp_ctx *ctx, const mbp_params *p, const mbp_tuning *tuning, mbp_queue **out) {
    if (!out) return fail(MBP_EINVAL, "mbp_queue_create: out is NULL");
    *out = nullptr;
    if (!ctx || !p) return fail(MBP_EINVAL, "mbp_queue_create: null ctx or params");
    // the parameter checks of a batched decode (the codes come with the batches)
    if (int rc = check_batched_params("mbp_queue_create", p); rc != MBP_OK) return rc;
    const mbp_tuning tu = tuning ? *tuning : mbp::default_tuning();
    if (int rc = mbp::check_tuning(tu); rc != MBP_OK) return rc;
    mbp_queue *q = new (std::nothrow) mbp_queue();
    if (!q) return fail(MBP_ENOMEM, "mbp_queue_create: out of host memory");
    q->ctx = ctx;
    q->params = *p;
    q->tuning = tu;
    ctx->live_codes++;  // a queue, like a code, keeps the context record
    *out = q;
    return MBP_OK;
}

int mbp_queue_submit(mbp_queue *q, int32_t nbatches, const mbp_batch *batches) {
    if (!q) return fail(MBP_EINVAL, "mbp_queue_submit: queue is NULL");
    int rc = check_batches("mbp_queue_submit", q->ctx, nbatches, batches, &q->params, nullptr);
    if (rc != MBP_OK) return rc;
    for (int32_t i = 0; i < nbatches; ++i) {
        q->pending.push_back(batches[i]);
        q->pending_frames += batches[i].nframes;
    }
    return MBP_OK;
}

int mbp_queue_flush(mbp_queue *q, void *stream) {
    if (!q) return fail(MBP_EINVAL, "mbp_queue_flush: queue is NULL");
    if (q->pending.empty()) return MBP_OK;
    const int32_t nb = static_cast<int32_t>(q->pending.size());
    int rc = check_batches("mbp_queue_flush", q->ctx, nb, q->pending.data(), &q->params, nullptr);
    if (rc != MBP_OK) return rc;
    hipError_t e = hipSetDevice(q->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    // one batched launch at a time: its blocks must all be resident together
    if (!q->flights.empty() && (e = hipStreamWaitEvent(s, q->flights.back().done, 0)) != hipSuccess)
        return hip_fail(e, "hipStreamWaitEvent");
    mbp_queue::Flight f;
    f.frames = q->pending_frames;
    if ((e = hipMalloc(&f.ws, mbp::batched_workspace_bytes(nb, q->pending.data(), q->tuning))) != hipSuccess)
        return hip_fail(e, "mbp_queue_flush: workspace");
    if ((e = hipEventCreateWithFlags(&f.done, hipEventDisableTiming)) != hipSuccess) {
        (void)hipFree(f.ws);
        return hip_fail(e, "hipEventCreate");
    }
    rc = mbp::batched_launch(q->ctx, nb, q->pending.data(), &q->params, q->tuning, f.ws, s, &f.err_dev);
    if (rc == MBP_OK && (e = hipEventRecord(f.done, s)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
    if (rc != MBP_OK) {
        (void)hipStreamSynchronize(s);
        (void)hipEventDestroy(f.done);
        (void)hipFree(f.ws);
        return rc;
    }
    q->flights.push_back(f);
    q->pending.clear();
    q->pending_frames = 0;
    return MBP_OK;
}

// Retire the completed flushes, oldest first (all of them, waiting, if `block`).
static int queue_retire(mbp_queue *q, bool block) {
    hipError_t e = hipSetDevice(q->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int rc = MBP_OK;
    size_t k = 0;
    for (; k < q->flights.size(); ++k) {
        mbp_queue::Flight &f = q->flights[k];
        e = block ? hipEventSynchronize(f.done) : hipEventQuery(f.done);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) {
            rc = hip_fail(e, "queue completion");
            break;
        }
        int32_t flag = 0;
        if ((e = hipMemcpy(&flag, f.err_dev, sizeof(flag), hipMemcpyDeviceToHost)) != hipSuccess)
            rc = hip_fail(e, "queue error flag");
        else if (flag)
            rc = fail(MBP_EDEVICE, "queue flush: a grid barrier timed out");
        (void)hipEventDestroy(f.done);
        (void)hipFree(f.ws);
        q->done_frames += f.frames;
        if (rc != MBP_OK) {
            ++k;
            break;
        }
    }
    q->flights.erase(q->flights.begin(), q->flights.begin() + static_cast<std::ptrdiff_t>(k));
    return rc;
}

int mbp_queue_poll(mbp_queue *q, int64_t *frames_done) {
    if (!q || !frames_done) return fail(MBP_EINVAL, "mbp_queue_poll: null queue or output");
    const int rc = queue_retire(q, false);
    *frames_done = q->done_frames;
    return rc;
}

int mbp_queue_wait(mbp_queue *q) {
    if (!q) return fail(MBP_EINVAL, "mbp_queue_wait: queue is NULL");
    return queue_retire(q, true);
}

void mbp_queue_destroy(mbp_queue *q) {
    if (!q) return;
    (void)queue_retire(q, true);
    for (mbp_queue::Flight &f : q->flights) {  // left by an error: wait, then free
        (void)hipEventSynchronize(f.done);
        (void)hipEventDestroy(f.done);
        (void)hipFree(f.ws);
    }
    mbp_ctx *ctx = q->ctx;
    delete q;
    if (--ctx->live_codes == 0 && ctx->closed) delete ctx;
}

// Text cache of autotuned settings: one line per batch mix,
// "<key> <rows_per_wave> <vars_per_wave> <blocks_per_cu> <schedule> <compact> <ms>".
static std::string tune_key(int32_t nb, const mbp_batch *b, const mbp_params *p) {
    std::ostringstream k;
    k << "a" << p->algo << "T" << p->max_iter << "e" << p->early_exit;
    for (int32_t i = 0; i < nb; ++i)
        k << "|n" << b[i].code->n << "M" << b[i].code->M << "E" << b[i].code->E << "u" << b[i].code->u << "f"
          << b[i].nframes;
    return k.str();
}

int mbp_autotune(mbp_ctx *ctx, int32_t nbatches, const mbp_batch *batches, const mbp_params *p,
                 const char *cache_path, mbp_tuning *out) {
    if (!out) return fail(MBP_EINVAL, "mbp_autotune: out is NULL");
    int rc = check_batches("mbp_autotune", ctx, nbatches, batches, p, nullptr);
    if (rc != MBP_OK) return rc;
    const std::string key = tune_key(nbatches, batches, p);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            mbp_tuning t{};
            double ms = 0;
            if ((ls >> k >> t.rows_per_wave >> t.vars_per_wave >> t.blocks_per_cu >> t.schedule >> t.compact >>
                 ms) &&
                k == key && mbp::check_tuning(t) == MBP_OK) {
                *out = t;
                return MBP_OK;
            }
        }
    }
    auto time_one = [&](const mbp_tuning &t, double *ms) {
        int r = mbp::batched_decode(ctx, nbatches, batches, p, t, nullptr);  // warm
        if (r != MBP_OK) return r;
        const auto t0 = std::chrono::steady_clock::now();
        r = mbp::batched_decode(ctx, nbatches, batches, p, t, nullptr);
        *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return r;
    };
    mbp_tuning best = mbp::default_tuning();
    double best_ms = 0;
    if ((rc = time_one(best, &best_ms)) != MBP_OK) return rc;
    // coordinate descent over each knob, twice
    const int rows[] = {1, 2, 4, 8}, vars[] = {1, 2, 4, 8}, bpcs[] = {1, 2, 3, 4}, binary[] = {0, 1};
    for (int pass = 0; pass < 2; ++pass) {
        for (int knob = 0; knob < 5; ++knob) {
            const int *vals = knob == 0 ? rows : knob == 1 ? vars : knob == 2 ? bpcs : binary;
            const int nv = knob <= 2 ? 4 : 2;
            for (int i = 0; i < nv; ++i) {
                mbp_tuning t = best;
                int *field = knob == 0   ? &t.rows_per_wave
                             : knob == 1 ? &t.vars_per_wave
                             : knob == 2 ? &t.blocks_per_cu
                             : knob == 3 ? &t.schedule
                                         : &t.compact;
                if (*field == vals[i]) continue;
                *field = vals[i];
                double ms = 0;
                if ((rc = time_one(t, &ms)) != MBP_OK) return rc;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
        }
    }
    *out = best;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << key << " " << best.rows_per_wave << " " << best.vars_per_wave << " " << best.blocks_per_cu << " "
          << best.schedule << " " << best.compact << " " << best_ms << "\n";
    }
    return MBP_OK;
}

int mbp_profile_enable(mbp_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(MBP_EINVAL, "mbp_profile_enable: ctx is NULL");
    if (enable < 0 || enable > MBP_PROFILE_ALL) return fail(MBP_EINVAL, "mbp_profile_enable: mask outside 0..63");
    ctx->profiling = enable;
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
