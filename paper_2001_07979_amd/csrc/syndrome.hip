// Alice's side of the reconciliation (Sec. 2, eq. (1)): the syndromes
// z^l = H_l x of every matrix for a batch of frames (mbp_syndrome).
#include <mutex>

#include "mbp_kernels.h"

// Scratch of the allocation-free syndrome call (mbp_syndrome_noalloc): the
// 64-frame key-bit words, one per variable and group, in this fixed array
// instead of the context's workspace. Each GPU the library runs on holds its
// own copy until the process ends. In host code `scratch` only names the
// array; its device address comes from hipGetSymbolAddress (scratch_setup).
static __device__ __align__(256) uint64_t scratch[mbp::kNoallocWords];

namespace mbp {
namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch;  // device address of `scratch`, per device

// One thread per (check, 64-frame group): the XOR of the group's bit words at
// the check's variables is the check's parity for all 64 frames at once (bit
// k: frame 64g + k). The bit words of a group (8 bytes per variable) stay in
// cache across the gathers. The parities go out as bytes [frame][M]; for a
// given frame the threads of a block write consecutive checks.
__global__ __launch_bounds__(kBlock) void k_syndrome(const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const uint64_t *__restrict__ xb, uint8_t *__restrict__ z,
                                                     int32_t nframes, int32_t n, int32_t M) {
    const int g = blockIdx.y;
    const int r = blockIdx.x * kBlock + static_cast<int>(threadIdx.x);
    if (r >= M) return;
    const uint64_t *xg = xb + static_cast<size_t>(g) * n;
    uint64_t par = 0;
    const int e1 = row_ptr[r + 1];
    for (int e = row_ptr[r]; e < e1; ++e) par ^= xg[col[e]];
    const int nf = min(G, nframes - g * G);
    uint8_t *zg = z + static_cast<size_t>(g) * G * M + r;
    for (int k = 0; k < nf; ++k) zg[static_cast<size_t>(k) * M] = static_cast<uint8_t>((par >> k) & 1);
}

}  // namespace

int scratch_setup(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0) return fail(MBP_EINVAL, "scratch_setup: bad device");
    if (static_cast<size_t>(device) >= g_scratch.size()) g_scratch.resize(device + 1, nullptr);
    if (g_scratch[device]) return MBP_OK;
    void *p = nullptr;
    // the caller has made `device` current: the address is that device's copy
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[device] = p;
    return MBP_OK;
}

int syndrome_noalloc_impl(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, const uint8_t *x, uint8_t *z,
                          hipStream_t stream) {
    (void)hipGetLastError();  // errors of earlier, unrelated calls are not ours
    const int32_t n = code->n, M = code->M;
    const int64_t ngroups = (nframes + G - 1) / G;
    if (ngroups * n > static_cast<int64_t>(kNoallocWords))
        return fail(MBP_EINVAL, "mbp_syndrome_noalloc: ceil(nframes / 64) * n = " + std::to_string(ngroups * n) +
                                    " bit words exceed the scratch of " + std::to_string(kNoallocWords));
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (static_cast<size_t>(ctx->device) < g_scratch.size()) ptr = g_scratch[ctx->device];
    }
    if (!ptr) return fail(MBP_ESTATE, "mbp_syndrome_noalloc: scratch of this device was not set up");
    hipError_t err = hipSetDevice(ctx->device);
    if (err != hipSuccess) return hip_fail(err, "hipSetDevice");
    uint64_t *xb = static_cast<uint64_t *>(ptr);
    // Alice's key bits as 64-frame words per variable: every word the
    // syndrome kernel reads is written here first, so nothing is cleared
    k_stage_synd<<<dim3((n + kBlock - 1) / kBlock, static_cast<unsigned>(ngroups)), kBlock, 0, stream>>>(
        x, xb, nframes, n);
    if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "k_stage_synd launch");
    k_syndrome<<<dim3((M + kBlock - 1) / kBlock, static_cast<unsigned>(ngroups)), kBlock, 0, stream>>>(
        code->d_row_ptr, code->d_col, xb, z, nframes, n, M);
    if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "k_syndrome launch");
    return MBP_OK;
}

int syndrome_impl(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, const uint8_t *x, uint8_t *z,
                  hipStream_t stream) {
    (void)hipGetLastError();  // errors of earlier, unrelated calls are not ours
    hipError_t err = hipSetDevice(ctx->device);
    if (err != hipSuccess) return hip_fail(err, "hipSetDevice");
    const int32_t n = code->n, M = code->M;
    const int32_t ngroups = (nframes + G - 1) / G;
    int rc = ensure_workspace(ctx, align_up(static_cast<size_t>(ngroups) * n * sizeof(uint64_t)));
    if (rc != MBP_OK) return rc;
    uint64_t *xb = static_cast<uint64_t *>(ctx->ws);
    // Alice's key bits as 64-frame words per variable
    k_stage_synd<<<dim3((n + kBlock - 1) / kBlock, ngroups), kBlock, 0, stream>>>(x, xb, nframes, n);
    if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "k_stage_synd launch");
    k_syndrome<<<dim3((M + kBlock - 1) / kBlock, ngroups), kBlock, 0, stream>>>(code->d_row_ptr, code->d_col, xb,
                                                                              z, nframes, n, M);
    if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "k_syndrome launch");
    // the context's workspace is free for the next call once this returns
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
    return MBP_OK;
}

}  // namespace mbp
