// Alice's side of the reconciliation (Sec. 2, eq. (1)): the syndromes
// z^l = H_l x of every matrix for a batch of frames (mbp_syndrome).
#include "mbp_kernels.h"

namespace mbp {
namespace {

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
