/*
 * mbp.h — C-ABI of the MI355X multi-matrix syndrome belief-propagation
 * (MBP) decoder, after Guo, Gao, Jiang and Chen, "100Mbps Reconciliation for
 * Quantum Key Distribution Using a Single Graphics Processing Unit",
 * arXiv 2001.07979.
 *
 * Bob holds u sparse parity-check matrices H_1..H_u (m_l x n) shared with
 * Alice, his sifted key frames y (n bits each) and Alice's u syndromes
 * z^l = H_l x (Sec. 2, eq. (1)). He decodes every frame by belief
 * propagation over all u matrices, forms the soft decision of eq. (2),
 * decides the bits and stops once every syndrome holds or the iteration
 * limit is reached (Sec. 2; Algorithm 1 in Sec. 3A).
 *
 * Conventions used by every call:
 *   - LLRs are ln(P(bit=0)/P(bit=1)); the decided bit is 1 iff L < 0.
 *   - The u matrices are decoded as one stacked graph [H_1; ...; H_u] with
 *     syndrome [z^1; ...; z^u] and a flooding schedule (all checks of all
 *     matrices from the previous iteration's messages, then all variables).
 *   - Pointers documented as "device" are HIP device memory (for example
 *     torch tensors on the GPU); they are borrowed: the library never frees
 *     them, and they must stay valid until the call has returned.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Every call returns MBP_OK (0) or a negative MBP_E* code, and records a
 *     message readable with mbp_last_error() on the calling thread. No call
 *     aborts or throws across the ABI.
 *   - A context belongs to one device; calls on one context must not overlap
 *     (they share its workspace).
 */
#ifndef MBP_H
#define MBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MBP_OK 0
#define MBP_EINVAL (-1)       /* bad argument */
#define MBP_ENOMEM (-2)       /* host or device allocation failed */
#define MBP_EDEVICE (-3)      /* a HIP call failed */
#define MBP_ESTATE (-4)       /* object used in the wrong state */
#define MBP_EUNSUPPORTED (-5) /* valid, but outside what this build handles */

#define MBP_ALGO_SPA 0 /* sum-product check rule, Sec. 3B eq. (6) */
#define MBP_ALGO_NMS 1 /* normalized min-sum check rule */

#define MBP_F32 0
#define MBP_F64 1

typedef struct mbp_ctx mbp_ctx;
typedef struct mbp_code mbp_code;

/* Decoder parameters.
 *   algo       MBP_ALGO_SPA: c = (-1)^z 2 atanh(prod_{other} tanh(q/2)) (eq. (6));
 *              MBP_ALGO_NMS: c = (-1)^z alpha prod_{other} sgn(q) min_{other} |q|.
 *   dtype      arithmetic and message type: MBP_F32 or MBP_F64 (llr and
 *              llr_out of mbp_decode have this element type).
 *   max_iter   iteration limit T, 1..10000 (a frame not done by T fails).
 *   early_exit 1: a frame stops at the first iteration whose decisions meet
 *              every syndrome; 0: every frame runs T iterations.
 *   alpha      min-sum normalization, finite and > 0 (ignored by SPA).
 *   llr_clip   C: variable-to-check messages are clipped to [-C, C] before
 *              the check rule; finite, > 0, and <= 30 for SPA. */
typedef struct {
    int32_t algo;
    int32_t dtype;
    int32_t max_iter;
    int32_t early_exit;
    double alpha;
    double llr_clip;
} mbp_params;

/* Message of the last failed call on this thread ("" if none). */
const char *mbp_last_error(void);

/* ABI version of this library (currently 1). */
int32_t mbp_version(void);

/* Create a context on HIP device `device`; *out receives it.
 * Errors: EINVAL (null out, bad device), EDEVICE, ENOMEM. */
int mbp_ctx_create(int32_t device, mbp_ctx **out);

/* Destroy a context and its workspace. Codes created on it must be destroyed
 * first. NULL is ignored. */
void mbp_ctx_destroy(mbp_ctx *ctx);

/* Upload u parity-check matrices (Sec. 2: u PEG matrices, m_l x n each).
 *   n          key bits per frame, 1..2^30
 *   u          number of matrices, 1..64
 *   m          [u] host: checks per matrix, >= 1
 *   row_ptr    [u] host pointers to host CSR row offsets, m_l + 1 each,
 *              row_ptr[l][0] = 0, non-decreasing
 *   col_idx    [u] host pointers to host CSR columns, ascending and unique
 *              within each row, each in [0, n)
 * The CSR arrays are copied during the call (the caller keeps them); the
 * library builds and owns the device edge layouts. Every check needs at
 * least two edges, the stacked edge count must be below 2^31, and the
 * largest check degree at most 64 (EUNSUPPORTED above that).
 * Errors: EINVAL on any violation above, ENOMEM, EDEVICE. */
int mbp_code_create(mbp_ctx *ctx, int32_t n, int32_t u, const int32_t *m,
                    const int32_t *const *row_ptr, const int32_t *const *col_idx,
                    mbp_code **out);

/* Destroy a code. NULL is ignored. */
void mbp_code_destroy(mbp_code *code);

/* Sizes of an uploaded code: key bits n, matrices u, stacked checks M =
 * sum m_l, stacked edges E, largest check degree, largest stacked variable
 * degree. Any output pointer may be NULL. */
int mbp_code_info(const mbp_code *code, int32_t *n, int32_t *u, int32_t *M, int64_t *E,
                  int32_t *max_check_deg, int32_t *max_var_deg);

/* Channel LLRs from Bob's bits and each frame's error rate (Sec. 3B,
 * eq. (5), read as P1 = e + y(1-2e), P0 = 1 - P1, giving
 * llr = (1 - 2y) ln((1-e)/e)), computed in FP64 and stored as `dtype`.
 *   y        device [nframes][n] bytes, 0 = bit 0, nonzero = bit 1
 *   e        device [nframes] FP64 error rates, each in (0, 0.5]
 *   llr_out  device [nframes][n] of dtype
 * Errors: EINVAL (sizes, null pointers, dtype). Error rates are not read on
 * the host; a value outside (0, 0.5] gives a non-finite or sign-flipped LLR. */
int mbp_llr_from_bits(mbp_ctx *ctx, int32_t nframes, int32_t n, const uint8_t *y,
                      const double *e, int32_t dtype, void *llr_out, void *stream);

/* Decode nframes frames of one code (Sec. 2; Algorithm 1).
 *   llr       device [nframes][n] channel LLRs of p->dtype, finite
 *   synd      device [nframes][M] syndrome bytes (0 / nonzero), the u
 *             syndromes of each frame back to back in matrix order
 *   bits_out  device [nframes][n] decided bits, 0/1
 *   iters_out device [nframes] iterations run (1..T)
 *   ok_out    device [nframes] 1 iff the decided bits meet every syndrome
 *   llr_out   device [nframes][n] final soft decisions L of p->dtype, or NULL
 * A frame that does not converge is not an error: ok_out = 0 and
 * iters_out = T. With early exit, iters_out is the first iteration whose
 * decisions meet every syndrome, and bits_out / llr_out are that
 * iteration's. Work is enqueued on `stream`; the call polls the device for
 * convergence, so it returns once the whole decode has completed.
 * nframes may be 0 (nothing happens) and at most 65535 * 64.
 * Errors: EINVAL (bad parameters, sizes or null pointers), ENOMEM (the
 * workspace of 4 ceil(nframes/64) 64 (E + 2n) sizeof(dtype) bytes and
 * more could not be allocated), EDEVICE. */
int mbp_decode(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes,
               const void *llr, const uint8_t *synd, uint8_t *bits_out, int32_t *iters_out,
               uint8_t *ok_out, void *llr_out, void *stream);

/* Kernel timing. When enabled, every decode brackets each launch of its
 * check-node and variable-node kernels with HIP events on the decode's
 * stream and adds the elapsed times to per-kernel totals.
 *   mbp_profile_enable  0 / 1
 *   mbp_profile_reset   zero the totals
 *   mbp_profile_get     totals of kernel `which` (0 = check-node,
 *                       1 = variable-node, 2 = syndrome-only check,
 *                       3 = staging and output transposes): launches and
 *                       summed milliseconds. */
int mbp_profile_enable(mbp_ctx *ctx, int32_t enable);
int mbp_profile_reset(mbp_ctx *ctx);
int mbp_profile_get(const mbp_ctx *ctx, int32_t which, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* MBP_H */
