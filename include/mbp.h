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
 *              the check rule; finite, > 0, and <= 30 for SPA.
 *   compact    mbp_decode with early exit, 1: when the frames still running
 *              fit into at most 3/4 of the 64-frame groups they occupy, move
 *              them (with their state) into fewer spare groups so the late
 *              iterations cost less (the workspace holds a quarter more
 *              groups); 0: never. Results are the same either way. The
 *              batched calls use mbp_tuning.compact instead.
 *   schedule   MBP_FLOODING: every check of every matrix from the previous
 *              iteration's messages, then every variable (value 0);
 *              MBP_MATRIX_SERIAL: Algorithm 1 taken literally, the matrices
 *              in turn within an iteration, each matrix's check update
 *              followed by the soft decisions (eq. (2)) before the next
 *              matrix; the stopping test follows the last matrix. mbp_decode
 *              and mbp_decode_from_bits only (the batched and unrolled calls
 *              are flooding).
 *   coupling   how the u matrices combine (Sec. 2 and eq. (2)).
 *              MBP_JOINT (value 0): one Tanner graph of the stacked
 *              matrices; a variable-to-check message is the soft decision
 *              of eq. (2) minus the message on its own edge.
 *              MBP_INDEPENDENT: each matrix runs its own decoder, as Sec. 2
 *              forms the LLRs and messages of every matrix respectively:
 *              matrix l's variable-to-check message is lambda plus matrix
 *              l's other check messages at the variable, and only the soft
 *              decision of eq. (2) (and so the decided bits and the stopping
 *              test) joins the matrices. mbp_decode and mbp_decode_from_bits
 *              only, codes of at most 4 matrices (else EUNSUPPORTED); the
 *              workspace holds another 64 g u n sizeof(dtype) bytes for each
 *              matrix's posterior at every variable.
 *   msg_dtype  storage of the check-to-variable messages between passes.
 *              MBP_MSG_F32 (value 0): the dtype itself. MBP_MSG_F16: each new
 *              message (computed in FP32) is stored rounded to the nearest
 *              binary16, ties to even, and every later read (the variable
 *              pass, the next check pass's old message) uses the stored
 *              value; soft decisions stay FP32. Half the message bytes of a
 *              pass, at binary16's precision (2^-11 relative per message):
 *              the fewer-bytes-per-edge option of Sec. 3B's memory
 *              optimisation, not a way to the FP32 results. Requires dtype
 *              MBP_F32, the flooding schedule and the joint coupling (else
 *              EUNSUPPORTED) and codes of fewer than 2^23 stacked edges (else
 *              EUNSUPPORTED at the call); mbp_decode and mbp_decode_from_bits
 *              only (the batched calls refuse it).
 *              Min-sum keeps no compressed check state in this mode.
 * Soft decisions (eq. (2)) are summed with the equation's nesting: each
 * matrix's check messages at a variable are summed first (in check order),
 * and those sums are added to the channel LLR in matrix order. */
#define MBP_FLOODING 0
#define MBP_MATRIX_SERIAL 1
#define MBP_JOINT 0
#define MBP_INDEPENDENT 1
#define MBP_MSG_F32 0
#define MBP_MSG_F16 1
typedef struct {
    int32_t algo;
    int32_t dtype;
    int32_t max_iter;
    int32_t early_exit;
    double alpha;
    double llr_clip;
    int32_t compact;
    int32_t schedule;
    int32_t coupling;
    int32_t msg_dtype;
} mbp_params;

/* Message of the last failed call on this thread ("" if none). */
const char *mbp_last_error(void);

/* ABI version of this library (currently 3: mbp_params has coupling and
   msg_dtype fields). */
int32_t mbp_version(void);

/* Create a context on HIP device `device`; *out receives it.
 * Errors: EINVAL (null out, bad device), EDEVICE, ENOMEM. */
int mbp_ctx_create(int32_t device, mbp_ctx **out);

/* Destroy a context and its workspace. Codes and plans created on it may be
 * destroyed before or after it (nothing else may use the context
 * afterwards); the context's own record is freed with the last of them.
 * NULL is ignored. */
void mbp_ctx_destroy(mbp_ctx *ctx);

/* Upload u parity-check matrices (Sec. 2: u PEG matrices, m_l x n each).
 *   n          key bits per frame, 1..2^23
 *   u          number of matrices, 1..64
 *   m          [u] host: checks per matrix, >= 1
 *   row_ptr    [u] host pointers to host CSR row offsets, m_l + 1 each,
 *              row_ptr[l][0] = 0, non-decreasing
 *   col_idx    [u] host pointers to host CSR columns, ascending and unique
 *              within each row, each in [0, n)
 * The CSR arrays are copied during the call (the caller keeps them); the
 * library builds and owns the device edge layouts. Every check needs at
 * least two edges, the stacked edge count must be below 2^31, and both the
 * largest check degree and the largest variable degree over all u matrices
 * at most 64 (EUNSUPPORTED above that).
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

/* Alice's syndromes (Sec. 2, eq. (1)): z^l = H_l x over GF(2) for every
 * matrix of the code, for nframes key frames.
 *   x         device [nframes][n] key bits, bytes (0 = bit 0, nonzero = 1)
 *   synd_out  device [nframes][M] syndrome bytes 0/1, the u syndromes of
 *             each frame back to back in matrix order (the layout
 *             mbp_decode reads)
 * The call uses the context's workspace (8 bytes per variable per 64
 * frames) and returns once the syndromes are written. nframes may be 0 and
 * at most 65535 * 64.
 * Errors: EINVAL (null pointers, sizes, a code of another context), ENOMEM,
 * EDEVICE. */
int mbp_syndrome(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, const uint8_t *x, uint8_t *synd_out,
                 void *stream);

/* mbp_syndrome for callers that cannot allocate (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * outputs, bit for bit, with no allocation and no wait. The 64-frame key-bit
 * words go to a fixed device array of 2^21 words (16 MiB per GPU, held until
 * the process ends) instead of the context's workspace, so
 * ceil(nframes / 64) * n must be at most 2^21 (else EINVAL, nothing
 * enqueued); e.g. up to 512 frames at n = 2^18 or 2048 at n = 65536.
 * The call only enqueues two kernels on `stream` and returns: x must stay
 * valid, and synd_out is written, when the stream reaches them. Every call
 * on one GPU shares that GPU's array: calls on one stream are ordered, but
 * calls that overlap on one GPU (other streams, other threads) race, and
 * the caller must order them. Arguments and other errors as mbp_syndrome;
 * ESTATE if the array's address was not found when the context was created. */
int mbp_syndrome_noalloc(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, const uint8_t *x,
                         uint8_t *synd_out, void *stream);

/* Progressive edge-growth construction of u parity-check matrices (Sec. 2:
 * the u matrices are generated by PEG, after Hu, Eleftheriou and Arnold),
 * one workgroup per matrix. Variables are taken in index order; a
 * variable's first edge goes to a check of lowest current degree; each
 * further edge goes to a lowest-degree check among those that a
 * breadth-first expansion from the variable reaches last, or, when the
 * expansion stops growing or reaches max_depth levels, among the checks it
 * never reached. Ties are broken by a hash of the seed, the edge and the
 * check (random picks in a degree bucket first), so the matrices depend only
 * on the arguments; they are not those of the host generator, which draws
 * its ties sequentially. With depth bound b >= 0 no edge closes a cycle
 * shorter than 2 (b + 2).
 *   n, m       variables and checks per matrix
 *   u          number of matrices; matrix l uses seeds[l]
 *   var_deg    host [n] variable degrees, non-decreasing, in [1, min(m, 1024)]
 *   max_depth  expansion bound in levels (< 0: unbounded)
 *   row_ptr    host [u][m + 1] out: CSR row offsets of each matrix, from 0
 *   col_idx    host [u][E] out (E = sum of var_deg): columns, ascending in
 *              each row
 * Synchronous; allocates and frees its own device memory.
 * Errors: EINVAL (sizes, degrees, null buffers, or a variable left with no
 * check for an edge), EUNSUPPORTED (a check degree would pass ceil(E/m) +
 * 32), ENOMEM, EDEVICE. */
int mbp_peg_build(mbp_ctx *ctx, int32_t n, int32_t m, int32_t u, const int32_t *var_deg, const uint64_t *seeds,
                  int32_t max_depth, int32_t *row_ptr, int32_t *col_idx);

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
 * context's workspace, about 64 g (E + 2n) sizeof(dtype) + 8 g (M + n)
 * bytes for g = ceil(nframes/64) groups, plus a quarter more groups with
 * p->compact and early exit; with the matrix-serial schedule and u <= 4,
 * another 64 g u n sizeof(dtype) for each matrix's sum at every variable;
 * with FP32 min-sum and check degrees <= 24, another 768 g M bytes of
 * compressed check state; could not be allocated), EDEVICE. */
int mbp_decode(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes,
               const void *llr, const uint8_t *synd, uint8_t *bits_out, int32_t *iters_out,
               uint8_t *ok_out, void *llr_out, void *stream);

/* mbp_decode with the channel given as Bob's bits and each frame's error
 * rate (Sec. 2 and Sec. 3B, eq. (5)) instead of LLR rows: the decoder forms
 * lambda = (1 - 2y) ln((1-e)/e) itself, exactly as mbp_llr_from_bits would
 * (ln((1-e)/e) in FP64, rounded once to p->dtype), so every output equals
 * mbp_llr_from_bits followed by mbp_decode, bit for bit. The LLRs are never
 * stored as rows: the kernels read 64-frame bit words and one magnitude per
 * frame, which saves the first iteration's LLR gathers and the LLR reads of
 * every variable pass. In FP32 with one check pass per iteration (flooding,
 * or u = 1) and no compressed min-sum state, the first iteration's messages
 * are not stored either: with every |lambda| of a frame equal, the message
 * from slot j of a check of degree d has a magnitude set by (d, j) and the
 * frame, and a sign set by the check's parity and the variable's bit, so the
 * first variable pass and the second check pass rebuild each message from a
 * small table and two bits (the same values, bit for bit). Error rates
 * outside (0, 1) give NaN outputs that may differ from the two-call path in
 * their NaN bits.
 *   y     device [nframes][n] bytes, 0 = bit 0, nonzero = bit 1
 *   e     device [nframes] FP64 error rates, each in (0, 0.5]
 * Every other argument, the output contract and the errors are those of
 * mbp_decode (the workspace holds 8 g n bytes of bit words and 64 g
 * magnitudes in place of the 64 g n LLRs; with the first iteration in
 * closed form, also 8 g M bytes of parity words and 256 g R bytes of table,
 * R = the sum of the code's distinct check degrees). Error rates are not read on the
 * host; a value outside (0, 0.5] gives non-finite or sign-flipped LLRs. */
int mbp_decode_from_bits(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes,
                         const uint8_t *y, const double *e, const uint8_t *synd, uint8_t *bits_out,
                         int32_t *iters_out, uint8_t *ok_out, void *llr_out, void *stream);

/* Unrolled normalized min-sum with a hand-written adjoint (for training the
 * min-sum weights, or any gradient through the decoder). The forward runs K
 * flooding iterations of the min-sum check rule of mbp_decode with no
 * stopping test and weight alpha[t][l] for the checks of matrix l at
 * iteration t, and returns L^K (eq. (2) after K iterations). The backward
 * returns dJ/dllr and dJ/dalpha for a given dJ/dL^K: the exact reverse of the
 * forward, with subgradients sgn' = 0, the derivative of a minimum going to
 * the smallest other edge (lowest edge position among equal values), and the
 * clip passing sgn(q) where |q| < C and 0 otherwise.
 * Only the states of every ckpt_every-th iteration are kept; the backward
 * recomputes the others segment by segment, so the result does not depend on
 * ckpt_every. FP32 throughout; results are deterministic.
 *   nframes, K     frames (>= 1, <= 65535 * 64) and iterations (1..1000)
 *   ckpt_every     1..K
 *   llr_clip       C, finite and > 0
 *   llr            device [nframes][n] f32
 *   synd           device [nframes][M] syndrome bytes (as mbp_decode)
 *   alpha          device [K][u] f32 weights
 *   llr_out        device [nframes][n] f32: L^K
 *   grad_out       device [nframes][n] f32: dJ/dL^K
 *   grad_llr       device [nframes][n] f32: dJ/dllr
 *   grad_alpha     device [K][u] f32: dJ/dalpha, summed over frames
 *   workspace      device, at least mbp_unrolled_workspace_bytes(...) bytes,
 *                  owned by the caller; the backward must get the workspace
 *                  the forward filled, unchanged, with the same inputs.
 * Both calls only enqueue work on `stream`.
 * Errors: EINVAL (sizes, pointers, K, ckpt_every, clip), EDEVICE. */
int mbp_unrolled_workspace_bytes(const mbp_code *code, int32_t nframes, int32_t K,
                                 int32_t ckpt_every, uint64_t *bytes);
int mbp_nms_unrolled_fwd(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, int32_t K,
                         int32_t ckpt_every, double llr_clip, const float *llr, const uint8_t *synd,
                         const float *alpha, float *llr_out, void *workspace,
                         uint64_t workspace_bytes, void *stream);
int mbp_nms_unrolled_bwd(mbp_ctx *ctx, const mbp_code *code, int32_t nframes, int32_t K,
                         int32_t ckpt_every, double llr_clip, const float *llr, const uint8_t *synd,
                         const float *alpha, const float *grad_out, float *grad_llr,
                         float *grad_alpha, void *workspace, uint64_t workspace_bytes,
                         void *stream);

/* Batched persistent decode of frames of several codes at once.
 *
 * Each mbp_batch is one uploaded code and its frames (the same buffers as
 * mbp_decode: llr and llr_out f32, device memory, borrowed). All batches are
 * decoded by one persistent kernel that runs every iteration itself (a grid
 * barrier between the check and variable passes, early exit when every frame
 * has stopped), so the whole decode is one launch plus staging and output
 * kernels, and can be captured into a hipGraph (mbp_plan_*). The results equal
 * mbp_decode's bit for bit for the same parameters. FP32 with the flooding
 * schedule (p->dtype = MBP_F32, p->schedule = MBP_FLOODING; EUNSUPPORTED
 * otherwise), with either check rule: normalized min-sum (MBP_ALGO_NMS) for
 * any code, or sum-product (MBP_ALGO_SPA, Sec. 3B eq. (6)) for codes whose
 * largest check degree is at most 34 (EUNSUPPORTED above that).
 *
 * mbp_tuning: work-item shape and schedule of the persistent kernel.
 *   rows_per_wave, vars_per_wave  checks / variables per wave per work item
 *                                 (1..64; 4 waves per item)
 *   blocks_per_cu                 resident blocks per compute unit (1..4)
 *   schedule                      0: item = block + k * grid (interleaved);
 *                                 1: each block takes a contiguous run
 *   compact                       1: when a batch's running frames fit into
 *                                 at most 3/4 of the groups they occupy, move
 *                                 them (with their state) into the fewest
 *                                 spare groups; 0: never (results are the
 *                                 same either way)
 * mbp_autotune times a set of tunings on the given batches (their outputs are
 * overwritten) and returns the fastest; with cache_path it first looks the
 * batch mix (with the check rule and iteration limit) up in that text file
 * and appends new results to it. */
typedef struct {
    const mbp_code *code;
    int32_t nframes;     /* 1 .. 65535 * 64 */
    const float *llr;    /* device [nframes][n] */
    const uint8_t *synd; /* device [nframes][M] */
    uint8_t *bits_out;   /* device [nframes][n] */
    int32_t *iters_out;  /* device [nframes] */
    uint8_t *ok_out;     /* device [nframes] */
    float *llr_out;      /* device [nframes][n], or NULL */
} mbp_batch;

typedef struct {
    int32_t rows_per_wave;
    int32_t vars_per_wave;
    int32_t blocks_per_cu;
    int32_t schedule;
    int32_t compact;
} mbp_tuning;

typedef struct mbp_plan mbp_plan;

int mbp_tuning_default(mbp_tuning *out);

/* Decode all batches (tuning may be NULL for the default). Uses the
 * context's workspace; returns when the decode has completed.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE (also if a grid barrier timed
 * out, which only happens if blocks could not all be resident). */
int mbp_decode_batched(mbp_ctx *ctx, int32_t nbatches, const mbp_batch *batches,
                       const mbp_params *p, const mbp_tuning *tuning, void *stream);

/* A captured hipGraph of the same decode for fixed batches: the plan owns its
 * workspace; each launch re-reads the batches' input buffers and rewrites
 * their outputs. The persistent kernel's node carries the cooperative launch
 * attribute, so each launch has all its blocks resident at once;
 * mbp_plan_create fails (EDEVICE) if the runtime refuses that attribute.
 * mbp_plan_launch only enqueues; mbp_plan_wait synchronizes the stream and
 * reports a barrier timeout of the last launch as EDEVICE. */
int mbp_plan_create(mbp_ctx *ctx, int32_t nbatches, const mbp_batch *batches, const mbp_params *p,
                    const mbp_tuning *tuning, mbp_plan **out);
int mbp_plan_launch(mbp_plan *plan, void *stream);
int mbp_plan_wait(mbp_plan *plan, void *stream);
void mbp_plan_destroy(mbp_plan *plan);

int mbp_autotune(mbp_ctx *ctx, int32_t nbatches, const mbp_batch *batches, const mbp_params *p,
                 const char *cache_path, mbp_tuning *out);

/* Serving queue over the batched decode, for callers that receive frames a
 * few at a time (the batched decode's queue of heterogeneous frames).
 *   mbp_queue_create   parameters as for mbp_decode_batched (FP32, flooding,
 *                      either check rule); tuning may be NULL for the default. The
 *                      queue keeps the context's record alive until it is
 *                      destroyed.
 *   mbp_queue_submit   append batches (descriptors are copied; the device
 *                      buffers they name are borrowed until their flush has
 *                      completed). Nothing runs yet.
 *   mbp_queue_flush    decode every batch submitted since the last flush in
 *                      one batched launch, enqueued on `stream` after the
 *                      previous flush's launch (one runs at a time: its
 *                      blocks must all be resident); allocates that launch's
 *                      workspace; returns without waiting.
 *   mbp_queue_poll     without blocking, retire the flushes that completed
 *                      (oldest first) and report how many submitted frames
 *                      have their outputs written.
 *   mbp_queue_wait     block until every flush has completed.
 *   mbp_queue_destroy  wait, then free. NULL is ignored.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE (also if a flush's grid
 * barrier timed out; its frames count as done, their outputs undefined). */
typedef struct mbp_queue mbp_queue;
int mbp_queue_create(mbp_ctx *ctx, const mbp_params *p, const mbp_tuning *tuning, mbp_queue **out);
int mbp_queue_submit(mbp_queue *q, int32_t nbatches, const mbp_batch *batches);
int mbp_queue_flush(mbp_queue *q, void *stream);
int mbp_queue_poll(mbp_queue *q, int64_t *frames_done);
int mbp_queue_wait(mbp_queue *q);
void mbp_queue_destroy(mbp_queue *q);

/* Kernel timing. Every plain decode brackets each launch of the kernels
 * selected by the mask with HIP events on the decode's stream and adds the
 * elapsed times to per-kernel totals. Kernel ids: 0 = check-node pass,
 * 1 = variable-node pass, 2 = stopping test, 3 = staging and output
 * transposes, 4 = the first iteration in closed form (decoding from Bob's
 * bits: its check parity words, magnitude table and variable pass), 5 = the
 * check pass after it (which rebuilds the first iteration's messages).
 * Events between launches cost a few microseconds each, so timing only the
 * kernel of interest disturbs the run least.
 *   mbp_profile_enable  mask: bit k times kernel id k (0 = off,
 *                       MBP_PROFILE_ALL = every kernel); EINVAL outside 0..63
 *   mbp_profile_reset   zero the totals
 *   mbp_profile_get     totals of kernel id `which`: launches and summed
 *                       milliseconds. */
#define MBP_PROFILE_ALL 0x3F
int mbp_profile_enable(mbp_ctx *ctx, int32_t enable);
int mbp_profile_reset(mbp_ctx *ctx);
int mbp_profile_get(const mbp_ctx *ctx, int32_t which, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* MBP_H */
