// Unrolled normalized min-sum and its adjoint.
//
// Forward: K flooding iterations of the min-sum check rule with no stopping
// test and a weight alpha[t][l] for the checks of matrix l at iteration t
// (the plain decoder's kernels, k_check and k_variable); output L^K.
//
// Backward: the exact reverse of that forward for dJ/dL^K given, with these
// subgradients: sgn has derivative 0; a minimum passes the whole derivative to
// the smallest of the other edges (the lowest edge position among equal
// values); the cap min(|q|, C) passes sgn(q) when |q| < C and 0 otherwise.
// With q^t = L^{t-1}[v] - c^{t-1}, c^t = rule(q^t, alpha_t) and
// L^t = lambda + sum c^t over the variable's edges, one reverse step t is
//   gc^t     = gL^t[v] - gq^{t+1}                 (per edge)
//   gq^t     = adjoint of the check rule applied to gc^t
//   galpha_t = sum over edges of (-1)^z prod sgn * min * gc^t
//   gL^{t-1} = sum of gq^t over the variable's edges
// and dJ/dlambda = gL^K + ... + gL^0.
//
// Memory: the states (c^t, L^t) at every ckpt-th iteration are kept by the
// forward. The backward walks the segments from the last, recomputes each
// segment's states from its checkpoint with the forward kernels (the same
// arithmetic, so the same bits), then runs the segment's reverse steps.
#include "mbp_kernels.h"

namespace mbp {
namespace {

// Adjoint of the min-sum check rule at iteration t (a.t). a.flag = 1 at
// t = K, where no gq^{t+1} exists yet.
//   L_prev, c_prev  state t-1 (c_prev unused at t = 1)
//   gL              dJ/dL^t, [g][n][64]
//   gq              per edge: read dJ/dq^{t+1}, then overwritten with dJ/dq^t
//   galpha_row      [g][M]: dJ/dalpha_{t, l(r)} contributed by check r,
//                   summed over the lanes of group g in a fixed order
template <int DMAX>
__global__ __launch_bounds__(kBlock) void k_check_adjoint(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ row_mat, const float *__restrict__ alpha_l,
    const uint64_t *__restrict__ zb, const uint64_t *__restrict__ act,
    const float *__restrict__ L_prev, const float *__restrict__ c_prev,
    const float *__restrict__ gL, float *gq, float *__restrict__ galpha_row, const Dims a) {
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const float clip = static_cast<float>(a.clip);
    const bool first = a.t == 1, last = a.flag != 0;
    const int64_t total = static_cast<int64_t>(a.ngroups) * a.ntiles;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int g = static_cast<int>(w / a.ntiles);
        const int tile = static_cast<int>(w % a.ntiles);
        const bool on = (act[kStride * g] >> lane) & 1;
        const float *Lg = L_prev + static_cast<size_t>(g) * a.n * G;
        const float *gLg = gL + static_cast<size_t>(g) * a.n * G;
        const uint64_t *zg = zb + static_cast<size_t>(g) * a.M;
        for (int k = 0; k < kRowsPerWave; ++k) {
            const int r = tile * kRowsPerTile + k * kWaves + wave;
            if (r >= a.M) break;
            const int e0 = row_ptr[r];
            const int d = row_ptr[r + 1] - e0;
            const int zbit = static_cast<int>((zg[r] >> lane) & 1);
            const float alpha = alpha_l[row_mat[r]];
            const size_t cb = (static_cast<size_t>(g) * a.E + e0) * G;
            const float *cp = c_prev + cb;
            float *gqr = gq + cb;
            int v[DMAX];
#pragma unroll
            for (int j = 0; j < DMAX; ++j) v[j] = col[e0 + j];
            float contrib = 0.0f;
            if (on) {
                float q[DMAX], gc[DMAX];
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    if (j < d) {
                        q[j] = (Lg + static_cast<size_t>(v[j]) * G)[lane];
                        gc[j] = (gLg + static_cast<size_t>(v[j]) * G)[lane];
                    }
                }
                float co[DMAX], gn[DMAX];
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    if (j < d) {
                        co[j] = first ? 0.0f : (cp + j * G)[lane];
                        gn[j] = last ? 0.0f : (gqr + j * G)[lane];
                    }
                }
                uint64_t neg = 0;
                int sx = zbit;
                float m1 = INFINITY, m2 = INFINITY;
                int i1 = 0, i2 = 0;
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    if (j < d) {
                        q[j] -= co[j];
                        gc[j] -= gn[j];
                        const int s = q[j] < 0.0f ? 1 : 0;
                        sx ^= s;
                        neg |= static_cast<uint64_t>(s) << j;
                        float aj = fabsf(q[j]);
                        aj = aj < clip ? aj : clip;
                        if (aj < m1) {
                            m2 = m1;
                            i2 = i1;
                            m1 = aj;
                            i1 = j;
                        } else if (aj < m2) {
                            m2 = aj;
                            i2 = j;
                        }
                    }
                }
                // sigma_j = (-1)^z prod_{k != j} sgn(q_k); c_j = alpha sigma_j min_j
                float to_i1 = 0.0f, from_i1 = 0.0f, q1 = 0.0f, q2 = 0.0f;
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    if (j < d) {
                        const float sigma = (sx ^ static_cast<int>((neg >> j) & 1)) ? -1.0f : 1.0f;
                        const bool is1 = j == i1;
                        contrib += sigma * (is1 ? m2 : m1) * gc[j];
                        if (is1) {
                            from_i1 = sigma * gc[j];
                            q1 = q[j];
                        } else {
                            to_i1 += sigma * gc[j];
                        }
                        if (j == i2) q2 = q[j];
                    }
                }
                const float d1 = fabsf(q1) < clip ? (q1 < 0.0f ? -1.0f : 1.0f) : 0.0f;
                const float d2 = fabsf(q2) < clip ? (q2 < 0.0f ? -1.0f : 1.0f) : 0.0f;
                const float g1 = alpha * d1 * to_i1, g2 = alpha * d2 * from_i1;
#pragma unroll
                for (int j = 0; j < DMAX; ++j)
                    if (j < d) (gqr + j * G)[lane] = j == i1 ? g1 : (j == i2 ? g2 : 0.0f);
            }
            // fixed-order butterfly over the 64 lanes
            for (int off = 32; off >= 1; off >>= 1) contrib += __shfl_xor(contrib, off);
            if (lane == 0) galpha_row[static_cast<size_t>(g) * a.M + r] = contrib;
        }
    }
}

// dJ/dL^{t-1} = sum of dJ/dq^t over each variable's edges (in edge order);
// dJ/dlambda accumulates it.
__global__ __launch_bounds__(kBlock) void k_variable_adjoint(
    const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_edge,
    const uint64_t *__restrict__ act, const float *__restrict__ gq, float *__restrict__ gL_prev,
    float *__restrict__ glam, const Dims a) {
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const int64_t total = static_cast<int64_t>(a.ngroups) * a.ntiles;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int g = static_cast<int>(w / a.ntiles);
        const int tile = static_cast<int>(w % a.ntiles);
        if (!((act[kStride * g] >> lane) & 1)) continue;
        const size_t gb = static_cast<size_t>(g) * a.n * G;
        const float *gqg = gq + static_cast<size_t>(g) * a.E * G;
        for (int k = 0; k < kVarsPerWave; ++k) {
            const int i = tile * kVarsPerTile + k * kWaves + wave;
            if (i >= a.n) break;
            const int k0 = var_ptr[i], k1 = var_ptr[i + 1];
            float s = 0.0f;
            for (int kk = k0; kk < k1; kk += kIdxChunk) {
                int ev[kIdxChunk];
#pragma unroll
                for (int j = 0; j < kIdxChunk; ++j) ev[j] = var_edge[kk + j];
                float x[kIdxChunk];
#pragma unroll
                for (int j = 0; j < kIdxChunk; ++j)
                    if (kk + j < k1) x[j] = (gqg + static_cast<size_t>(ev[j]) * G)[lane];
#pragma unroll
                for (int j = 0; j < kIdxChunk; ++j)
                    if (kk + j < k1) s += x[j];
            }
            (gL_prev + gb + static_cast<size_t>(i) * G)[lane] = s;
            (glam + gb + static_cast<size_t>(i) * G)[lane] += s;
        }
    }
}

// dJ/dalpha[t][l] = sum over groups and the checks of matrix l of
// galpha_row[t][g][r], accumulated in FP64 in a fixed order. Block (t, l).
__global__ __launch_bounds__(kBlock) void k_alpha_reduce(const float *__restrict__ galpha_row,
                                                         const int32_t *__restrict__ mat_off,
                                                         float *__restrict__ grad_alpha, int32_t u,
                                                         int32_t M, int32_t ngroups) {
    __shared__ double part[kBlock];
    const int t = blockIdx.x, l = blockIdx.y;
    const int r0 = mat_off[l], r1 = mat_off[l + 1];
    const int64_t len = static_cast<int64_t>(r1 - r0) * ngroups;
    const float *base = galpha_row + static_cast<size_t>(t) * ngroups * M;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < len; k += kBlock) {
        const int64_t g = k / (r1 - r0), r = r0 + k % (r1 - r0);
        acc += static_cast<double>(base[g * M + r]);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s >= 1; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad_alpha[static_cast<size_t>(t) * u + l] = static_cast<float>(part[0]);
}

// Workspace carve-up (all offsets 256-byte aligned).
struct Layout {
    size_t lam, zb, act, uns, ckpt_c, ckpt_L, seg_c, seg_L, gq, gLa, gLb, glam, galpha, total;
    size_t sz_c, sz_L;
    int32_t ngroups, nckpt;
};

Layout layout(const mbp_code *code, int32_t F, int32_t K, int32_t ck) {
    Layout L{};
    L.ngroups = (F + G - 1) / G;
    L.nckpt = (K - 1) / ck;  // states at ck, 2ck, ... below K
    const size_t ng = L.ngroups;
    L.sz_c = align_up(ng * code->E * G * sizeof(float));
    L.sz_L = align_up(ng * code->n * G * sizeof(float));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes);
        return at;
    };
    L.lam = take(L.sz_L);
    L.zb = take(ng * code->M * sizeof(uint64_t));
    L.act = take(ng * kStride * sizeof(uint64_t));
    L.uns = take(ng * kStride * sizeof(uint64_t));
    L.ckpt_c = take(L.sz_c * L.nckpt);
    L.ckpt_L = take(L.sz_L * L.nckpt);
    L.seg_c = take(L.sz_c * ck);
    L.seg_L = take(L.sz_L * ck);
    L.gq = take(L.sz_c);
    L.gLa = take(L.sz_L);
    L.gLb = take(L.sz_L);
    L.glam = take(L.sz_L);
    L.galpha = take(static_cast<size_t>(K) * ng * code->M * sizeof(float));
    L.total = o;
    return L;
}

struct State {
    const float *c;  // null at t = 0 (no message yet)
    float *c_mut;
    float *L;
};

// Where state t lives: t = 0 is (no c, L = lambda); a checkpoint when t is a
// multiple of ck below K; otherwise segment slot (t - 1) mod ck.
State state_at(char *ws, const Layout &Ly, int32_t t, int32_t K, int32_t ck) {
    if (t == 0) return {nullptr, nullptr, reinterpret_cast<float *>(ws + Ly.lam)};
    if (t % ck == 0 && t < K) {
        const size_t j = t / ck - 1;
        float *c = reinterpret_cast<float *>(ws + Ly.ckpt_c + j * Ly.sz_c);
        return {c, c, reinterpret_cast<float *>(ws + Ly.ckpt_L + j * Ly.sz_L)};
    }
    const size_t j = (t - 1) % ck;
    float *c = reinterpret_cast<float *>(ws + Ly.seg_c + j * Ly.sz_c);
    return {c, c, reinterpret_cast<float *>(ws + Ly.seg_L + j * Ly.sz_L)};
}

using FwdFn = void (*)(const int32_t *, const int32_t *, const int32_t *, const float *,
                       const uint64_t *, const uint64_t *, const float *, const float *, float *, Dims);
using AdjPtr = void (*)(const int32_t *, const int32_t *, const int32_t *, const float *,
                        const uint64_t *, const uint64_t *, const float *, const float *,
                        const float *, float *, float *, Dims);

void pick(int dmax, FwdFn *f, AdjPtr *b) {
    switch (dmax) {
        case 8: *f = &k_check<float, MBP_ALGO_NMS, 8>; *b = &k_check_adjoint<8>; break;
        case 10: *f = &k_check<float, MBP_ALGO_NMS, 10>; *b = &k_check_adjoint<10>; break;
        case 16: *f = &k_check<float, MBP_ALGO_NMS, 16>; *b = &k_check_adjoint<16>; break;
        case 24: *f = &k_check<float, MBP_ALGO_NMS, 24>; *b = &k_check_adjoint<24>; break;
        case 32: *f = &k_check<float, MBP_ALGO_NMS, 32>; *b = &k_check_adjoint<32>; break;
        case 48: *f = &k_check<float, MBP_ALGO_NMS, 48>; *b = &k_check_adjoint<48>; break;
        default: *f = &k_check<float, MBP_ALGO_NMS, 64>; *b = &k_check_adjoint<64>; break;
    }
}

int dmax_of(int d) {
    for (int c : {8, 10, 16, 24, 32, 48}) if (d <= c) return c;
    return 64;
}

// Shared set-up of both directions: stage lambda and the syndromes, mark
// every frame running.
struct Run {
    mbp_ctx *ctx;
    const mbp_code *code;
    int32_t F, K, ck;
    double clip;
    const float *alpha;
    char *ws;
    Layout Ly;
    hipStream_t stream;
    FwdFn fwd;
    AdjPtr adj;
    VarFn<float> kv;
    Dims dc, dv;
    int grid_c, grid_v, grid_a;

    int setup(const float *llr, const uint8_t *synd) {
        const int32_t n = code->n, M = code->M, ng = Ly.ngroups;
        int rc = ensure_status(ctx, ng);
        if (rc != MBP_OK) return rc;
        pick(dmax_of(code->max_check_deg), &fwd, &adj);
        dc = Dims{code->E, n, M, ng, (M + kRowsPerTile - 1) / kRowsPerTile, 0, 0, 0.0, clip};
        int vpt = 0;
        kv = variable_kernel<float>(code->max_var_deg, &vpt);
        dv = Dims{code->E, n, M, ng, (n + vpt - 1) / vpt, 0, 0, 0.0, clip};
        // the iteration kernels index their (group, tile) work items in 32 bits
        if (static_cast<int64_t>(ng) * std::max(dc.ntiles, dv.ntiles) >= INT32_MAX)
            return fail(MBP_EUNSUPPORTED, "unrolled: too many frame groups times tiles for one call");
        grid_c = grid_for(ctx, reinterpret_cast<const void *>(fwd), static_cast<int64_t>(ng) * dc.ntiles);
        grid_a = grid_for(ctx, reinterpret_cast<const void *>(adj), static_cast<int64_t>(ng) * dc.ntiles);
        grid_v = grid_for(ctx, reinterpret_cast<const void *>(kv),
                          static_cast<int64_t>(ng) * dv.ntiles);
        float *lam = reinterpret_cast<float *>(ws + Ly.lam);
        uint64_t *act = reinterpret_cast<uint64_t *>(ws + Ly.act);
        uint64_t *uns = reinterpret_cast<uint64_t *>(ws + Ly.uns);
        k_init_running<<<(ng * G + 255) / 256, 256, 0, stream>>>(act, ctx->status_dev,
                                                                 reinterpret_cast<StopTail *>(uns), nullptr, F,
                                                                 ng, 0);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return hip_fail(err, "k_init_groups launch");
        // lam is staged twice into one buffer: k_stage_llr writes both outputs
        k_stage_llr<float><<<dim3((n + 63) / 64, ng), kBlock, 0, stream>>>(llr, lam, lam, F, n);
        if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "k_stage_llr launch");
        k_stage_synd<<<dim3((M + kBlock - 1) / kBlock, ng), kBlock, 0, stream>>>(
            synd, reinterpret_cast<uint64_t *>(ws + Ly.zb), F, M);
        if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "k_stage_synd launch");
        return MBP_OK;
    }

    // one forward iteration t: state t-1 -> state t
    void step(int32_t t) {
        const State a = state_at(ws, Ly, t - 1, K, ck), b = state_at(ws, Ly, t, K, ck);
        const uint64_t *act = reinterpret_cast<const uint64_t *>(ws + Ly.act);
        const uint64_t *zb = reinterpret_cast<const uint64_t *>(ws + Ly.zb);
        dc.t = t;
        dv.t = t;
        fwd<<<grid_c, kBlock, 0, stream>>>(code->d_row_ptr, code->d_col, code->d_row_mat,
                                           alpha + static_cast<size_t>(t - 1) * code->u, zb, act,
                                           a.L, a.c ? a.c : b.c, b.c_mut, dc);
        kv<<<grid_v, kBlock, 0, stream>>>(code->d_var_ptr, code->d_var_edge_f, b.c,
                                          reinterpret_cast<const float *>(ws + Ly.lam), b.L, act, nullptr, dv);
    }
};

}  // namespace

uint64_t unrolled_workspace_bytes(const mbp_code *code, int32_t nframes, int32_t K, int32_t ckpt) {
    return layout(code, nframes, K, ckpt).total;
}

int unrolled_forward(mbp_ctx *ctx, const mbp_code *code, int32_t F, int32_t K, int32_t ck,
                     double clip, const float *llr, const uint8_t *synd, const float *alpha,
                     float *llr_out, void *ws, hipStream_t stream) {
    (void)hipGetLastError();  // errors of earlier, unrelated calls are not ours
    hipError_t err = hipSetDevice(ctx->device);
    if (err != hipSuccess) return hip_fail(err, "hipSetDevice");
    Run R{ctx, code, F, K, ck, clip, alpha, static_cast<char *>(ws), layout(code, F, K, ck), stream};
    int rc = R.setup(llr, synd);
    if (rc != MBP_OK) return rc;
    for (int32_t t = 1; t <= K; ++t) R.step(t);
    if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "unrolled forward iteration launch");
    const State s = state_at(R.ws, R.Ly, K, K, ck);
    k_output<float><<<dim3((code->n + 63) / 64, R.Ly.ngroups), kBlock, 0, stream>>>(s.L, nullptr, llr_out, F,
                                                                                  code->n);
    err = hipGetLastError();
    return err == hipSuccess ? MBP_OK : hip_fail(err, "unrolled forward launch");
}

int unrolled_backward(mbp_ctx *ctx, const mbp_code *code, int32_t F, int32_t K, int32_t ck,
                      double clip, const float *llr, const uint8_t *synd, const float *alpha,
                      const float *grad_out, float *grad_llr, float *grad_alpha, void *ws,
                      hipStream_t stream) {
    (void)hipGetLastError();  // errors of earlier, unrelated calls are not ours
    hipError_t err = hipSetDevice(ctx->device);
    if (err != hipSuccess) return hip_fail(err, "hipSetDevice");
    Run R{ctx, code, F, K, ck, clip, alpha, static_cast<char *>(ws), layout(code, F, K, ck), stream};
    int rc = R.setup(llr, synd);
    if (rc != MBP_OK) return rc;
    const Layout &Ly = R.Ly;
    char *w = R.ws;
    const int32_t n = code->n, ng = Ly.ngroups;
    float *gA = reinterpret_cast<float *>(w + Ly.gLa), *gB = reinterpret_cast<float *>(w + Ly.gLb);
    float *glam = reinterpret_cast<float *>(w + Ly.glam), *gq = reinterpret_cast<float *>(w + Ly.gq);
    float *galpha = reinterpret_cast<float *>(w + Ly.galpha);
    const uint64_t *act = reinterpret_cast<const uint64_t *>(w + Ly.act);
    const uint64_t *zb = reinterpret_cast<const uint64_t *>(w + Ly.zb);
    // dJ/dL^K into gA and into the running dJ/dlambda
    k_stage_llr<float><<<dim3((n + 63) / 64, ng), kBlock, 0, stream>>>(grad_out, glam, gA, F, n);
    Dims da = R.dc;
    Dims dva = R.dv;
    dva.ntiles = (n + kVarsPerTile - 1) / kVarsPerTile;  // k_variable_adjoint's tile
    const int grid_va = grid_for(ctx, reinterpret_cast<const void *>(&k_variable_adjoint),
                                 static_cast<int64_t>(ng) * dva.ntiles);
    const int32_t nseg = (K + ck - 1) / ck;
    for (int32_t j = nseg - 1; j >= 0; --j) {
        const int32_t t0 = j * ck, t1 = std::min(t0 + ck, K);
        for (int32_t t = t0 + 1; t < t1; ++t) R.step(t);  // recompute the segment's states
        for (int32_t t = t1; t > t0; --t) {
            const State sp = state_at(w, Ly, t - 1, K, ck);
            da.t = t;
            da.flag = t == K ? 1 : 0;
            R.adj<<<R.grid_a, kBlock, 0, stream>>>(code->d_row_ptr, code->d_col, code->d_row_mat,
                                                   alpha + static_cast<size_t>(t - 1) * code->u, zb, act, sp.L,
                                                   sp.c ? sp.c : gq, gA, gq,
                                                   galpha + static_cast<size_t>(t - 1) * ng * code->M, da);
            k_variable_adjoint<<<grid_va, kBlock, 0, stream>>>(code->d_var_ptr, code->d_var_edge, act, gq, gB,
                                                                glam, dva);
            std::swap(gA, gB);
        }
    }
    k_output<float><<<dim3((n + 63) / 64, ng), kBlock, 0, stream>>>(glam, nullptr, grad_llr, F, n);
    k_alpha_reduce<<<dim3(K, code->u), kBlock, 0, stream>>>(galpha, code->d_mat_off, grad_alpha, code->u,
                                                            code->M, ng);
    err = hipGetLastError();
    return err == hipSuccess ? MBP_OK : hip_fail(err, "unrolled backward launch");
}

}  // namespace mbp
