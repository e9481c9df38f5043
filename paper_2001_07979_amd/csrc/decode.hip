// Host-side iteration driver of the plain multi-matrix syndrome BP decode
// (mbp_decode) and the channel-LLR entry (mbp_llr_from_bits). The kernels are
// in mbp_kernels.h.
#include <type_traits>
#include <vector>

#include "mbp_kernels.h"

namespace mbp {
namespace {

template <typename T>
using CheckFn = void (*)(const int32_t *, const int32_t *, const int32_t *, const float *,
                         const uint64_t *, const uint64_t *, const T *, const T *, T *, Dims);

template <typename T, int ALGO, bool BITS = false>
CheckFn<T> check_kernel(int dmax) {
    switch (dmax) {
        case 8: return &k_check<T, ALGO, 8, BITS>;
        case 10: return &k_check<T, ALGO, 10, BITS>;
        case 16: return &k_check<T, ALGO, 16, BITS>;
        case 18: return &k_check<T, ALGO, 18, BITS>;
        case 24: return &k_check<T, ALGO, 24, BITS>;
        case 32: return &k_check<T, ALGO, 32, BITS>;
        case 34: return &k_check<T, ALGO, 34, BITS>;
        case 48: return &k_check<T, ALGO, 48, BITS>;
        default: return &k_check<T, ALGO, 64, BITS>;
    }
}

template <typename T, bool BITS = false>
CheckFn<T> check_kernel_for(int algo, int dmax) {
    return algo == MBP_ALGO_NMS ? check_kernel<T, kNMS, BITS>(dmax) : check_kernel<T, kSPA, BITS>(dmax);
}

// FP32 min-sum instances with the compressed check state (null: the slot
// count has none).
template <bool BITS>
CheckFn<float> check_kernel_state(int dmax) {
    switch (dmax) {
        case 8: return &k_check<float, kNMS, 8, BITS, true>;
        case 10: return &k_check<float, kNMS, 10, BITS, true>;
        case 16: return &k_check<float, kNMS, 16, BITS, true>;
        case 18: return &k_check<float, kNMS, 18, BITS, true>;
        case 24: return &k_check<float, kNMS, 24, BITS, true>;
        default: return nullptr;
    }
}

// FP32 instances with binary16 message storage.
template <int ALGO, bool BITS>
CheckFn<float> check_kernel_half(int dmax) {
    switch (dmax) {
        case 8: return &k_check<float, ALGO, 8, BITS, false, true>;
        case 10: return &k_check<float, ALGO, 10, BITS, false, true>;
        case 16: return &k_check<float, ALGO, 16, BITS, false, true>;
        case 18: return &k_check<float, ALGO, 18, BITS, false, true>;
        case 24: return &k_check<float, ALGO, 24, BITS, false, true>;
        case 32: return &k_check<float, ALGO, 32, BITS, false, true>;
        case 34: return &k_check<float, ALGO, 34, BITS, false, true>;
        case 48: return &k_check<float, ALGO, 48, BITS, false, true>;
        default: return &k_check<float, ALGO, 64, BITS, false, true>;
    }
}

template <bool BITS>
CheckFn<float> check_kernel_half_for(int algo, int dmax) {
    return algo == MBP_ALGO_NMS ? check_kernel_half<kNMS, BITS>(dmax) : check_kernel_half<kSPA, BITS>(dmax);
}

// FP32 instances of the second iteration after a first in closed form: the
// old messages rebuilt from the magnitude table and the sign bits.
template <int ALGO, bool H>
CheckFn<float> check_kernel_short(int dmax) {
    switch (dmax) {
        case 8: return &k_check<float, ALGO, 8, false, false, H, true>;
        case 10: return &k_check<float, ALGO, 10, false, false, H, true>;
        case 16: return &k_check<float, ALGO, 16, false, false, H, true>;
        case 18: return &k_check<float, ALGO, 18, false, false, H, true>;
        case 24: return &k_check<float, ALGO, 24, false, false, H, true>;
        case 32: return &k_check<float, ALGO, 32, false, false, H, true>;
        case 34: return &k_check<float, ALGO, 34, false, false, H, true>;
        case 48: return &k_check<float, ALGO, 48, false, false, H, true>;
        default: return &k_check<float, ALGO, 64, false, false, H, true>;
    }
}

template <bool H>
CheckFn<float> check_kernel_short_for(int algo, int dmax) {
    return algo == MBP_ALGO_NMS ? check_kernel_short<kNMS, H>(dmax) : check_kernel_short<kSPA, H>(dmax);
}

using FirstTableFn = void (*)(float *, const uint32_t *, Dims);
template <bool H>
FirstTableFn first_table_kernel(int algo) {
    return algo == MBP_ALGO_NMS ? &k_first_table<kNMS, H> : &k_first_table<kSPA, H>;
}

// The channel of a decode: LLR rows [F][n] of the decode's element type, or
// Bob's bits y [F][n] (bytes, nonzero = 1) with the error rate e [F] of each
// frame, from which lambda = (1 - 2y) ln((1 - e)/e) is formed inside the
// kernels (eq. (5)).
struct Channel {
    const void *llr;
    const uint8_t *y;
    const double *e;
};

// H: the check messages are stored as binary16 (FP32 decode, flooding,
// stacked graph; the caller has checked that).
template <typename T, bool H = false>
int run_decode(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t F,
               const Channel &ch, const uint8_t *synd, uint8_t *bits_out, int32_t *iters_out,
               uint8_t *ok_out, void *llr_out, hipStream_t stream) {
    const bool from_bits = ch.y != nullptr;
    const int32_t n = code->n, M = code->M;
    const int64_t E = code->E;
    const int32_t ngroups = (F + G - 1) / G;
    // spare groups that compaction may fill: a quarter of the groups (none
    // for a single group, which has nothing to compact)
    const int32_t nspare = p->compact && p->early_exit && ngroups >= 2 ? std::max(1, ngroups / 4) : 0;
    const int32_t ntot = ngroups + nspare;
    const size_t s = sizeof(T);
    const size_t sz_c = align_up(static_cast<size_t>(ntot) * E * G * (H ? 2 : s));
    const size_t sz_L = align_up(static_cast<size_t>(ntot) * n * G * s);
    const size_t sz_z = align_up(static_cast<size_t>(ntot) * M * sizeof(uint64_t));
    const size_t sz_d = align_up(static_cast<size_t>(ntot) * n * sizeof(uint64_t));
    const size_t sz_f = align_up(static_cast<size_t>(ntot) * G * sizeof(int32_t));
    const int dmax = dmax_for(code->max_check_deg);
    // FP32 min-sum keeps a compressed check state in place of re-reading
    // every old message (where the slot count allows one)
    const bool with_state =
        std::is_same<T, float>::value && !H && p->algo == MBP_ALGO_NMS && dmax <= kStateMaxDeg;
    const size_t sz_cs = with_state ? align_up(static_cast<size_t>(ntot) * M * kStateRows * G * sizeof(uint32_t))
                                    : 0;
    // the matrix-serial variable passes keep each matrix's sum at every
    // variable, so a pass reads only its own matrix's messages
    const bool phase_sums = p->schedule == MBP_MATRIX_SERIAL && code->u > 1 && code->u <= kPhaseMaxU;
    // independent decoders: every matrix's posterior at every variable,
    // after the stored sums in the same per-group block of rows
    const bool indep = p->coupling == MBP_INDEPENDENT;
    const int32_t lm0 = phase_sums ? code->u : 0;
    const int32_t prows = lm0 + (indep ? code->u : 0);
    const size_t sz_ps = prows ? align_up(static_cast<size_t>(ntot) * prows * n * G * s) : 0;
    // FP32 flooding with the stacked graph: the variable pass per degree
    // class (its buffer loads address a group's messages with 32-bit offsets)
    const bool per_class = std::is_same<T, float>::value && !indep && E * G * static_cast<int64_t>(sizeof(float)) < INT32_MAX;
    // From Bob's bits, FP32 flooding (one phase), the per-class variable pass
    // and no compressed state: the first iteration in closed form (its
    // messages rebuilt from a table of magnitudes and the checks' parity
    // words, never stored)
    const bool closed1 = std::is_same<T, float>::value && from_bits && per_class && !with_state &&
                         (p->schedule != MBP_MATRIX_SERIAL || code->u == 1) && code->d_var_rt != nullptr &&
                         static_cast<int64_t>(ntot) * n < INT32_MAX;
    const int32_t mrows = closed1 ? code->first_rows : 0;
    const size_t sz_sp = closed1 ? align_up(static_cast<size_t>(ntot) * M * sizeof(uint64_t)) +
                                       align_up(static_cast<size_t>(ntot) * 2 * sizeof(uint64_t)) +
                                       align_up(static_cast<size_t>(ngroups) * mrows * G * sizeof(float))
                                 : 0;
    // lambda: rows like L, or Bob's bit words and one magnitude per slot
    const size_t sz_lam = from_bits ? sz_d + align_up(static_cast<size_t>(ntot) * G * s) : sz_L;
    // status words, one 256-byte line per group, then the stopping-test counters
    const size_t sz_m = align_up(static_cast<size_t>(ntot) * kStride * sizeof(uint64_t)) + 256;
    int rc = ensure_workspace(ctx, sz_c + sz_L + sz_lam + sz_z + sz_d + 2 * sz_f + sz_m + sz_cs + sz_ps + sz_sp);
    if (rc != MBP_OK) return rc;
    if ((rc = ensure_status(ctx, ntot)) != MBP_OK) return rc;
    char *base = static_cast<char *>(ctx->ws);
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        char *at = base + off;
        off += bytes;
        return at;
    };
    T *c = reinterpret_cast<T *>(carve(sz_c));
    T *Lp = reinterpret_cast<T *>(carve(sz_L));
    T *lam = nullptr;
    uint64_t *yb = nullptr;
    T *ymag = nullptr;
    if (from_bits) {
        yb = reinterpret_cast<uint64_t *>(carve(sz_d));
        ymag = reinterpret_cast<T *>(carve(sz_lam - sz_d));
    } else {
        lam = reinterpret_cast<T *>(carve(sz_L));
    }
    uint64_t *zb = reinterpret_cast<uint64_t *>(carve(sz_z));
    uint64_t *D = reinterpret_cast<uint64_t *>(carve(sz_d));
    int32_t *fid = reinterpret_cast<int32_t *>(carve(sz_f));
    int32_t *src = reinterpret_cast<int32_t *>(carve(sz_f));
    uint64_t *words = reinterpret_cast<uint64_t *>(carve(sz_m - 256));
    StopTail *tail = reinterpret_cast<StopTail *>(carve(256));
    T *cs = with_state ? reinterpret_cast<T *>(carve(sz_cs)) : nullptr;
    T *ps = prows ? reinterpret_cast<T *>(carve(sz_ps)) : nullptr;
    T *lm = indep ? ps + static_cast<size_t>(lm0) * n * G : nullptr;
    uint64_t *spar = nullptr, *smask = nullptr;
    float *mtab = nullptr;
    if (closed1) {
        spar = reinterpret_cast<uint64_t *>(carve(align_up(static_cast<size_t>(ntot) * M * sizeof(uint64_t))));
        smask = reinterpret_cast<uint64_t *>(carve(align_up(static_cast<size_t>(ntot) * 2 * sizeof(uint64_t))));
        mtab = reinterpret_cast<float *>(carve(align_up(static_cast<size_t>(ngroups) * mrows * G * sizeof(float))));
    }

    Timer tm{ctx, stream, {}, 0};
    hipError_t err;
#define LAUNCH_OR_FAIL(which, ...)                                      \
    do {                                                                \
        err = tm.run(which, [&] { __VA_ARGS__; });                      \
        if (err != hipSuccess) return hip_fail(err, "kernel launch");   \
    } while (0)

    LAUNCH_OR_FAIL(kStaging, k_init_running<<<(ntot * G + 255) / 256, 256, 0, stream>>>(
                                 words, ctx->status_dev, tail, fid, F, ngroups, nspare));
    if (from_bits) {
        // Bob's bits as 64-frame words per variable, and |lambda| per slot
        LAUNCH_OR_FAIL(kStaging, k_stage_synd<<<dim3((n + kBlock - 1) / kBlock, ngroups), kBlock, 0, stream>>>(
                                     ch.y, yb, F, n));
        LAUNCH_OR_FAIL(kStaging, k_stage_mag<T><<<(ntot * G + kBlock - 1) / kBlock, kBlock, 0, stream>>>(
                                     ch.e, ymag, F, ntot * G));
    } else {
        // L^0 = lambda: the first check pass reads lam, so only lam is staged
        const dim3 tgrid((n + 63) / 64, ngroups);
        LAUNCH_OR_FAIL(kStaging, k_stage_llr<T><<<tgrid, kBlock, 0, stream>>>(
                                     static_cast<const T *>(ch.llr), lam, nullptr, F, n));
    }
    LAUNCH_OR_FAIL(kStaging, k_stage_synd<<<dim3((M + kBlock - 1) / kBlock, ngroups), kBlock, 0, stream>>>(
                                 synd, zb, F, M));

    CheckFn<T> kc = check_kernel_for<T>(p->algo, dmax);
    // the first iteration's first check pass starts from lambda
    CheckFn<T> kc1 = from_bits ? check_kernel_for<T, true>(p->algo, dmax) : kc;
    if constexpr (std::is_same<T, float>::value) {
        if (with_state) {
            kc = check_kernel_state<false>(dmax);
            kc1 = from_bits ? check_kernel_state<true>(dmax) : kc;
        }
        if (H) {
            kc = check_kernel_half_for<false>(p->algo, dmax);
            kc1 = from_bits ? check_kernel_half_for<true>(p->algo, dmax) : kc;
        }
    }
    // with the first iteration in closed form, the second iteration's check
    // pass rebuilds the old messages
    CheckFn<T> kc2 = kc;
    if constexpr (std::is_same<T, float>::value) {
        if (closed1) kc2 = check_kernel_short_for<H>(p->algo, dmax);
    }
    Dims dc{E, n, M, ntot, (M + kRowsPerTile - 1) / kRowsPerTile, 0, 0, p->alpha, p->llr_clip};
    int vpt = 0;
    const VarFn<T> kv = from_bits ? variable_kernel<T, true>(code->max_var_deg, &vpt)
                                  : variable_kernel<T>(code->max_var_deg, &vpt);
    Dims dv{E, n, M, ntot, (n + vpt - 1) / vpt, 0, 0, p->alpha, p->llr_clip};
    dc.live = dv.live = &tail->live;
    dc.ybits = dv.ybits = yb;
    dc.ymag = dv.ymag = ymag;
    dc.cstate = cs;
    dc.spar = dv.spar = spar;
    dc.smask = dv.smask = smask;
    dc.mtab = dv.mtab = mtab;
    dc.mrows = dv.mrows = mrows;
    dv.var_rt = code->d_var_rt;
    dv.reverse = 1;
    dv.lm = lm;
    dv.prows = prows;
    for (int32_t l = 1; l < code->u && l <= 3; ++l) dv.emat[l - 1] = static_cast<int32_t>(code->e_off[l]);
    int vpt_p = 0;
    const VarPhaseFn<T> kvp = from_bits ? variable_phase_kernel<T, true>(code->max_var_deg_matrix, &vpt_p)
                                        : variable_phase_kernel<T>(code->max_var_deg_matrix, &vpt_p);
    Dims dvs = dv;  // the matrix-serial phase passes
    dvs.ntiles = (n + vpt_p - 1) / vpt_p;
    dvs.u = code->u;
    dvs.vmptr = code->d_var_mptr;
    dvs.psum = ps;
    Dims ds{E, n, M, ntot, (M + kBlock - 1) / kBlock, 0, 0, p->alpha, p->llr_clip, p->max_iter, ngroups,
            nspare};
    ds.live = &tail->live;
    // FP32 flooding with the stacked graph: the variable pass per degree
    // class, specialised (its buffer loads address a group's messages with
    // 32-bit offsets)
    struct VarLaunch {
        VarFastFn fn;
        Dims d;
        int grid;
    };
    std::vector<VarLaunch> fast_v;
    struct VarFirstLaunch {
        VarFirstFn fn;
        Dims d;
        int grid;
    };
    std::vector<VarFirstLaunch> first_v;
    if (per_class) {
        for (const mbp_var_class &vc : code->var_classes) {
            int vpt_k = 0;
            const VarFastFn fn = from_bits ? variable_fast_kernel<true, H>(vc.dv, &vpt_k)
                                           : variable_fast_kernel<false, H>(vc.dv, &vpt_k);
            Dims d = dv;
            d.vbeg = vc.i0;
            d.vend = vc.i1;
            d.ntiles = (vc.i1 - vc.i0 + vpt_k - 1) / vpt_k;
            d.runs = code->d_var_runs;
            fast_v.push_back({fn, d, grid_for(ctx, reinterpret_cast<const void *>(fn),
                                              static_cast<int64_t>(ngroups) * d.ntiles)});
            if (closed1) {
                const VarFirstFn f1 = variable_first_kernel(vc.dv, &vpt_k);
                d.ntiles = (vc.i1 - vc.i0 + vpt_k - 1) / vpt_k;
                first_v.push_back({f1, d, grid_for(ctx, reinterpret_cast<const void *>(f1),
                                                   static_cast<int64_t>(ngroups) * d.ntiles)});
            }
        }
    }
    // binary16 messages are read by the per-class variable pass only
    if (H && fast_v.empty())
        return fail(MBP_EUNSUPPORTED, "binary16 messages: code too large for the per-class variable pass");
    // the iteration kernels index their (group, tile) work items in 32 bits
    if (static_cast<int64_t>(ntot) * std::max({dc.ntiles, dv.ntiles, dvs.ntiles}) >= INT32_MAX)
        return fail(MBP_EUNSUPPORTED, "decode: too many frame groups times tiles for one call");
    const int grid_c = grid_for(ctx, reinterpret_cast<const void *>(kc),
                                static_cast<int64_t>(ngroups) * dc.ntiles);
    const int grid_vp = grid_for(ctx, reinterpret_cast<const void *>(kvp),
                                 static_cast<int64_t>(ngroups) * dvs.ntiles);
    const int grid_v = grid_for(ctx, reinterpret_cast<const void *>(kv),
                                static_cast<int64_t>(ngroups) * dv.ntiles);
    // one block per CU at most: the test is short, and every block meets the
    // others at the last-block counter (a fence and an atomic on one word)
    const int grid_s = std::min(ctx->num_cus, grid_for(ctx, reinterpret_cast<const void *>(&k_stop_test),
                                                       static_cast<int64_t>(ntot) * ds.ntiles));
    const int grid_m = grid_for(ctx, reinterpret_cast<const void *>(&k_move<T, H>),
                                static_cast<int64_t>(std::max(nspare, 1)) * (E + 2 * n + M) / kMoveRows);

    if (ctx->poll_events.size() < 2) {
        for (size_t k = ctx->poll_events.size(); k < 2; ++k) {
            hipEvent_t e;
            if ((err = hipEventCreateWithFlags(&e, hipEventDisableTiming)) != hipSuccess)
                return hip_fail(err, "hipEventCreate");
            ctx->poll_events.push_back(e);
        }
    }

    // The check passes of one iteration: all checks at once (flooding), or
    // one pass per matrix, each followed by the variable pass (matrix-serial).
    struct Phase {
        Dims d;
        int grid;
    };
    std::vector<Phase> phases;
    if (p->schedule == MBP_MATRIX_SERIAL) {
        int32_t r0 = 0;
        for (int32_t l = 0; l < code->u; ++l) {
            Dims d = dc;
            d.row0 = r0;
            d.row1 = r0 + code->m[l];
            d.ntiles = (code->m[l] + kRowsPerTile - 1) / kRowsPerTile;
            phases.push_back({d, grid_for(ctx, reinterpret_cast<const void *>(kc),
                                          static_cast<int64_t>(ngroups) * d.ntiles)});
            r0 = d.row1;
        }
    } else {
        phases.push_back({dc, grid_c});
    }

    // Iteration t: check pass, variable pass (L^t and the decision words),
    // per phase; then, with early exit or on the last iteration, the
    // stopping test, which retires the frames whose decisions meet every
    // syndrome.
    Dims dfp = ds;  // the first iteration's parity words: one thread per check
    dfp.ybits = yb;
    dfp.ymag = ymag;
    Dims dtab = dc;  // its magnitude table, for the groups holding frames
    dtab.ngroups = ngroups;
    const int grid_fp = closed1 ? grid_for(ctx, reinterpret_cast<const void *>(&k_first_parity),
                                           static_cast<int64_t>(ntot) * dfp.ntiles)
                                : 0;
    const int grid_tab = static_cast<int>(std::min<int64_t>(
        4 * static_cast<int64_t>(ctx->num_cus), (static_cast<int64_t>(ngroups) * mrows * G + kBlock - 1) / kBlock));
    for (int32_t t = 1; t <= p->max_iter; ++t) {
        dv.t = ds.t = t;
        ds.flag = t == p->max_iter ? 1 : 0;
        const bool closed_now = closed1 && t == 1;
        if (closed_now) {
            // the first check pass in closed form: the magnitude table and the
            // checks' parity words; then the variable pass rebuilds each message
            if constexpr (std::is_same<T, float>::value) {
                LAUNCH_OR_FAIL(kFirst, first_table_kernel<H>(p->algo)<<<std::max(grid_tab, 1), kBlock, 0, stream>>>(
                                           mtab, code->d_first_rowdj, dtab));
                LAUNCH_OR_FAIL(kFirst, k_first_parity<<<grid_fp, kBlock, 0, stream>>>(
                                           code->d_row_ptr, code->d_col, zb, words, spar, smask, dfp));
                for (const VarFirstLaunch &vl : first_v) {
                    Dims dk = vl.d;
                    dk.t = t;
                    LAUNCH_OR_FAIL(kFirst, vl.fn<<<vl.grid, kBlock, 0, stream>>>(code->d_var_ptr, Lp, words, D, dk));
                }
            }
        }
        for (size_t ph = 0; ph < phases.size() && !closed_now; ++ph) {
            Dims d = phases[ph].d;
            d.t = t;
            // L^0 = lambda until the first variable pass has run; each
            // independent decoder starts from lambda in its first check pass
            const bool start = t == 1 && (ph == 0 || indep);
            const T *Lin = start ? lam : indep ? lm : Lp;
            if (indep && !start) {
                d.lstride = static_cast<int64_t>(prows) * n * G;
                d.mstride = static_cast<int64_t>(n) * G;
            }
            const bool second = closed1 && t == 2;
            const CheckFn<T> kct = start ? kc1 : second ? kc2 : kc;
            LAUNCH_OR_FAIL(second ? kSecond : kCheckNode, kct<<<phases[ph].grid, kBlock, 0, stream>>>(
                                           code->d_row_ptr, code->d_col, code->d_row_mat, nullptr, zb, words, Lin,
                                           c, c, d));
            // decision words only after the iteration's last phase
            uint64_t *Dout = ph + 1 == phases.size() ? D : nullptr;
            // in the first serial iteration only matrices 0..ph have sent
            // check messages; the others' are zero, so their edges are left out
            if (phase_sums) {
                Dims dp = dvs;
                dp.t = t;
                dp.phase = static_cast<int32_t>(ph);
                LAUNCH_OR_FAIL(kVarNode, kvp<<<grid_vp, kBlock, 0, stream>>>(
                                             code->d_var_ptr, code->d_var_edge, c, lam, Lp, words, Dout, dp));
            } else {
                // flooding, or a serial schedule of more matrices than the
                // stored sums cover: every message summed again; in the first
                // serial iteration only the matrices visited so far count
                Dims dvp = dv;
                dvp.emax = t == 1 && phases.size() > 1 ? code->e_off[ph + 1] : -1;
                if (dvp.emax < 0 && !fast_v.empty()) {
                    if constexpr (std::is_same<T, float>::value) {
                        for (const VarLaunch &vl : fast_v) {
                            Dims dk = vl.d;
                            dk.t = t;
                            LAUNCH_OR_FAIL(kVarNode, vl.fn<<<vl.grid, kBlock, 0, stream>>>(
                                                         code->d_var_ptr, code->d_var_edge, c, lam, Lp, words, Dout,
                                                         dk));
                        }
                    }
                } else {
                    LAUNCH_OR_FAIL(kVarNode, kv<<<grid_v, kBlock, 0, stream>>>(code->d_var_ptr, code->d_var_edge_f,
                                                                               c, lam, Lp, words, Dout, dvp));
                }
            }
        }
        if (!p->early_exit && t < p->max_iter) continue;
        // no compaction after a first iteration in closed form: its messages
        // exist only as the groups' tables and parity words, which stay put
        Dims dst = ds;
        if (closed_now) dst.nspare = 0;
        LAUNCH_OR_FAIL(kSyndrome, k_stop_test<<<grid_s, kBlock, 0, stream>>>(
                                      code->d_row_ptr, code->d_col, zb, D, words, ctx->status_dev,
                                      iters_out, ok_out, fid, src, tail, dst));
        // fills the spare groups the stopping test's compaction planned
        if (nspare && t <= p->max_iter - 2 && !closed_now)
            LAUNCH_OR_FAIL(kSyndrome, k_move<T, H><<<grid_m, kBlock, 0, stream>>>(
                                          c, Lp, lam, zb, yb, ymag, cs, ps, prows, src, tail, E, n, M));
        if (p->early_exit) {
            if ((err = hipEventRecord(ctx->poll_events[t & 1], stream)) != hipSuccess)
                return hip_fail(err, "hipEventRecord");
            if (t >= 2) {
                // wait for iteration t-1 while iteration t runs, then read
                // the running sets it (or a later iteration) left behind
                if ((err = hipEventSynchronize(ctx->poll_events[(t - 1) & 1])) != hipSuccess)
                    return hip_fail(err, "hipEventSynchronize");
                bool any = false;
                volatile uint64_t *st = ctx->status_host;
                for (int32_t g = 0; g < ntot && !any; ++g) any = st[g] != 0;
                if (!any) break;
            }
        }
    }
    LAUNCH_OR_FAIL(kStaging, launch_output_slots<T>(Lp, fid, bits_out, static_cast<T *>(llr_out), n, ntot,
                                                     stream));
#undef LAUNCH_OR_FAIL
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
    if ((err = tm.collect()) != hipSuccess) return hip_fail(err, "hipEventElapsedTime");
    return MBP_OK;
}

}  // namespace

int decode_impl(mbp_ctx *ctx, const mbp_code *code, const mbp_params *p, int32_t nframes,
                const void *llr, const uint8_t *y, const double *e, const uint8_t *synd, uint8_t *bits_out,
                int32_t *iters_out, uint8_t *ok_out, void *llr_out, hipStream_t stream) {
    (void)hipGetLastError();  // errors of earlier, unrelated calls are not ours
    hipError_t err = hipSetDevice(ctx->device);
    if (err != hipSuccess) return hip_fail(err, "hipSetDevice");
    const Channel ch{llr, y, e};
    if (p->dtype == MBP_F32 && p->msg_dtype == MBP_MSG_F16)
        return run_decode<float, true>(ctx, code, p, nframes, ch, synd, bits_out, iters_out, ok_out, llr_out,
                                       stream);
    if (p->dtype == MBP_F32)
        return run_decode<float>(ctx, code, p, nframes, ch, synd, bits_out, iters_out, ok_out, llr_out, stream);
    return run_decode<double>(ctx, code, p, nframes, ch, synd, bits_out, iters_out, ok_out, llr_out, stream);
}

int llr_impl(mbp_ctx *ctx, int32_t nframes, int32_t n, const uint8_t *y, const double *e,
             int32_t dtype, void *llr_out, hipStream_t stream) {
    (void)hipGetLastError();  // errors of earlier, unrelated calls are not ours
    hipError_t err = hipSetDevice(ctx->device);
    if (err != hipSuccess) return hip_fail(err, "hipSetDevice");
    constexpr int32_t kMaxGridY = 65535;
    for (int32_t f0 = 0; f0 < nframes; f0 += kMaxGridY) {
        const int32_t nf = std::min(kMaxGridY, nframes - f0);
        const dim3 grid((n + kLlrPerBlock - 1) / kLlrPerBlock, nf);
        const size_t off = static_cast<size_t>(f0) * n;
        const bool vec = n % kLlrPerThread == 0 && reinterpret_cast<uintptr_t>(y) % 8 == 0 &&
                         reinterpret_cast<uintptr_t>(llr_out) % 16 == 0;
        if (dtype == MBP_F32) {
            float *o = static_cast<float *>(llr_out) + off;
            if (vec) k_llr<float, true><<<grid, kBlock, 0, stream>>>(y + off, e + f0, o, n);
            else k_llr<float, false><<<grid, kBlock, 0, stream>>>(y + off, e + f0, o, n);
        } else {
            double *o = static_cast<double *>(llr_out) + off;
            if (vec) k_llr<double, true><<<grid, kBlock, 0, stream>>>(y + off, e + f0, o, n);
            else k_llr<double, false><<<grid, kBlock, 0, stream>>>(y + off, e + f0, o, n);
        }
    }
    err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(err, "k_llr launch");
    return MBP_OK;
}

}  // namespace mbp
