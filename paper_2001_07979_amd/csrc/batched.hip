// Batched persistent decode: frames of many codes (different n, rates and
// numbers of matrices) decoded by one persistent, cooperatively launched
// kernel that runs every iteration itself.
//
// Each batch is one code with its frames; its frames form 64-frame groups as
// in the plain decode (same layout, same per-group status words). The kernel
// walks rounds: the check pass of iteration t over the tiles of every live
// group of every batch, a grid barrier, the variable pass, a grid barrier;
// it stops when every group has retired (early exit) or after T iterations,
// then tests the last decisions of groups still running. Work items (group,
// tile) are spread over the blocks by a schedule the autotuner picks:
// interleaved (item = block + k * grid) or in contiguous runs per block.
//
// The check rule is normalized min-sum in FP32, evaluated in chunks of the
// check's edges so any check degree up to 64 shares one kernel: the first
// pass keeps only the two smallest magnitudes, the position of the smallest
// and the sign bits; the second pass writes every message from those.
//
// The barrier spins with a bounded wait: a block that waits longer than two
// seconds, or sees another block give up, sets an error flag and leaves, so
// the grid always drains (the host then reports a device error).
#include <cstddef>
#include <string>

#include "mbp_kernels.h"

namespace mbp {
namespace {

constexpr int kChunk = 16;  // edges of a check gathered per round trip

// Loads of data that no kernel of the decode writes (graph arrays, group
// descriptors, syndromes) through the constant address space, so uniform
// addresses become scalar loads.
template <typename T>
__device__ __forceinline__ T ldc(const T *p, int64_t i) {
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// State pointers come out of descriptors, so the compiler cannot tell they
// address global memory; these keep their accesses global (not flat) loads
// and stores, which do not tie up the scalar-load counter.
template <typename T>
__device__ __forceinline__ T ldg(const T *p, int64_t i) {
    return ((const __attribute__((address_space(1))) T *)p)[i];
}
template <typename T>
__device__ __forceinline__ void stg(T *p, int64_t i, T v) {
    ((__attribute__((address_space(1))) T *)p)[i] = v;
}

struct GroupDesc {
    const int32_t *row_ptr, *col, *var_ptr, *var_edge;
    float *c, *Lp;
    const float *lam;
    const uint64_t *zb;
    int32_t *iters_out;  // first frame of the group
    uint8_t *ok_out;
    int64_t E;
    int32_t n, M;
    int32_t cn_tiles, vn_tiles;
    int64_t cn_first, vn_first;  // first work item of the group in a round
};

static_assert(sizeof(GroupDesc) % 8 == 0, "descriptors are copied as 64-bit words");
constexpr int kCnFirstWord = offsetof(GroupDesc, cn_first) / 8;
constexpr int kVnFirstWord = offsetof(GroupDesc, vn_first) / 8;

// One descriptor, read word by word through the constant address space.
__device__ __forceinline__ GroupDesc load_desc(const GroupDesc *gd, int g) {
    GroupDesc d;
    uint64_t *dst = reinterpret_cast<uint64_t *>(&d);
    const uint64_t *src = reinterpret_cast<const uint64_t *>(gd + g);
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(GroupDesc) / 8); ++i) dst[i] = ldc(src, i);
    return d;
}

struct Barrier {
    unsigned count, gen, done, err;
    int32_t last;  // last iteration run (for the finalize kernels)
    int32_t pad[11];
};

struct PArgs {
    const GroupDesc *gd;
    uint64_t *act, *uns;  // [group][kStride]
    Barrier *bar;
    int64_t cn_items, vn_items;
    int32_t ngroups, T, early_exit;
    int32_t rows_per_wave, vars_per_wave, schedule;
    float alpha, clip;
};

// A barrier wait gives up after this long on the 100 MHz real-time clock
// (2 s); a legitimate wait is one round of work, far shorter.
constexpr uint64_t kWaitTicks = 200000000ull;
// Resident blocks per compute unit that the persistent kernel may use: well
// inside its register-limited occupancy (7 waves per SIMD, one wave of each
// block per SIMD), so every block of the grid is resident at once.
constexpr int kMaxBlocksPerCu = 4;

__device__ bool grid_sync(Barrier *b) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();  // make this block's writes visible device-wide
        const unsigned gen = __hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = atomicAdd(&b->count, 1u);
        int good = 1;
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(8);
                if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks ||
                    __hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    good = 0;
                    atomicExch(&b->err, 1u);
                    break;
                }
            }
        }
        __threadfence();
        ok = good && __hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    }
    __syncthreads();
    return ok != 0;
}

// Group of work item w (gd sorted by first item): scalar binary search.
__device__ __forceinline__ int group_of(const GroupDesc *gd, int ngroups, int64_t w, bool cn) {
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t *words = reinterpret_cast<const int64_t *>(gd + mid);
        const int64_t first = ldc(words, cn ? kCnFirstWord : kVnFirstWord);
        if (first <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The k-th work item of this block under the schedule, or -1 when done.
__device__ __forceinline__ int64_t item_at(int64_t k, int64_t total, int schedule) {
    if (schedule == 0) {
        const int64_t w = static_cast<int64_t>(blockIdx.x) + k * gridDim.x;
        return w < total ? w : -1;
    }
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    if (k >= per) return -1;
    const int64_t w = static_cast<int64_t>(blockIdx.x) * per + k;
    return w < total ? w : -1;
}

// Min-sum check pass over one tile of a group (rows rpw per wave).
__device__ void cn_tile(const GroupDesc &G_, int tile, int t, const PArgs &a, uint64_t gact,
                        uint64_t *uns_word, bool test, uint64_t *sh_bad) {
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const bool on = (gact >> lane) & 1;
    const bool first = t == 1;
    const int rpt = a.rows_per_wave * kWaves;
    uint64_t bad = 0;
    for (int k = 0; k < a.rows_per_wave; ++k) {
        const int r = tile * rpt + k * kWaves + wave;
        if (r >= G_.M) break;
        const int e0 = ldc(G_.row_ptr, r);
        const int d = ldc(G_.row_ptr, r + 1) - e0;
        const int zbit = static_cast<int>((ldc(G_.zb, r) >> lane) & 1);
        const size_t cb = static_cast<size_t>(e0) * G;
        float *cg = G_.c + cb;
        int par = 0;
        uint64_t neg = 0;
        int sx = zbit;
        float m1 = INFINITY, m2 = INFINITY;
        int i1 = 0;
        for (int j0 = 0; j0 < d; j0 += kChunk) {
            int v[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) v[j] = ldc(G_.col, e0 + j0 + j);
            if (on) {
                float Lv[kChunk], cv[kChunk];
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    if (j0 + j < d) {
                        Lv[j] = ldg(G_.Lp, static_cast<int64_t>(v[j]) * G + lane);
                        cv[j] = first ? 0.0f : ldg(cg, static_cast<int64_t>(j0 + j) * G + lane);
                    }
                }
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    if (j0 + j < d) {
                        par ^= Lv[j] < 0.0f ? 1 : 0;
                        const float q = Lv[j] - cv[j];
                        const int s = q < 0.0f ? 1 : 0;
                        sx ^= s;
                        neg |= static_cast<uint64_t>(s) << (j0 + j);
                        float aj = fabsf(q);
                        aj = aj < a.clip ? aj : a.clip;
                        if (aj < m1) {
                            m2 = m1;
                            m1 = aj;
                            i1 = j0 + j;
                        } else if (aj < m2) {
                            m2 = aj;
                        }
                    }
                }
            }
        }
        if (on) {
            const float mag1 = a.alpha * m1, mag2 = a.alpha * m2;
            for (int j = 0; j < d; ++j) {
                const float mag = j == i1 ? mag2 : mag1;
                const int s = sx ^ static_cast<int>((neg >> j) & 1);
                stg(cg, static_cast<int64_t>(j) * G + lane, s ? -mag : mag);
            }
        }
        bad |= __ballot(on && (par != zbit));
    }
    if (test) {
        if (lane == 0) sh_bad[wave] = bad;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t b = 0;
            for (int i = 0; i < kWaves; ++i) b |= sh_bad[i];
            or_unmet(uns_word, b);
        }
        __syncthreads();
    }
}

// Syndrome-only pass over one tile (stopping test of the decisions in Lp).
__device__ void syn_tile(const GroupDesc &G_, int tile, const PArgs &a, uint64_t gact,
                         uint64_t *uns_word, uint64_t *sh_bad) {
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const bool on = (gact >> lane) & 1;
    const int rpt = a.rows_per_wave * kWaves;
    uint64_t bad = 0;
    for (int k = 0; k < a.rows_per_wave; ++k) {
        const int r = tile * rpt + k * kWaves + wave;
        if (r >= G_.M) break;
        const int e0 = ldc(G_.row_ptr, r);
        const int d = ldc(G_.row_ptr, r + 1) - e0;
        const int zbit = static_cast<int>((ldc(G_.zb, r) >> lane) & 1);
        int par = 0;
        for (int j0 = 0; j0 < d; j0 += kChunk) {
            int v[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) v[j] = ldc(G_.col, e0 + j0 + j);
            if (on) {
#pragma unroll
                for (int j = 0; j < kChunk; ++j)
                    if (j0 + j < d) par ^= ldg(G_.Lp, static_cast<int64_t>(v[j]) * G + lane) < 0.0f ? 1 : 0;
            }
        }
        bad |= __ballot(on && (par != zbit));
    }
    if (lane == 0) sh_bad[wave] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t b = 0;
        for (int i = 0; i < kWaves; ++i) b |= sh_bad[i];
        or_unmet(uns_word, b);
    }
    __syncthreads();
}

// Variable pass over one tile; the tile-0 wave does the group's bookkeeping.
__device__ void vn_tile(const GroupDesc &G_, int g, int tile, int t, const PArgs &a) {
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const int pt = t & 1, nt = (t + 1) & 1;
    uint64_t *actg = a.act + static_cast<size_t>(kStride) * g;
    uint64_t *unsg = a.uns + static_cast<size_t>(kStride) * g;
    const uint64_t gact = actg[pt];
    const uint64_t U = (a.early_exit && t > 1) ? unsg[pt] : ~0ull;
    const uint64_t run = gact & U;
    if (tile == 0 && wave == 0) {
        const uint64_t conv = gact & ~U;
        if (lane == 0) {
            actg[nt] = run;
            unsg[nt] = 0;
            if (gact != 0 && run == 0) atomicAdd(&a.bar->done, 1u);
        }
        if ((conv >> lane) & 1) {
            stg(G_.iters_out, lane, t - 1);
            stg(G_.ok_out, lane, static_cast<uint8_t>(1));
        }
    }
    if (!((run >> lane) & 1)) return;
    const int vpt = a.vars_per_wave * kWaves;
    for (int k = 0; k < a.vars_per_wave; ++k) {
        const int i = tile * vpt + k * kWaves + wave;
        if (i >= G_.n) break;
        const int k0 = ldc(G_.var_ptr, i), k1 = ldc(G_.var_ptr, i + 1);
        float s = ldg(G_.lam, static_cast<int64_t>(i) * G + lane);
        for (int kk = k0; kk < k1; kk += kIdxChunk) {
            int ev[kIdxChunk];
#pragma unroll
            for (int j = 0; j < kIdxChunk; ++j) ev[j] = ldc(G_.var_edge, kk + j);
            float x[kIdxChunk];
#pragma unroll
            for (int j = 0; j < kIdxChunk; ++j)
                if (kk + j < k1) x[j] = ldg(G_.c, static_cast<int64_t>(ev[j]) * G + lane);
#pragma unroll
            for (int j = 0; j < kIdxChunk; ++j)
                if (kk + j < k1) s += x[j];
        }
        stg(G_.Lp, static_cast<int64_t>(i) * G + lane, s);
    }
}

__global__ __launch_bounds__(kBlock) void k_persistent(PArgs a) {
    __shared__ uint64_t sh_bad[kWaves];
    int32_t t = 1;
    bool alive = true;
    for (; t <= a.T && alive; ++t) {
        const int pt = t & 1;
        const bool test = a.early_exit && t > 1;
        for (int64_t k = 0;; ++k) {
            const int64_t w = item_at(k, a.cn_items, a.schedule);
            if (w < 0) break;
            const int g = group_of(a.gd, a.ngroups, w, true);
            const GroupDesc G_ = load_desc(a.gd, g);
            const uint64_t gact = a.act[static_cast<size_t>(kStride) * g + pt];
            if (gact == 0) continue;
            cn_tile(G_, static_cast<int>(w - G_.cn_first), t, a, gact,
                    a.uns + static_cast<size_t>(kStride) * g + pt, test, sh_bad);
        }
        if (!grid_sync(a.bar)) { alive = false; break; }
        for (int64_t k = 0;; ++k) {
            const int64_t w = item_at(k, a.vn_items, a.schedule);
            if (w < 0) break;
            const int g = group_of(a.gd, a.ngroups, w, false);
            const GroupDesc G_ = load_desc(a.gd, g);
            vn_tile(G_, g, static_cast<int>(w - G_.vn_first), t, a);
        }
        if (!grid_sync(a.bar)) { alive = false; break; }
        if (a.early_exit &&
            __hip_atomic_load(&a.bar->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                static_cast<unsigned>(a.ngroups)) {
            ++t;
            break;
        }
    }
    if (!alive) return;
    const int32_t last = t - 1;
    // stopping test of the last decisions for groups still running
    const int pf = (last + 1) & 1;
    for (int64_t k = 0;; ++k) {
        const int64_t w = item_at(k, a.cn_items, a.schedule);
        if (w < 0) break;
        const int g = group_of(a.gd, a.ngroups, w, true);
        const GroupDesc G_ = load_desc(a.gd, g);
        const uint64_t gact = a.act[static_cast<size_t>(kStride) * g + pf];
        if (gact == 0) continue;
        syn_tile(G_, static_cast<int>(w - G_.cn_first), a, gact, a.uns + static_cast<size_t>(kStride) * g + pf,
                 sh_bad);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.bar->last = last;
}

__global__ void k_reset_barrier(Barrier *b) {
    if (threadIdx.x == 0) {
        b->count = 0;
        b->gen = 0;
        b->done = 0;
        b->err = 0;
        b->last = 0;
    }
}

// ok / iters of frames still running after the last iteration (read from the
// barrier record, which the persistent kernel filled).
__global__ void k_finalize_last(const uint64_t *act, const uint64_t *uns, int32_t *iters_out,
                                uint8_t *ok_out, int32_t nframes, const Barrier *bar) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nframes) return;
    const int32_t last = bar->last;
    const int g = f / G, lane = f % G, p = (last + 1) & 1;
    if ((act[kStride * g + p] >> lane) & 1) {
        ok_out[f] = ((uns[kStride * g + p] >> lane) & 1) ? 0 : 1;
        iters_out[f] = last;
    }
}

__global__ void k_flag_error(const Barrier *bar, int32_t *err_out) {
    if (threadIdx.x == 0) *err_out = static_cast<int32_t>(bar->err);
}

// ------------------------------------------------------------------- host
struct BatchPlace {
    int32_t group0, ngroups;
    size_t c, Lp, lam, zb;  // byte offsets of the batch's first group
};

struct Built {
    std::vector<GroupDesc> gd;
    std::vector<BatchPlace> place;
    size_t off_gd, off_act, off_uns, off_bar, off_err, total;
    int64_t cn_items, vn_items;
    int32_t ngroups;
};

Built lay_out(int32_t nb, const mbp_batch *b, const mbp_tuning &tu) {
    Built B{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes);
        return at;
    };
    int32_t ng = 0;
    for (int32_t i = 0; i < nb; ++i) ng += (b[i].nframes + G - 1) / G;
    B.ngroups = ng;
    B.off_gd = take(sizeof(GroupDesc) * std::max(ng, 1));
    B.off_act = take(sizeof(uint64_t) * kStride * std::max(ng, 1));
    B.off_uns = take(sizeof(uint64_t) * kStride * std::max(ng, 1));
    B.off_bar = take(sizeof(Barrier));
    B.off_err = take(sizeof(int32_t));
    const int rpt = tu.rows_per_wave * kWaves, vpt = tu.vars_per_wave * kWaves;
    int64_t cn = 0, vn = 0;
    for (int32_t i = 0; i < nb; ++i) {
        const mbp_code *code = b[i].code;
        BatchPlace P{};
        P.group0 = static_cast<int32_t>(B.gd.size());
        P.ngroups = (b[i].nframes + G - 1) / G;
        // per-group strides are the ones the staging and output kernels index
        // with (g * E * G, g * n * G, g * M); each batch's region is aligned
        const size_t sc = static_cast<size_t>(code->E) * G * sizeof(float);
        const size_t sl = static_cast<size_t>(code->n) * G * sizeof(float);
        const size_t sz = static_cast<size_t>(code->M) * sizeof(uint64_t);
        P.c = take(sc * P.ngroups);
        P.Lp = take(sl * P.ngroups);
        P.lam = take(sl * P.ngroups);
        P.zb = take(sz * P.ngroups);
        for (int32_t k = 0; k < P.ngroups; ++k) {
            GroupDesc d{};
            d.row_ptr = code->d_row_ptr;
            d.col = code->d_col;
            d.var_ptr = code->d_var_ptr;
            d.var_edge = code->d_var_edge;
            // state pointers are filled in once the workspace base is known
            d.c = reinterpret_cast<float *>(P.c + k * sc);
            d.Lp = reinterpret_cast<float *>(P.Lp + k * sl);
            d.lam = reinterpret_cast<const float *>(P.lam + k * sl);
            d.zb = reinterpret_cast<const uint64_t *>(P.zb + k * sz);
            d.iters_out = b[i].iters_out + k * G;
            d.ok_out = b[i].ok_out + k * G;
            d.E = code->E;
            d.n = code->n;
            d.M = code->M;
            d.cn_tiles = (code->M + rpt - 1) / rpt;
            d.vn_tiles = (code->n + vpt - 1) / vpt;
            d.cn_first = cn;
            d.vn_first = vn;
            cn += d.cn_tiles;
            vn += d.vn_tiles;
            B.gd.push_back(d);
        }
        B.place.push_back(P);
    }
    B.cn_items = cn;
    B.vn_items = vn;
    B.total = o;
    return B;
}

void rebase(Built &B, char *base) {
    for (GroupDesc &d : B.gd) {
        d.c = reinterpret_cast<float *>(base + reinterpret_cast<size_t>(d.c));
        d.Lp = reinterpret_cast<float *>(base + reinterpret_cast<size_t>(d.Lp));
        d.lam = reinterpret_cast<const float *>(base + reinterpret_cast<size_t>(d.lam));
        d.zb = reinterpret_cast<const uint64_t *>(base + reinterpret_cast<size_t>(d.zb));
    }
}

int persistent_blocks_per_cu() {
    static int cached = 0;
    if (!cached) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_persistent),
                                                         kBlock, 0) != hipSuccess ||
            nb < 1) {
            (void)hipGetLastError();
            nb = 1;
        }
        cached = nb;
    }
    return cached;
}

// Upload the group descriptors (synchronous) after pointing them into the
// workspace at `base`.
int upload_descriptors(Built &B, char *base) {
    rebase(B, base);
    hipError_t err = hipMemcpy(base + B.off_gd, B.gd.data(), sizeof(GroupDesc) * B.gd.size(),
                               hipMemcpyHostToDevice);
    return err == hipSuccess ? MBP_OK : hip_fail(err, "descriptor upload");
}

// Enqueue the whole batched decode on `stream` (kernels only, so it can be
// captured into a graph): staging, the persistent decode, finalize, outputs.
int enqueue_kernels(mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu,
                    const Built &B, char *base, hipStream_t stream, bool cooperative) {
    uint64_t *act = reinterpret_cast<uint64_t *>(base + B.off_act);
    uint64_t *uns = reinterpret_cast<uint64_t *>(base + B.off_uns);
    Barrier *bar = reinterpret_cast<Barrier *>(base + B.off_bar);
    k_reset_barrier<<<1, 64, 0, stream>>>(bar);
    for (int32_t i = 0; i < nb; ++i) {
        const BatchPlace &P = B.place[i];
        const mbp_code *code = b[i].code;
        const int32_t F = b[i].nframes, n = code->n, M = code->M;
        k_init_groups<<<(P.ngroups + 63) / 64, 64, 0, stream>>>(act + static_cast<size_t>(kStride) * P.group0,
                                                               uns + static_cast<size_t>(kStride) * P.group0,
                                                               ctx->status_dev + P.group0, F, P.ngroups);
        float *lam = reinterpret_cast<float *>(base + P.lam), *Lp = reinterpret_cast<float *>(base + P.Lp);
        k_stage_llr<float><<<dim3((n + 63) / 64, P.ngroups), kBlock, 0, stream>>>(b[i].llr, lam, Lp, F, n);
        k_stage_synd<<<dim3((M + kBlock - 1) / kBlock, P.ngroups), kBlock, 0, stream>>>(
            b[i].synd, reinterpret_cast<uint64_t *>(base + P.zb), F, M);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(err, "batched staging launch");
    PArgs a{reinterpret_cast<const GroupDesc *>(base + B.off_gd), act, uns, bar, B.cn_items, B.vn_items,
            B.ngroups, p->max_iter, p->early_exit, tu.rows_per_wave, tu.vars_per_wave, tu.schedule,
            static_cast<float>(p->alpha), static_cast<float>(p->llr_clip)};
    const int bpc = std::max(1, std::min({tu.blocks_per_cu, persistent_blocks_per_cu(), kMaxBlocksPerCu}));
    const int grid = ctx->num_cus * bpc;
    void *args[] = {&a};
    if (cooperative)
        err = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_persistent), dim3(grid), dim3(kBlock),
                                         args, 0, stream);
    else
        err = hipLaunchKernel(reinterpret_cast<const void *>(&k_persistent), dim3(grid), dim3(kBlock), args, 0,
                              stream);
    if (err != hipSuccess) return hip_fail(err, "persistent decode launch");
    for (int32_t i = 0; i < nb; ++i) {
        const BatchPlace &P = B.place[i];
        const mbp_code *code = b[i].code;
        const int32_t F = b[i].nframes, n = code->n;
        k_finalize_last<<<(F + 255) / 256, 256, 0, stream>>>(act + static_cast<size_t>(kStride) * P.group0,
                                                            uns + static_cast<size_t>(kStride) * P.group0,
                                                            b[i].iters_out, b[i].ok_out, F, bar);
        k_output<float><<<dim3((n + 63) / 64, P.ngroups), kBlock, 0, stream>>>(
            reinterpret_cast<const float *>(base + P.Lp), b[i].bits_out, b[i].llr_out, F, n);
    }
    k_flag_error<<<1, 64, 0, stream>>>(bar, reinterpret_cast<int32_t *>(base + B.off_err));
    if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "batched output launch");
    return MBP_OK;
}

}  // namespace

mbp_tuning default_tuning() { return mbp_tuning{4, 4, 2, 0}; }

int check_tuning(const mbp_tuning &tu) {
    if (tu.rows_per_wave < 1 || tu.rows_per_wave > 64 || tu.vars_per_wave < 1 || tu.vars_per_wave > 64 ||
        tu.blocks_per_cu < 1 || tu.blocks_per_cu > kMaxBlocksPerCu || tu.schedule < 0 || tu.schedule > 1)
        return fail(MBP_EINVAL, "tuning out of range (rows/vars per wave 1..64, blocks per CU 1..4, "
                                "schedule 0..1)");
    return MBP_OK;
}

uint64_t batched_workspace_bytes(int32_t nb, const mbp_batch *b, const mbp_tuning &tu) {
    return lay_out(nb, b, tu).total;
}

int batched_decode(mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu,
                   hipStream_t stream) {
    (void)hipGetLastError();  // errors of earlier, unrelated calls are not ours
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    Built B = lay_out(nb, b, tu);
    int rc = ensure_workspace(ctx, B.total);
    if (rc == MBP_OK) rc = ensure_status(ctx, B.ngroups);
    if (rc != MBP_OK) return rc;
    char *base = static_cast<char *>(ctx->ws);
    // the previous user of the workspace may still be running on another stream
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    if ((rc = upload_descriptors(B, base)) != MBP_OK) return rc;
    if ((rc = enqueue_kernels(ctx, nb, b, p, tu, B, base, stream, true)) != MBP_OK) return rc;
    int32_t flag = 0;
    if ((e = hipMemcpyAsync(&flag, base + B.off_err, sizeof(flag), hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return hip_fail(e, "batched decode completion");
    if (flag) return fail(MBP_EDEVICE, "batched decode: a grid barrier timed out");
    return MBP_OK;
}

int batched_plan_capture(mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu,
                         void *ws, hipGraphExec_t *exec, int32_t **err_dev) {
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    Built B = lay_out(nb, b, tu);
    char *base = static_cast<char *>(ws);
    int rc = ensure_status(ctx, B.ngroups);
    if (rc == MBP_OK) rc = upload_descriptors(B, base);
    if (rc != MBP_OK) return rc;
    hipStream_t cap;
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    hipGraph_t graph = nullptr;
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = enqueue_kernels(ctx, nb, b, p, tu, B, base, cap, false);
    const hipError_t e2 = hipStreamEndCapture(cap, &graph);
    (void)hipStreamDestroy(cap);
    if (rc != MBP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *err_dev = reinterpret_cast<int32_t *>(base + B.off_err);
    return MBP_OK;
}

}  // namespace mbp
