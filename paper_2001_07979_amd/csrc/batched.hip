// Batched persistent decode: frames of many codes (different n, rates and
// numbers of matrices) decoded by one persistent, cooperatively launched
// kernel that runs every iteration itself.
//
// Each batch is one code with its frames, in 64-frame groups as in the plain
// decode (same interleaved layout). A batch owns twice its groups: the first
// half holds its frames at the start; the second half are spare groups that
// frame compaction fills. Every round of the kernel is
//   check pass t | variable pass t (L^t and decision words) | stopping test
//   of iteration t | settle (retire the frames that met every syndrome)
// with a grid barrier after each phase, and, when a batch's running frames
// fit into clearly fewer groups than they occupy, compaction: its running
// frames are gathered, with their whole state (c^t, L^t, lambda, syndrome
// bits), into the fewest spare groups, so the late iterations of frames that
// converge slowly or not at all stop dragging partly empty groups along. A
// frame's arithmetic does not depend on its slot, so the results equal the
// plain decode's bit for bit. Each slot carries the index of the frame it
// holds (-1 once vacated); iteration counts, flags and outputs go through it.
//
// Work inside a phase is spread over the blocks per live group: the tiles of
// the groups still running form one item space, which the blocks take either
// interleaved (item = block + k * grid) or in contiguous runs, as the tuning
// says; retired and unused groups cost one load.
//
// The check rule is normalized min-sum or sum-product in FP32. Min-sum is
// evaluated in chunks of the check's edges so any check degree up to 64
// shares one code path: the first pass keeps only the two smallest
// magnitudes, the position of the smallest and the sign bits; the second
// pass writes every message from those. Sum-product takes the plain check
// pass's row rule (complements of the tanh product, prefix and suffix over
// the check's slots) with the slot count of each group's code, up to
// kBatchedSpaMaxDeg edges per check, so its messages equal the plain
// decode's bit for bit too.
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

// Loads of data that no phase of the kernel writes (graph arrays, group and
// batch descriptors) through the constant address space, so uniform
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

// A word that a compaction may have rewritten earlier in this launch: a
// coherent vector load even where the address is uniform.
__device__ __forceinline__ uint64_t ld_fresh(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct GroupDesc {
    const int32_t *row_ptr, *col, *var_ptr, *var_edge;
    float *c, *Lp, *lam;
    uint64_t *zb, *D;
    int64_t E;
    int32_t n, M;
    int32_t item;  // batch of the group
    int32_t cn_tiles, vn_tiles, st_tiles;
    int32_t dslots;  // sum-product: unrolled slots of the check rule (dmax_for of the code)
    int32_t pad_;
};

static_assert(sizeof(GroupDesc) % 8 == 0, "descriptors are copied as 64-bit words");

// One descriptor, read word by word through the constant address space.
__device__ __forceinline__ GroupDesc load_desc(const GroupDesc *gd, int g) {
    GroupDesc d;
    uint64_t *dst = reinterpret_cast<uint64_t *>(&d);
    const uint64_t *src = reinterpret_cast<const uint64_t *>(gd + g);
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(GroupDesc) / 8); ++i) dst[i] = ldc(src, i);
    return d;
}

struct ItemDesc {
    int32_t *iters_out;
    uint8_t *ok_out;
    int32_t g0, ng;  // groups [g0, g0 + ng) hold the frames; [g0 + ng, g0 + 2 ng) are spare
    int32_t nframes, pad;
};

// Per-batch counters; running and live by round parity (a round writes one
// parity while the previous round's readers may still read the other).
struct ItemState {
    uint32_t running[2], live[2];  // frames / groups still running after settle
    uint32_t next_spare;           // spare groups filled so far
    uint32_t pad[3];
};

struct Barrier {
    unsigned count, gen, err;
    unsigned live[2];  // groups still running after settle, by round parity
    unsigned nnew[2];  // groups compaction filled, by round parity
    int32_t pad[9];
};

struct PArgs {
    const GroupDesc *gd;
    const ItemDesc *items;
    ItemState *ist;
    uint64_t *words;  // [group][kStride]: kRun, kUnmet
    int32_t *fid;     // [group * 64 + lane]: frame (within its batch) the slot holds, or -1
    int32_t *src;     // [group * 64 + lane]: slot a compaction moves here, or -1
    int32_t *newg;    // groups filled by the current round's compaction
    Barrier *bar;
    int32_t ngroups, nitems, T, early_exit;
    int32_t rows_per_wave, vars_per_wave, schedule, compact;
    float alpha, clip;
    int32_t algo;  // kNMS or kSPA
};

// A barrier wait gives up after this long on the 100 MHz real-time clock
// (2 s); a legitimate wait is one phase of work, far shorter.
constexpr uint64_t kWaitTicks = 200000000ull;
// Resident blocks per compute unit that the persistent kernel may use: well
// inside its register-limited occupancy (one wave of each block per SIMD),
// so every block of the grid is resident at once.
constexpr int kMaxBlocksPerCu = 4;

__device__ __forceinline__ bool grid_sync(Barrier *b) {
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

__device__ __forceinline__ uint64_t run_of(const PArgs &a, int g) {
    return ld_fresh(&a.words[static_cast<size_t>(kStride) * g + kRun]);
}

// Calls fn(g, desc, run, tile) for this block's share of the tiles of the
// groups still running; tile_field is the phase's tile count in GroupDesc.
// Schedule 0 interleaves the live item space over the blocks (item w to
// block w mod grid); schedule 1 gives each block one contiguous run of it.
template <typename Fn>
__device__ __forceinline__ void for_live_tiles(const PArgs &a, int32_t GroupDesc::*tile_field, Fn fn) {
    const int64_t grid = gridDim.x, b = blockIdx.x;
    int64_t per = 0;
    if (a.schedule == 1) {
        int64_t total = 0;
        for (int g = 0; g < a.ngroups; ++g)
            if (run_of(a, g)) total += ldc(&(a.gd[g].*tile_field), 0);
        per = (total + grid - 1) / grid;
    }
    int64_t base = 0;
    for (int g = 0; g < a.ngroups; ++g) {
        const uint64_t run = run_of(a, g);
        if (!run) continue;
        const int64_t nt = ldc(&(a.gd[g].*tile_field), 0);
        int64_t j0, j1, step;
        if (a.schedule == 0) {
            j0 = ((b - base) % grid + grid) % grid;
            j1 = nt;
            step = grid;
        } else {
            j0 = b * per - base;
            j1 = j0 + per;
            j0 = j0 < 0 ? 0 : j0;
            j1 = j1 > nt ? nt : j1;
            step = 1;
        }
        base += nt;
        if (j0 >= j1) continue;
        const GroupDesc G_ = load_desc(a.gd, g);
        for (int64_t j = j0; j < j1; j += step) fn(g, G_, run, static_cast<int>(j));
    }
}

// Min-sum check pass over one tile of a group (rows_per_wave rows per wave).
__device__ __forceinline__ void cn_tile(const GroupDesc &G_, int tile, int t, const PArgs &a, uint64_t run) {
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const bool on = (run >> lane) & 1;
    const bool first = t == 1;
    const int rpt = a.rows_per_wave * kWaves;
    for (int k = 0; k < a.rows_per_wave; ++k) {
        const int r = tile * rpt + k * kWaves + wave;
        if (r >= G_.M) break;
        const int e0 = ldc(G_.row_ptr, r);
        const int d = ldc(G_.row_ptr, r + 1) - e0;
        const int zbit = static_cast<int>((ld_fresh(G_.zb + r) >> lane) & 1);
        float *cg = G_.c + static_cast<size_t>(e0) * G;
        // the plain pass's FP32 min-sum rule (same results, bit for bit):
        // signs as IEEE sign bits (q + 0 turns -0 into +0: sgn(0) = +1),
        // the second minimum as med3(m1, a, m2)
        uint64_t neg = 0;
        uint32_t sxb = static_cast<uint32_t>(zbit) << 31;
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
                        const float q = (Lv[j] - cv[j]) + 0.0f;
                        const uint32_t qb = __float_as_uint(q);
                        sxb ^= qb;
                        neg |= static_cast<uint64_t>(qb >> 31) << (j0 + j);
                        const float aj = fminf(fabsf(q), a.clip);
                        m2 = __builtin_amdgcn_fmed3f(m1, aj, m2);
                        i1 = aj < m1 ? j0 + j : i1;
                        m1 = fminf(m1, aj);
                    }
                }
            }
        }
        if (on) {
            const float mag1 = a.alpha * m1, mag2 = a.alpha * m2;  // >= 0
            const uint32_t sx = sxb >> 31;
            for (int j = 0; j < d; ++j) {
                const float mag = j == i1 ? mag2 : mag1;
                const uint32_t sb = (sx ^ static_cast<uint32_t>((neg >> j) & 1)) << 31;
                stg(cg, static_cast<int64_t>(j) * G + lane, __uint_as_float(__float_as_uint(mag) | sb));
            }
        }
    }
}

// Sum-product check pass over one tile of a group (rows_per_wave checks per
// wave) with the plain pass's check_row_f32 and DMAX slots: all gathers of a
// check in flight, the complement prefix and suffix products in registers.
// The wave's checks form a software-pipelined stream: while a check's
// gathers are in flight it loads the next check's column indices (one
// vector load: lane j holds column j; the column array is padded past E, so
// DMAX indices are always in bounds) and the scalars of the one after (one
// per-lane gather: lanes 0-1 the row pointers, 2-3 the syndrome word). Every
// lane runs the rule (a stopped frame's slots hold stale but readable
// values) and only running frames store, so the loads stay uniform.
template <int DMAX>
__device__ __forceinline__ void spa_row(const GroupDesc &G_, int r, bool first, const PArgs &a, unsigned lane,
                                        bool on) {
    const int e0 = ldc(G_.row_ptr, r);
    const int d = ldc(G_.row_ptr, r + 1) - e0;
    const uint32_t zbit = static_cast<uint32_t>((ld_fresh(G_.zb + r) >> lane) & 1);
    int v[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) v[j] = ldc(G_.col, e0 + j);
    float *cg = G_.c + static_cast<size_t>(e0) * G;
    // default caching of the message rows (NT false)
    check_row_f32<kSPA, DMAX, false, false, false, false, false>([&v](int j) { return v[j]; }, d, zbit, a.alpha,
                                                                  a.clip, first, buf_rsrc(G_.Lp, kBufAll), cg, cg,
                                                                  lane, 0.0f, nullptr, NoPrefetch(), on);
}
template <int DMAX>
__device__ __forceinline__ void spa_tile(const GroupDesc &G_, int tile, bool first, const PArgs &a, unsigned lane,
                                         bool on) {
    const int rpt = a.rows_per_wave * kWaves;
    for (int k = 0; k < a.rows_per_wave; ++k) {
        const int r = tile * rpt + k * kWaves + wave_id();
        if (r >= G_.M) break;
        spa_row<DMAX>(G_, r, first, a, lane, on);
    }
}

// Sum-product check pass over one tile of a group; the slot count is
// uniform over the group.
__device__ __forceinline__ void cn_tile_spa(const GroupDesc &G_, int tile, int t, const PArgs &a, uint64_t run) {
    const unsigned lane = lane_id();
    const bool on = (run >> lane) & 1;
    const bool first = t == 1;
    switch (G_.dslots) {
        case 8: spa_tile<8>(G_, tile, first, a, lane, on); break;
        case 10: spa_tile<10>(G_, tile, first, a, lane, on); break;
        case 16: spa_tile<16>(G_, tile, first, a, lane, on); break;
        case 18: spa_tile<18>(G_, tile, first, a, lane, on); break;
        case 24: spa_tile<24>(G_, tile, first, a, lane, on); break;
        case 32: spa_tile<32>(G_, tile, first, a, lane, on); break;
        default: spa_tile<kBatchedSpaMaxDeg>(G_, tile, first, a, lane, on); break;
    }
}

// Variable pass over one tile: L^t (eq. (2), in edge order) and the
// decision word of each variable. A wave takes its variables two at a time
// and issues the gathers of both (kVarChunk edges each) before summing.
constexpr int kVarChunk = 16;

__device__ __forceinline__ void vn_finish(const GroupDesc &G_, int i, float s, bool on, unsigned lane) {
    if (on) stg(G_.Lp, static_cast<int64_t>(i) * G + lane, s);
    const uint64_t bits = __ballot(on && s < 0.0f);
    if (lane == 0) stg(G_.D, i, bits);
}

__device__ __forceinline__ void vn_tile(const GroupDesc &G_, int tile, const PArgs &a, uint64_t run) {
    constexpr int VC = kVarChunk;
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const bool on = (run >> lane) & 1;
    const int vpt = a.vars_per_wave * kWaves;
    for (int k = 0; k < a.vars_per_wave; k += 2) {
        const int i0 = tile * vpt + k * kWaves + wave;
        if (i0 >= G_.n) break;
        const int i1 = i0 + kWaves;
        const bool two = k + 1 < a.vars_per_wave && i1 < G_.n;
        const int p0 = ldc(G_.var_ptr, i0), q0 = ldc(G_.var_ptr, i0 + 1);
        const int p1 = two ? ldc(G_.var_ptr, i1) : 0, q1 = two ? ldc(G_.var_ptr, i1 + 1) : 0;
        // eq. (2) nested: each matrix's messages summed from 0 (a0, a1),
        // each such sum added to L in matrix order; a flagged edge (bit 31)
        // starts the next matrix's run
        float s0 = on ? ldg(G_.lam, static_cast<int64_t>(i0) * G + lane) : 0.0f;
        float s1 = on && two ? ldg(G_.lam, static_cast<int64_t>(i1) * G + lane) : 0.0f;
        float a0 = 0.0f, a1 = 0.0f;
        const int dmax = q0 - p0 > q1 - p1 ? q0 - p0 : q1 - p1;
        for (int c0 = 0; c0 < dmax; c0 += VC) {
            int e0[VC], e1[VC];
#pragma unroll
            for (int j = 0; j < VC; ++j) {
                e0[j] = ldc(G_.var_edge, p0 + c0 + j);
                e1[j] = ldc(G_.var_edge, p1 + c0 + j);
            }
            if (on) {
                float x0[VC], x1[VC];
#pragma unroll
                for (int j = 0; j < VC; ++j) {
                    if (p0 + c0 + j < q0) x0[j] = ldg(G_.c, static_cast<int64_t>(e0[j] & 0x7fffffff) * G + lane);
                    if (p1 + c0 + j < q1) x1[j] = ldg(G_.c, static_cast<int64_t>(e1[j] & 0x7fffffff) * G + lane);
                }
#pragma unroll
                for (int j = 0; j < VC; ++j) {
                    if (p0 + c0 + j < q0) {
                        if (e0[j] < 0) {
                            s0 += a0;
                            a0 = 0.0f;
                        }
                        a0 += x0[j];
                    }
                    if (p1 + c0 + j < q1) {
                        if (e1[j] < 0) {
                            s1 += a1;
                            a1 = 0.0f;
                        }
                        a1 += x1[j];
                    }
                }
            }
        }
        if (q0 > p0) s0 += a0;
        if (q1 > p1) s1 += a1;
        vn_finish(G_, i0, s0, on, lane);
        if (two) vn_finish(G_, i1, s1, on, lane);
    }
}

// Stopping test over one tile of kBlock checks: one thread per check XORs
// the check's decision words with its syndrome word; the frames whose
// parity differs are ORed into the group's kUnmet word.
__device__ __forceinline__ void st_tile(const GroupDesc &G_, int g, int tile, const PArgs &a, uint64_t run,
                        uint32_t *sh_or) {
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const int r = tile * kBlock + static_cast<int>(threadIdx.x);
    uint64_t unmet = 0;
    if (r < G_.M) {
        uint64_t par = ld_fresh(G_.zb + r);
        const int e1 = ldg(G_.row_ptr, r + 1);
        for (int e = ldg(G_.row_ptr, r); e < e1; e += kIdxChunk) {
            int v[kIdxChunk];
#pragma unroll
            for (int j = 0; j < kIdxChunk; ++j) v[j] = ldg(G_.col, e + j);
            uint64_t dw[kIdxChunk];
#pragma unroll
            for (int j = 0; j < kIdxChunk; ++j) dw[j] = e + j < e1 ? ldg(G_.D, v[j]) : 0;
#pragma unroll
            for (int j = 0; j < kIdxChunk; ++j) par ^= dw[j];
        }
        unmet = par & run;
    }
    uint32_t lo = static_cast<uint32_t>(unmet), hi = static_cast<uint32_t>(unmet >> 32);
    for (int o = 32; o > 0; o >>= 1) {
        lo |= __shfl_xor(lo, o);
        hi |= __shfl_xor(hi, o);
    }
    if (lane == 0) {
        sh_or[2 * wave] = lo;
        sh_or[2 * wave + 1] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t bits = 0;
        for (int i = 0; i < kWaves; ++i)
            bits |= static_cast<uint64_t>(sh_or[2 * i]) | (static_cast<uint64_t>(sh_or[2 * i + 1]) << 32);
        or_unmet(&a.words[static_cast<size_t>(kStride) * g + kUnmet], bits);
    }
    __syncthreads();
}

// Settle of round t for one group (one wave): frames with no unmet check
// stop at t with ok = 1; on the last iteration the others stop with ok = 0.
__device__ __forceinline__ void settle_group(const PArgs &a, int g, int t, int par) {
    const unsigned lane = lane_id();
    uint64_t *w = a.words + static_cast<size_t>(kStride) * g;
    const uint64_t run = ld_fresh(&w[kRun]);
    if (!run) return;
    const uint64_t un = ld_fresh(&w[kUnmet]);
    const bool last = t == a.T;
    const uint64_t next = last ? 0 : (run & un);
    const int item = ldc(&a.gd[g].item, 0);
    if (((run & ~next) >> lane) & 1) {
        const int f = a.fid[static_cast<size_t>(g) * G + lane];
        stg(ldc(&a.items[item].iters_out, 0), f, static_cast<int32_t>(t));
        stg(ldc(&a.items[item].ok_out, 0), f, static_cast<uint8_t>(((un >> lane) & 1) ? 0 : 1));
    }
    if (lane == 0) {
        w[kRun] = next;
        w[kUnmet] = 0;
        if (next) {
            atomicAdd(&a.ist[item].running[par], static_cast<unsigned>(__popcll(next)));
            atomicAdd(&a.ist[item].live[par], 1u);
            atomicAdd(&a.bar->live[par], 1u);
        }
    }
}

// Whether batch i compacts after round t: its running frames fit into at
// most three quarters of the groups they occupy, enough spare groups remain,
// and at least two iterations remain to profit from it. *K = groups needed.
__device__ __forceinline__ bool wants_compaction(const PArgs &a, int i, int t, int par, int *K) {
    if (!a.compact || t > a.T - 2) return false;
    ItemState *s = a.ist + i;
    const uint32_t R = __hip_atomic_load(&s->running[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t L = __hip_atomic_load(&s->live[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t used = __hip_atomic_load(&s->next_spare, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t ng = static_cast<uint32_t>(ldc(&a.items[i].ng, 0));
    const uint32_t k = (R + G - 1) / G;
    *K = static_cast<int>(k);
    return L >= 2 && 4 * k <= 3 * L && used + k <= ng;
}

// Compaction plan of batch i (one block): the running frames of its groups,
// in group and lane order, go to consecutive slots of K fresh spare groups;
// their old groups stop running.
__device__ __forceinline__ void plan_compaction(const PArgs &a, int i, int K, int par) {
    __shared__ uint32_t scan[kBlock];
    __shared__ uint32_t sh_base;
    const int g0 = ldc(&a.items[i].g0, 0), ng = ldc(&a.items[i].ng, 0);
    ItemState *s = a.ist + i;
    const uint32_t used = __hip_atomic_load(&s->next_spare, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int first_new = g0 + ng + static_cast<int>(used);
    const int ncand = ng + static_cast<int>(used);  // the originals and the spares filled so far
    if (threadIdx.x == 0) sh_base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < ncand; c0 += kBlock) {
        const int ci = c0 + static_cast<int>(threadIdx.x);
        const int g = g0 + ci;
        const uint64_t run = ci < ncand ? run_of(a, g) : 0;
        const uint32_t cnt = static_cast<uint32_t>(__popcll(run));
        scan[threadIdx.x] = cnt;
        __syncthreads();
        for (int o = 1; o < kBlock; o <<= 1) {  // inclusive scan
            const uint32_t v = threadIdx.x >= static_cast<unsigned>(o) ? scan[threadIdx.x - o] : 0;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        uint32_t k = sh_base + scan[threadIdx.x] - cnt;
        const uint32_t room = static_cast<uint32_t>(K) * G;  // equals the frames counted at settle
        for (uint64_t r = run; r && k < room; r &= r - 1) {
            const int l = __ffsll(static_cast<unsigned long long>(r)) - 1;
            const size_t from = static_cast<size_t>(g) * G + l;
            const size_t to = static_cast<size_t>(first_new) * G + k;
            a.src[to] = static_cast<int32_t>(from);
            a.fid[to] = a.fid[from];
            a.fid[from] = -1;
            ++k;
        }
        if (run) a.words[static_cast<size_t>(kStride) * g + kRun] = 0;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) sh_base += scan[kBlock - 1];
        __syncthreads();
    }
    const uint32_t R = sh_base;
    for (int j = threadIdx.x; j < K * G; j += kBlock)
        if (static_cast<uint32_t>(j) >= R) a.src[static_cast<size_t>(first_new) * G + j] = -1;
    for (int j = threadIdx.x; j < K; j += kBlock) {
        const uint32_t lo = static_cast<uint32_t>(j) * G;
        const uint32_t cnt = R - lo >= static_cast<uint32_t>(G) ? G : R - lo;
        const uint64_t mask = cnt >= static_cast<uint32_t>(G) ? ~0ull : ((1ull << cnt) - 1ull);
        uint64_t *w = a.words + static_cast<size_t>(kStride) * (first_new + j);
        w[kRun] = mask;
        w[kUnmet] = 0;
        const unsigned at = atomicAdd(&a.bar->nnew[par], 1u);
        a.newg[at] = first_new + j;
    }
    if (threadIdx.x == 0) s->next_spare = used + static_cast<uint32_t>(K);
}

// Work items per group a compaction fills; each covers a contiguous share
// of the group's rows, which its waves take in runs of kMovePerWave with all
// loads of a run issued before its stores.
constexpr int kBatchMovePieces = 1024;

// Fills piece p of a group a compaction filled: rows of c (E), L and lambda
// (n each) and syndrome words (M), each lane from its source slot.
__device__ __forceinline__ void move_piece(const PArgs &a, int g, int p) {
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const GroupDesc G_ = load_desc(a.gd, g);
    const int32_t s = a.src[static_cast<size_t>(g) * G + lane];
    const bool has = s >= 0;
    const int sg = has ? s / G : g, sl = has ? s % G : 0;
    const float *sc = ldg(&a.gd[sg].c, 0), *sL = ldg(&a.gd[sg].Lp, 0), *slam = ldg(&a.gd[sg].lam, 0);
    const uint64_t *szb = ldg(&a.gd[sg].zb, 0);
    auto span = [&](int64_t rows, int64_t *r0, int64_t *r1) {
        const int64_t per = (rows + kBatchMovePieces - 1) / kBatchMovePieces;
        *r0 = p * per;
        *r1 = *r0 + per < rows ? *r0 + per : rows;
    };
    constexpr int R = kMovePerWave;
    int64_t r0, r1;
    span(G_.E, &r0, &r1);
    for (int64_t rb = r0 + wave * R; rb < r1; rb += kWaves * R) {
        float v[R];
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (has && rb + j < r1) v[j] = ldg(sc, (rb + j) * G + sl);
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (has && rb + j < r1) stg(G_.c, (rb + j) * G + lane, v[j]);
    }
    span(G_.n, &r0, &r1);
    for (int64_t rb = r0 + wave * R; rb < r1; rb += kWaves * R) {
        float v[R], u[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (has && rb + j < r1) {
                v[j] = ldg(sL, (rb + j) * G + sl);
                u[j] = ldg(slam, (rb + j) * G + sl);
            }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (has && rb + j < r1) {
                stg(G_.Lp, (rb + j) * G + lane, v[j]);
                stg(G_.lam, (rb + j) * G + lane, u[j]);
            }
        }
    }
    span(G_.M, &r0, &r1);
    for (int64_t rb = r0 + wave * R; rb < r1; rb += kWaves * R) {
        uint64_t v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = has && rb + j < r1 ? ld_fresh(szb + rb + j) : 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const uint64_t bits = __ballot((v[j] >> sl) & 1);
            if (lane == 0 && rb + j < r1) stg(G_.zb, rb + j, bits);
        }
    }
}

// The decode, one instance per check rule (one kernel each below).
template <int ALGO>
__device__ __forceinline__ void persistent_body(PArgs a) {
    __shared__ uint32_t sh_or[2 * kWaves];
    for (int t = 1; t <= a.T; ++t) {
        const int par = t & 1;
        // clear the next round's counters (their readers finished in round t-1)
        if (blockIdx.x == 0) {
            for (int i = threadIdx.x; i < a.nitems; i += kBlock) {
                a.ist[i].running[par ^ 1] = 0;
                a.ist[i].live[par ^ 1] = 0;
            }
            if (threadIdx.x == 0) {
                a.bar->live[par ^ 1] = 0;
                a.bar->nnew[par ^ 1] = 0;
            }
        }
        for_live_tiles(a, &GroupDesc::cn_tiles, [&](int, const GroupDesc &G_, uint64_t run, int tile) {
                      if constexpr (ALGO == kSPA)
                          cn_tile_spa(G_, tile, t, a, run);
                      else
                          cn_tile(G_, tile, t, a, run);
                  });
        if (!grid_sync(a.bar)) return;
        for_live_tiles(a, &GroupDesc::vn_tiles, [&](int, const GroupDesc &G_, uint64_t run, int tile) { vn_tile(G_, tile, a, run); });
        if (!grid_sync(a.bar)) return;
        if (!a.early_exit && t < a.T) continue;
        for_live_tiles(a, &GroupDesc::st_tiles, [&](int g, const GroupDesc &G_, uint64_t run, int tile) {
                      st_tile(G_, g, tile, a, run, sh_or);
                  });
        if (!grid_sync(a.bar)) return;
        for (int g = blockIdx.x * kWaves + wave_id(); g < a.ngroups; g += gridDim.x * kWaves)
            settle_group(a, g, t, par);
        if (!grid_sync(a.bar)) return;
        if (__hip_atomic_load(&a.bar->live[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
        for (int i = blockIdx.x; i < a.nitems; i += gridDim.x) {
            int K = 0;
            if (wants_compaction(a, i, t, par, &K)) plan_compaction(a, i, K, par);
        }
        if (!grid_sync(a.bar)) return;
        const unsigned nnew =
            __hip_atomic_load(&a.bar->nnew[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (nnew == 0) continue;
        for (int64_t w = blockIdx.x; w < static_cast<int64_t>(nnew) * kBatchMovePieces; w += gridDim.x)
            move_piece(a, a.newg[w / kBatchMovePieces], static_cast<int>(w % kBatchMovePieces));
        if (!grid_sync(a.bar)) return;
    }
}

// Min-sum keeps the register budget of its chunked rule (four waves per
// SIMD); sum-product pays for its unrolled slots alone and is held to three
// waves per SIMD.
__global__ __launch_bounds__(kBlock) void k_persistent_nms(PArgs a) { persistent_body<kNMS>(a); }
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_persistent_spa(PArgs a) {
    persistent_body<kSPA>(a);
}

__global__ void k_reset(Barrier *b, ItemState *ist, int32_t nitems) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        b->count = 0;
        b->gen = 0;
        b->err = 0;
        b->live[0] = b->live[1] = 0;
        b->nnew[0] = b->nnew[1] = 0;
    }
    if (i < nitems) {
        ist[i].running[0] = ist[i].running[1] = 0;
        ist[i].live[0] = ist[i].live[1] = 0;
        ist[i].next_spare = 0;
    }
}

// Slots of a batch's 2 ng groups (originals, then spares) before the decode:
// running masks of its frames, their frame indices, empty spares.
__global__ void k_init_slots(uint64_t *words, int32_t *fid, int32_t g0, int32_t ng, int32_t nframes) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 2 * ng * G) return;
    const int k = j / G, lane = j % G;
    const bool orig = k < ng;
    const int f = k * G + lane;
    fid[static_cast<size_t>(g0) * G + j] = orig && f < nframes ? f : -1;
    if (lane == 0) {
        const int rem = nframes - k * G;
        const uint64_t valid = !orig ? 0 : rem >= G ? ~0ull : ((1ull << rem) - 1ull);
        words[static_cast<size_t>(kStride) * (g0 + k) + kRun] = valid;
        words[static_cast<size_t>(kStride) * (g0 + k) + kUnmet] = 0;
    }
}

__global__ void k_flag_error(const Barrier *bar, int32_t *err_out) {
    if (threadIdx.x == 0) *err_out = static_cast<int32_t>(bar->err);
}

// ------------------------------------------------------------------- host
struct BatchPlace {
    int32_t group0, ngroups;  // first group; groups holding frames (as many spares follow)
    size_t c, Lp, lam, zb, D;  // byte offsets of the batch's arrays
};

struct Built {
    std::vector<GroupDesc> gd;
    std::vector<ItemDesc> items;
    std::vector<BatchPlace> place;
    size_t off_gd, off_items, off_ist, off_words, off_src, off_newg, off_fid, off_bar, off_err, total;
    int32_t ngroups;
    int64_t nwork;  // work items of the largest phase over every group
};

// The persistent kernel indexes the tiles of a group with 32-bit integers.
int check_items(const Built &B) {
    if (B.nwork >= INT32_MAX)
        return fail(MBP_EUNSUPPORTED, "batched decode: more than 2^31 work items in one phase");
    return MBP_OK;
}

Built lay_out(int32_t nb, const mbp_batch *b, const mbp_tuning &tu) {
    Built B{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes);
        return at;
    };
    int32_t ng = 0;
    for (int32_t i = 0; i < nb; ++i) ng += 2 * ((b[i].nframes + G - 1) / G);
    B.ngroups = ng;
    B.off_gd = take(sizeof(GroupDesc) * std::max(ng, 1));
    B.off_items = take(sizeof(ItemDesc) * std::max(nb, 1));
    B.off_ist = take(sizeof(ItemState) * std::max(nb, 1));
    B.off_words = take(sizeof(uint64_t) * kStride * std::max(ng, 1));
    B.off_src = take(sizeof(int32_t) * G * std::max(ng, 1));
    B.off_newg = take(sizeof(int32_t) * std::max(ng, 1));
    B.off_fid = take(sizeof(int32_t) * G * std::max(ng, 1));
    B.off_bar = take(sizeof(Barrier));
    B.off_err = take(sizeof(int32_t));
    const int rpt = tu.rows_per_wave * kWaves, vpt = tu.vars_per_wave * kWaves;
    for (int32_t i = 0; i < nb; ++i) {
        const mbp_code *code = b[i].code;
        BatchPlace P{};
        P.group0 = static_cast<int32_t>(B.gd.size());
        P.ngroups = (b[i].nframes + G - 1) / G;
        const int32_t all = 2 * P.ngroups;
        // per-group strides are the ones the staging and output kernels index
        // with (g * E * G, g * n * G, g * M); each batch's region is aligned
        const size_t sc = static_cast<size_t>(code->E) * G * sizeof(float);
        const size_t sl = static_cast<size_t>(code->n) * G * sizeof(float);
        const size_t sz = static_cast<size_t>(code->M) * sizeof(uint64_t);
        const size_t sd = static_cast<size_t>(code->n) * sizeof(uint64_t);
        P.c = take(sc * all);
        P.Lp = take(sl * all);
        P.lam = take(sl * all);
        P.zb = take(sz * all);
        P.D = take(sd * all);
        ItemDesc it{};
        it.iters_out = b[i].iters_out;
        it.ok_out = b[i].ok_out;
        it.g0 = P.group0;
        it.ng = P.ngroups;
        it.nframes = b[i].nframes;
        B.items.push_back(it);
        for (int32_t k = 0; k < all; ++k) {
            GroupDesc d{};
            d.row_ptr = code->d_row_ptr;
            d.col = code->d_col;
            d.var_ptr = code->d_var_ptr;
            d.var_edge = code->d_var_edge_f;
            // state pointers are filled in once the workspace base is known
            d.c = reinterpret_cast<float *>(P.c + k * sc);
            d.Lp = reinterpret_cast<float *>(P.Lp + k * sl);
            d.lam = reinterpret_cast<float *>(P.lam + k * sl);
            d.zb = reinterpret_cast<uint64_t *>(P.zb + k * sz);
            d.D = reinterpret_cast<uint64_t *>(P.D + k * sd);
            d.E = code->E;
            d.n = code->n;
            d.dslots = dmax_for(code->max_check_deg);
            d.M = code->M;
            d.item = i;
            d.cn_tiles = (code->M + rpt - 1) / rpt;
            d.vn_tiles = (code->n + vpt - 1) / vpt;
            d.st_tiles = (code->M + kBlock - 1) / kBlock;
            B.nwork += std::max({d.cn_tiles, d.vn_tiles, d.st_tiles});
            B.gd.push_back(d);
        }
        B.place.push_back(P);
    }
    B.total = o;
    return B;
}

void rebase(Built &B, char *base) {
    for (GroupDesc &d : B.gd) {
        d.c = reinterpret_cast<float *>(base + reinterpret_cast<size_t>(d.c));
        d.Lp = reinterpret_cast<float *>(base + reinterpret_cast<size_t>(d.Lp));
        d.lam = reinterpret_cast<float *>(base + reinterpret_cast<size_t>(d.lam));
        d.zb = reinterpret_cast<uint64_t *>(base + reinterpret_cast<size_t>(d.zb));
        d.D = reinterpret_cast<uint64_t *>(base + reinterpret_cast<size_t>(d.D));
    }
}

const void *persistent_kernel(int algo) {
    return algo == kSPA ? reinterpret_cast<const void *>(&k_persistent_spa)
                        : reinterpret_cast<const void *>(&k_persistent_nms);
}

// Upload the group and batch descriptors (synchronous) after pointing them
// into the workspace at `base`.
int upload_descriptors(Built &B, char *base) {
    rebase(B, base);
    hipError_t err = hipMemcpy(base + B.off_gd, B.gd.data(), sizeof(GroupDesc) * B.gd.size(),
                               hipMemcpyHostToDevice);
    if (err == hipSuccess)
        err = hipMemcpy(base + B.off_items, B.items.data(), sizeof(ItemDesc) * B.items.size(),
                        hipMemcpyHostToDevice);
    return err == hipSuccess ? MBP_OK : hip_fail(err, "descriptor upload");
}

// Enqueue the whole batched decode on `stream` (kernels only, so it can be
// captured into a graph): staging, the persistent decode, outputs.
int enqueue_kernels(int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu, const Built &B,
                    char *base, int num_cus, hipStream_t stream, bool cooperative) {
    uint64_t *words = reinterpret_cast<uint64_t *>(base + B.off_words);
    int32_t *fid = reinterpret_cast<int32_t *>(base + B.off_fid);
    Barrier *bar = reinterpret_cast<Barrier *>(base + B.off_bar);
    ItemState *ist = reinterpret_cast<ItemState *>(base + B.off_ist);
    k_reset<<<(std::max(nb, 1) + 255) / 256, 256, 0, stream>>>(bar, ist, nb);
    for (int32_t i = 0; i < nb; ++i) {
        const BatchPlace &P = B.place[i];
        const mbp_code *code = b[i].code;
        const int32_t F = b[i].nframes, n = code->n, M = code->M;
        k_init_slots<<<(2 * P.ngroups * G + 255) / 256, 256, 0, stream>>>(words, fid, P.group0, P.ngroups, F);
        float *lam = reinterpret_cast<float *>(base + P.lam), *Lp = reinterpret_cast<float *>(base + P.Lp);
        k_stage_llr<float><<<dim3((n + 63) / 64, P.ngroups), kBlock, 0, stream>>>(b[i].llr, lam, Lp, F, n);
        k_stage_synd<<<dim3((M + kBlock - 1) / kBlock, P.ngroups), kBlock, 0, stream>>>(
            b[i].synd, reinterpret_cast<uint64_t *>(base + P.zb), F, M);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(err, "batched staging launch");
    PArgs a{reinterpret_cast<const GroupDesc *>(base + B.off_gd),
            reinterpret_cast<const ItemDesc *>(base + B.off_items),
            ist,
            words,
            fid,
            reinterpret_cast<int32_t *>(base + B.off_src),
            reinterpret_cast<int32_t *>(base + B.off_newg),
            bar,
            B.ngroups,
            nb,
            p->max_iter,
            p->early_exit,
            tu.rows_per_wave,
            tu.vars_per_wave,
            tu.schedule,
            tu.compact,
            static_cast<float>(p->alpha),
            static_cast<float>(p->llr_clip),
            p->algo == MBP_ALGO_SPA ? kSPA : kNMS};
    const void *kp = persistent_kernel(a.algo);
    const int bpc = std::max(1, std::min({tu.blocks_per_cu, blocks_per_cu(kp), kMaxBlocksPerCu}));
    const int grid = num_cus * bpc;
    void *args[] = {&a};
    if (cooperative)
        err = hipLaunchCooperativeKernel(kp, dim3(grid), dim3(kBlock), args, 0, stream);
    else
        err = hipLaunchKernel(kp, dim3(grid), dim3(kBlock), args, 0, stream);
    if (err != hipSuccess) return hip_fail(err, "persistent decode launch");
    for (int32_t i = 0; i < nb; ++i) {
        const BatchPlace &P = B.place[i];
        const int32_t n = b[i].code->n;
        launch_output_slots<float>(reinterpret_cast<const float *>(base + P.Lp),
                                   fid + static_cast<size_t>(P.group0) * G, b[i].bits_out, b[i].llr_out, n,
                                   2 * static_cast<int64_t>(P.ngroups), stream);
    }
    k_flag_error<<<1, 64, 0, stream>>>(bar, reinterpret_cast<int32_t *>(base + B.off_err));
    if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "batched output launch");
    return MBP_OK;
}

}  // namespace

mbp_tuning default_tuning() { return mbp_tuning{4, 4, 2, 0, 1}; }

int check_tuning(const mbp_tuning &tu) {
    if (tu.rows_per_wave < 1 || tu.rows_per_wave > 64 || tu.vars_per_wave < 1 || tu.vars_per_wave > 64 ||
        tu.blocks_per_cu < 1 || tu.blocks_per_cu > kMaxBlocksPerCu || tu.schedule < 0 || tu.schedule > 1 ||
        tu.compact < 0 || tu.compact > 1)
        return fail(MBP_EINVAL, "tuning out of range (rows/vars per wave 1..64, blocks per CU 1..4, "
                                "schedule 0..1, compact 0..1)");
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
    int rc = check_items(B);
    if (rc != MBP_OK) return rc;
    if ((rc = ensure_workspace(ctx, B.total)) != MBP_OK) return rc;
    char *base = static_cast<char *>(ctx->ws);
    // the previous user of the workspace may still be running on another stream
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    if ((rc = upload_descriptors(B, base)) != MBP_OK) return rc;
    if ((rc = enqueue_kernels(nb, b, p, tu, B, base, ctx->num_cus, stream, true)) != MBP_OK) return rc;
    int32_t flag = 0;
    if ((e = hipMemcpyAsync(&flag, base + B.off_err, sizeof(flag), hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return hip_fail(e, "batched decode completion");
    if (flag) return fail(MBP_EDEVICE, "batched decode: a grid barrier timed out");
    return MBP_OK;
}

int batched_launch(mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu,
                   void *ws, hipStream_t stream, int32_t **err_dev) {
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    Built B = lay_out(nb, b, tu);
    char *base = static_cast<char *>(ws);
    int rc = check_items(B);
    if (rc != MBP_OK) return rc;
    if ((rc = upload_descriptors(B, base)) != MBP_OK) return rc;
    if ((rc = enqueue_kernels(nb, b, p, tu, B, base, ctx->num_cus, stream, true)) != MBP_OK) return rc;
    *err_dev = reinterpret_cast<int32_t *>(base + B.off_err);
    return MBP_OK;
}

// Sets the cooperative launch attribute on every node of `graph` that
// launches a k_persistent instance (exactly one is expected).
static int mark_persistent_cooperative(hipGraph_t graph) {
    size_t count = 0;
    hipError_t e = hipGraphGetNodes(graph, nullptr, &count);
    if (e != hipSuccess) return hip_fail(e, "hipGraphGetNodes");
    std::vector<hipGraphNode_t> nodes(count);
    if (count && (e = hipGraphGetNodes(graph, nodes.data(), &count)) != hipSuccess)
        return hip_fail(e, "hipGraphGetNodes");
    int marked = 0;
    for (hipGraphNode_t node : nodes) {
        hipGraphNodeType type;
        if ((e = hipGraphNodeGetType(node, &type)) != hipSuccess) return hip_fail(e, "hipGraphNodeGetType");
        if (type != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp{};
        if ((e = hipGraphKernelNodeGetParams(node, &kp)) != hipSuccess)
            return hip_fail(e, "hipGraphKernelNodeGetParams");
        if (kp.func != persistent_kernel(kSPA) && kp.func != persistent_kernel(kNMS)) continue;
        hipKernelNodeAttrValue v{};
        v.cooperative = 1;
        if ((e = hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v)) != hipSuccess)
            return hip_fail(e, "hipGraphKernelNodeSetAttribute(cooperative)");
        ++marked;
    }
    if (marked != 1) return fail(MBP_EDEVICE, "plan capture: persistent kernel node not found");
    return MBP_OK;
}

int batched_plan_capture(mbp_ctx *ctx, int32_t nb, const mbp_batch *b, const mbp_params *p, const mbp_tuning &tu,
                         void *ws, hipGraphExec_t *exec, int32_t **err_dev) {
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    Built B = lay_out(nb, b, tu);
    char *base = static_cast<char *>(ws);
    int rc = check_items(B);
    if (rc != MBP_OK) return rc;
    if ((rc = upload_descriptors(B, base)) != MBP_OK) return rc;
    hipStream_t cap;
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    hipGraph_t graph = nullptr;
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = enqueue_kernels(nb, b, p, tu, B, base, ctx->num_cus, cap, false);
    const hipError_t e2 = hipStreamEndCapture(cap, &graph);
    (void)hipStreamDestroy(cap);
    if (rc != MBP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    // Stream capture records the persistent kernel as a plain kernel node.
    // Its grid barrier needs every block resident at once, which only a
    // cooperative launch guarantees, so that node is marked cooperative
    // before the graph is instantiated; a runtime that refuses the attribute
    // fails the plan rather than leaving a launch that could wait on blocks
    // that never start.
    if ((rc = mark_persistent_cooperative(graph)) != MBP_OK) {
        (void)hipGraphDestroy(graph);
        return rc;
    }
    e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *err_dev = reinterpret_cast<int32_t *>(base + B.off_err);
    return MBP_OK;
}

}  // namespace mbp
