// Device kernels and host launch helpers of the MBP decoder, shared by the
// plain decode driver (decode.hip) and the unrolled min-sum driver
// (unrolled.hip). Everything here has internal linkage.
//
// Layout in HBM. Frames are processed in groups of 64, one frame per lane of
// a wavefront, so every lane of a wave works on the same check or variable
// of the shared code and all graph indices are wave-uniform scalar loads.
// Per group g (all arrays frame-interleaved, 64 consecutive elements per
// graph node or edge):
//   c   [g][E][64]  check-to-variable messages, edges in check-major order
//   Lp  [g][n][64]  soft decisions L of eq. (2) (posterior LLRs)
//   lam [g][n][64]  channel LLRs
//   zb  [g][M]      syndrome bits, bit k = frame g*64+k
// A variable-to-check message is never stored: it is rebuilt as L - c from
// the previous iteration's L and c when the check pass reads them.
//
// One iteration t (flooding schedule over the stacked graph):
//   check pass     for every check of every matrix: q = L^{t-1} - c^{t-1} on
//                  each edge, c^t from the check rule of Sec. 3B eq. (6) (or
//                  normalized min-sum); it also XORs the decisions of L^{t-1}
//                  over the check, which is the stopping test of iteration
//                  t-1, and ORs unmet checks into a per-group lane mask;
//   variable pass  L^t = lambda + sum of c^t over the variable's edges in
//                  (matrix, check) order, eq. (2); frames whose test at t-1
//                  passed keep L^{t-1} and are retired with iters = t-1.
// After the last iteration a syndrome-only pass tests L^T.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "mbp_internal.h"

namespace mbp {
namespace {

constexpr int G = kLanes;
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kRowsPerWave = 4;
constexpr int kRowsPerTile = kRowsPerWave * kWaves;
constexpr int kVarsPerWave = 4;
constexpr int kVarsPerTile = kVarsPerWave * kWaves;
constexpr int kIdxChunk = 8;  // edge indices read per scalar batch

__device__ __forceinline__ unsigned lane_id() { return threadIdx.x & 63u; }
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

// 1 - tanh(a/2) = 2v / (1 + v) with v = e^-a, for a magnitude a >= 0 (at
// most the clip, so v does not underflow). v is the hardware exp2 of the
// rounded product -a log2(e): its relative error grows with a, to about 7e-7
// at a = 20, which becomes an absolute error of that size in a message that
// large (far inside the FP32 parity bound); the complement itself adds a few
// roundings (relative), and stays accurate where tanh is near 1.
__device__ __forceinline__ float tanh_complement(float a) {
    constexpr float kNegL2E = -1.44269504088896340736f;
    const float v = __builtin_amdgcn_exp2f(a * kNegL2E);
    return 2.0f * v * __builtin_amdgcn_rcpf(1.0f + v);
}

// IEEE sign bit of a float as a word (1u << 31 or 0).
__device__ __forceinline__ uint32_t sign_word(float x) { return __float_as_uint(x) & 0x80000000u; }

// Raw buffer access for the FP32 check pass: a descriptor per base address,
// a per-lane byte offset (the lane's slot in a 64-frame row) and a
// wave-uniform byte offset (the row), so a gather of a row costs no vector
// address arithmetic. Reads at or past num_records (measured from the
// per-lane offset) return 0 without touching memory.
// Compressed min-sum check state: rows per check, the largest degree it
// holds (one sign bit per edge below the position field) and where the
// position of the minimum sits in the third row.
constexpr int kStateRows = 3;
constexpr int kStateMaxDeg = 24;
constexpr int kStateArgShift = 26;

using BufRsrc = __amdgpu_buffer_rsrc_t;
constexpr uint32_t kBufAll = 0xFFFFFFFFu;
__device__ __forceinline__ BufRsrc buf_rsrc(const void *base, uint32_t num_records) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, static_cast<int>(num_records), 0x00020000);
}
__device__ __forceinline__ uint32_t buf_load(BufRsrc r, int lane_off, int row_off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, row_off, 0);
}
__device__ __forceinline__ void buf_store(uint32_t x, BufRsrc r, int lane_off, int row_off) {
    __builtin_amdgcn_raw_buffer_store_b32(x, r, lane_off, row_off, 0);
}
// Non-temporal access (the cache-policy operand's NT bit) for the check
// pass's message rows: each is read once and written once per pass, and
// marked so they do not push out of the caches the rows of L that the pass
// gathers many times over (the t >= 2 check pass at n = 2^18 takes 3.7 ms
// per average launch this way, 4.4 ms with default caching).
constexpr int kNonTemporal = 2;
__device__ __forceinline__ uint32_t buf_load_nt(BufRsrc r, int lane_off, int row_off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, row_off, kNonTemporal);
}
__device__ __forceinline__ void buf_store_nt(uint32_t x, BufRsrc r, int lane_off, int row_off) {
    __builtin_amdgcn_raw_buffer_store_b32(x, r, lane_off, row_off, kNonTemporal);
}
// Binary16 message storage: a message is read back as the float it rounds
// to, and stored rounded to the nearest binary16 (ties to even, the
// conversion's default mode). Non-temporal, as above.
__device__ __forceinline__ float buf_load_half(BufRsrc r, int lane_off, int row_off) {
    return static_cast<float>(
        __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, lane_off, row_off, kNonTemporal)));
}
__device__ __forceinline__ void buf_store_half(float x, BufRsrc r, int lane_off, int row_off) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, static_cast<_Float16>(x)), r,
                                          lane_off, row_off, kNonTemporal);
}

// 2 atanh(1 - E) = ln((2 - E) / E) for a complement E in (0, 1], with two
// hardware log2: no quotient is rounded, and nothing cancels where E is small
// (large messages). Where E is near 1 the result is small and carries an
// absolute error of a few 1e-8.
__device__ __forceinline__ float atanh2_of_complement(float E) {
    constexpr float kLn2 = 0.693147180559945309f;
    return (__builtin_amdgcn_logf(2.0f - E) - __builtin_amdgcn_logf(E)) * kLn2;
}

enum { kNMS = MBP_ALGO_NMS, kSPA = MBP_ALGO_SPA };

// Per-group status words (running mask and unmet-check mask, by iteration
// parity) sit kStride words apart, one 256-byte line per group.
constexpr int kStride = 32;

// OR lanes with an unmet check into a group's mask. A coherent read first
// skips the atomic when those lanes are already marked, which is the common
// case: the mask saturates after a few tiles in early iterations and stays
// near empty late, so few atomics reach the shared word.
__device__ __forceinline__ void or_unmet(uint64_t *word, uint64_t bits) {
    if (!bits) return;
    const uint64_t cur = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bits & ~cur)
        atomicOr(reinterpret_cast<unsigned long long *>(word), static_cast<unsigned long long>(bits));
}

// Scalars shared by the iteration kernels.
struct Dims {
    int64_t E;
    int32_t n, M, ngroups, ntiles;
    int32_t t;     // iteration (1-based)
    int32_t flag;  // stopping test: 1 on the last iteration (settles every frame)
    double alpha, clip;
    int32_t T = 0;        // stopping test: the iteration limit
    int32_t spare0 = 0;   // stopping test: first spare group (= groups holding frames)
    int32_t nspare = 0;   // stopping test: spare groups compaction may fill (0: none)
    int32_t row0 = 0;     // check pass: first stacked check of the pass
    int32_t row1 = -1;    // check pass: one past its last check (-1: M)
    int64_t emax = -1;    // variable pass: sum only edges below this (-1: all)
    // Channel LLRs given as Bob's bits (the BITS kernel instances): lambda of
    // slot k of group g at variable i is -mag or +mag, by bit k of
    // ybits[g * n + i], with mag = ymag[64 g + k] (element type T).
    const uint64_t *ybits = nullptr;
    const void *ymag = nullptr;
    // FP32 min-sum check pass with a compressed check state (CST instances):
    // per group and check, three 64-frame rows of words (kStateRows), read
    // at t >= 2 in place of the check's old messages and written every
    // iteration. Element type uint32_t.
    void *cstate = nullptr;
    // matrix-serial variable pass (k_variable_phase): the code's matrices,
    // this pass's matrix, the per-matrix positions of every variable's edges
    // ([l * n + i], l = 0..u) and the stored per-matrix sums
    // ([group][l][n][64], element type T)
    int32_t u = 1;
    int32_t phase = 0;
    const int32_t *vmptr = nullptr;
    void *psum = nullptr;
    // Independent decoders (coupling MBP_INDEPENDENT). The check pass reads
    // the posterior of each check's own matrix: its L input of group g is
    // at g * lstride (-1: n * 64, one L row per variable), plus
    // row_mat[r] * mstride for check r (0: the same L for every matrix).
    // The variable passes also write, per matrix l with an edge at the
    // variable, lambda + matrix l's messages summed (from 0, in check order)
    // to lm + g * prows * n * 64 + l * n * 64 (null: not written). emat
    // holds the first stacked edge of matrices 1, 2 and 3 (INT32_MAX past
    // the code's matrices), so an edge's matrix is the count it reaches.
    int64_t lstride = -1;
    int64_t mstride = 0;
    void *lm = nullptr;
    int32_t emat[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
    // Frames still running (StopTail::live), or null. Once the stopping
    // test has retired every frame, the iteration kernels the host launched
    // ahead of its poll return at once.
    const uint32_t *live = nullptr;
    // rows of n * 64 values per group in the array holding the stored
    // per-matrix sums (psum, rows 0..u-1) and the posteriors (lm)
    int32_t prows = 0;
    // variable pass (k_variable_fast): the variables [vbeg, vend) of one
    // degree class, and per variable the slots of its edge list that start
    // the next matrix's run (bit j: slot j, j >= 1)
    int32_t vbeg = 0, vend = 0;
    const uint64_t *runs = nullptr;
    // First iteration in closed form (from Bob's bits; k_first_parity,
    // k_first_table, k_variable_first and the SHORT check pass): per group
    // the checks' parity words ([g][M]), the lane masks of frames whose
    // lambda is negative for bit 0 and of frames with a nonzero lambda
    // ([g][2]), and the table of first-iteration message magnitudes
    // ([g][mrows][64], row d (d - 1) / 2 + j: slot j of a check of degree
    // d); per variable edge its check and table row (kRtShift packing).
    const uint64_t *spar = nullptr;
    const uint64_t *smask = nullptr;
    const float *mtab = nullptr;
    int32_t mrows = 0;
    const uint32_t *var_rt = nullptr;
    // variable pass: visit the groups last to first. The check pass visits
    // them first to last, so the variable pass starts on the group whose
    // messages were written last (the likeliest still in the last-level
    // cache), and the next check pass on the group read last.
    int32_t reverse = 0;
};

// Bob's bit words: each lane reads the 32-bit half of word i that holds its
// bit. The address is per lane, so the read is one vector load touching a
// single 8-byte word for the whole wave (a uniform address would become a
// chain of scalar loads, which measured slower than gathering 256-byte
// rows). Callers issue every such load before converting any (lam_of_half),
// so the loads stay in flight together.
__device__ __forceinline__ uint32_t bit_half(const uint64_t *yg, int i, unsigned lane) {
    return reinterpret_cast<const uint32_t *>(yg + i)[lane >> 5];
}
template <typename T>
__device__ __forceinline__ T lam_of_half(uint32_t half, unsigned lane, T mag) {
    return (half >> (lane & 31u)) & 1u ? -mag : mag;
}

// Counters after the plain decode's status words: the stopping test's
// arrival count, the spare groups filled so far, and the compaction the
// last stopping test planned (first new group, how many).
struct StopTail {
    uint32_t done, spare_used;
    int32_t move_first, move_count;
    uint32_t live;  // frames still running after the last settle
};

// Per-group status words for the plain and unrolled decodes: word kRun of
// group g (at kStride * g) holds the frames still running, word kUnmet the
// frames with an unmet check in the stopping test under way.
constexpr int kRun = 0, kUnmet = 1;

// Groups that still have running frames, as a bitmap in LDS that a block
// fills at the start of an iteration kernel (the running sets do not change
// while it runs); groups past the bitmap's capacity count as running. The
// kernels' work-item cursors use it to jump over retired groups.
constexpr int kLiveWords = 1024;  // 32768 groups
__device__ __forceinline__ void load_live(uint32_t *bits, const uint64_t *act, int ngroups) {
    const unsigned lane = threadIdx.x & 63u;
    const int ng = min(ngroups, kLiveWords * 32);
    for (int base = static_cast<int>(threadIdx.x >> 6) * 64; base < ng; base += kBlock) {
        const int g = base + static_cast<int>(lane);
        const uint64_t b = __ballot(g < ng && act[kStride * g + kRun] != 0);
        if (lane == 0) {
            bits[base / 32] = static_cast<uint32_t>(b);
            if (base / 32 + 1 < kLiveWords) bits[base / 32 + 1] = static_cast<uint32_t>(b >> 32);
        }
    }
    __syncthreads();
}
__device__ __forceinline__ bool is_live(const uint32_t *bits, int g) {
    return g >= kLiveWords * 32 || ((bits[g >> 5] >> (g & 31)) & 1u);
}
// The block's first work item at or after w (items blockIdx.x + k gridDim.x,
// ntiles per group, group index gw = w / ntiles, mapped to its group by
// `group`) whose group is running; total or more if none.
template <typename GroupOf>
__device__ __forceinline__ uint32_t live_item(uint32_t w, uint32_t total, uint32_t ntiles, const uint32_t *bits,
                                              GroupOf group) {
    while (w < total) {
        const uint32_t gw = w / ntiles;
        if (is_live(bits, group(static_cast<int>(gw)))) return w;
        // the block's first item in the next group
        const uint32_t start = (gw + 1) * ntiles;
        w += ((start - w + gridDim.x - 1) / gridDim.x) * gridDim.x;
    }
    return w;
}


// One check of the FP32 check pass, for the lanes of one wave (frames of
// one group): v(j) gives the check's j-th variable index, wave-uniform (it is
// read right where slot j's gather is issued; slots past the degree d read
// row 0), src the group's L rows (or, BITS, its bit
// words), ci / cg the check's first c^{t-1} / c^t row. Every slot loads,
// unconditionally (a slot past the degree reads row 0 and is neutralised
// below), so the loads carry no branches and no vector address arithmetic;
// only the stores test the degree.
//
// `prefetch` runs once the check's loads are issued (the caller's loads for
// its next check go out while these are in flight). Every lane loads and
// computes (so the caller's prefetched values stay wave-uniform); only lanes
// with `on` (frames still running) store.
//
// NT: the message rows with the non-temporal cache policy (the plain
// decode; the batched decode's cells are small enough that a pass's messages
// can stay in the Infinity Cache for the next pass, so it keeps the default).
//
// With CST (min-sum only, DMAX <= kStateMaxDeg) the check's state `st`
// replaces its old messages: row 0 holds alpha m1, row 1 alpha m2, row 2 the
// sign of each outgoing message (bit j) and the position of the minimum
// (bits 26-31). Every old message is rebuilt from them bit for bit, so the
// pass reads 3 rows per check instead of one per edge; it still writes
// every message (the variable pass reads them) and the new state.
//
// With SHORT (the second iteration after a first one in closed form) the old
// messages are not read from ci: message j of the first iteration has the
// magnitude oldmag(j) (first_mags of the check's degree, formed by the
// caller) and the sign S_r XOR s_j, S_r the check's parity bit and s_j the
// lambda sign bit of the slot's variable (its bit XOR flip, or 0 where
// lambda is zero), which is the message the check pass from bits would have
// stored, bit for bit.
struct NoPrefetch {
    __device__ void operator()() const {}
};

struct NoOldMag {
    __device__ float operator()(int) const { return 0.0f; }
};

// The sign of old message j in this lane's frame, as bit 31: S_r where
// lambda is zero, else S_r XOR flip XOR the frame's bit of slot j's
// variable, taken from that variable's bit word (word j of yrow, the
// 32-bit half holding the lane's bit) moved up to bit 31 by a shift.
struct FirstMsgs {
    const uint32_t *yrow;  // the check's bit words in LDS: [slot][low, high half]
    uint32_t shift;        // 31 - (lane mod 32)
    uint32_t k31;          // (S_r XOR flip) << 31
    uint32_t nz31;         // 1 << 31 where lambda is nonzero, else 0
    uint32_t z31;          // S_r << 31 where lambda is zero, else 0
    __device__ uint32_t sign(int j, unsigned lane) const {
        const uint32_t w = yrow[2 * j + static_cast<int>(lane >> 5)];
        return (((w << shift) ^ k31) & nz31) | z31;
    }
};

// The magnitudes of the first iteration's messages of a check of degree d
// when every lambda of the frame has the magnitude |ym| (decoding from Bob's
// bits), slot by slot, with the operations of the check pass from bits in
// the same order: sum-product merges the complements' prefix chain P_j with
// the suffix chain, which for equal complements is P_{d-1-j} (so slots j and
// d-1-j share one magnitude); min-sum takes alpha times the smaller of |ym|
// and the clip (the second minimum, +inf, at slot 0 of a degree-1 check).
// With H each is rounded to binary16, as the stored message is (the rounding
// is symmetric in the sign). Written to om[j * 64 + lane], j < d, in place:
// the chain first, then each pair of mirrored slots from its two chain
// values, so no register array is held.
//
// No multiply-add contraction here: the complement e is a product, and
// fusing it into the chain's sums (which the check pass from bits cannot do,
// as its e passes through a sign-bit merge) would round differently.
template <int ALGO, bool H>
__device__ __forceinline__ void first_mags(int d, float ym, float clip, float alpha, float *om, unsigned lane) {
#pragma clang fp contract(off)
    auto put = [&](int j, float v) {
        if constexpr (H) v = static_cast<float>(static_cast<_Float16>(v));
        om[j * G + lane] = v;
    };
    if constexpr (ALGO == kNMS) {
        const float m1 = fminf(fabsf(ym), clip);
        const float m2 = d >= 2 ? m1 : INFINITY;
        for (int j = 0; j < d; ++j) put(j, j == 0 ? alpha * m2 : alpha * m1);
    } else {
        const float e = tanh_complement(fminf(fabsf(ym), clip));
        float run = 0.0f;
        for (int j = 0; j < d; ++j) {
            om[j * G + lane] = run;
            run = fmaf(-run, e, run + e);
        }
        for (int j = 0; j <= d - 1 - j; ++j) {
            const int k = d - 1 - j;
            const float x = om[j * G + lane], y = om[k * G + lane];
            const float v = __uint_as_float(__float_as_uint(atanh2_of_complement(fmaf(-x, y, x + y))) & 0x7fffffffu);
            put(j, v);
            put(k, v);
        }
    }
}

template <int ALGO, int DMAX, bool BITS, bool CST = false, bool H = false, bool SHORT = false, bool NT = true,
          typename Cols, typename Prefetch = NoPrefetch, typename OldMag = NoOldMag>
__device__ __forceinline__ void check_row_f32(const Cols &v, int d, uint32_t zbit, float alpha,
                                              float clip, bool first, BufRsrc src, const void *ci, void *cg,
                                              unsigned lane, float ym, uint32_t *st = nullptr,
                                              Prefetch prefetch = Prefetch(), bool on = true,
                                              const FirstMsgs &fm = FirstMsgs(), const OldMag &oldmag = OldMag()) {
    static_assert(!SHORT || (!BITS && !CST), "closed-form old messages: the FP32 pass from messages");
    static_assert(!CST || (ALGO == kNMS && DMAX <= kStateMaxDeg), "compressed state: min-sum, small degree");
    static_assert(!(CST && H), "binary16 messages keep no compressed state");
    const int lo = static_cast<int>(lane) * 4;
    // messages: 4-byte floats, or (H) binary16 values in 2-byte slots
    constexpr int ES = H ? 2 : 4;
    const int lm = static_cast<int>(lane) * ES;
    // c^{t-1} of the check's edges (read only after the first iteration:
    // c^0 = 0). The descriptors' record counts are constants: a count chosen
    // at run time by a select can be formed in a vector register, and a
    // descriptor held in vector registers costs a loop around every access.
    const BufRsrc rin = buf_rsrc(ci, kBufAll);
    const BufRsrc rout = buf_rsrc(cg, kBufAll);
    const BufRsrc rst = buf_rsrc(st, kBufAll);
    // stores message j (its float bit pattern) into c^t
    const auto put = [&](int j, uint32_t word) {
        if constexpr (H)
            buf_store_half(__uint_as_float(word), rout, lm, j * G * ES);
        else if constexpr (NT)
            buf_store_nt(word, rout, lo, j * G * 4);
        else
            buf_store(word, rout, lo, j * G * 4);
    };
    float q[DMAX];
    if constexpr (CST && !BITS) {
        // the old messages from the state (zeros at t = 1: nothing to read)
        float o1 = 0.0f, o2 = 0.0f;
        uint32_t os = 0;
        if (!first) {
            o1 = __uint_as_float(buf_load(rst, lo, 0));
            o2 = __uint_as_float(buf_load(rst, lo, G * 4));
            os = buf_load(rst, lo, 2 * G * 4);
        }
        const int oi = static_cast<int>(os >> kStateArgShift);
#pragma unroll
        for (int j = 0; j < DMAX; ++j) q[j] = __uint_as_float(buf_load(src, lo, (j < d ? v(j) : 0) * G * 4));
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const float mag = j == oi ? o2 : o1;
            q[j] -= __uint_as_float(__float_as_uint(mag) | (((os >> j) & 1u) << 31));
        }
    } else if constexpr (BITS) {
        uint32_t yh[DMAX];
        const int hl = static_cast<int>(lane >> 5) * 4;  // the 32-bit half holding the lane's bit
#pragma unroll
        for (int j = 0; j < DMAX; ++j) yh[j] = buf_load(src, hl, (j < d ? v(j) : 0) * 8);
#pragma unroll
        for (int j = 0; j < DMAX; ++j) q[j] = lam_of_half(yh[j], lane, ym);
    } else {
        if (first) {
#pragma unroll
            for (int j = 0; j < DMAX; ++j) q[j] = __uint_as_float(buf_load(src, lo, (j < d ? v(j) : 0) * G * 4));
        } else if constexpr (SHORT) {
#pragma unroll
            for (int j = 0; j < DMAX; ++j) q[j] = __uint_as_float(buf_load(src, lo, (j < d ? v(j) : 0) * G * 4));
#pragma unroll
            for (int j = 0; j < DMAX; ++j)
                q[j] -= __uint_as_float(__float_as_uint(oldmag(j)) | fm.sign(j, lane));
        } else {
            float co[DMAX];
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                q[j] = __uint_as_float(buf_load(src, lo, (j < d ? v(j) : 0) * G * 4));
                if constexpr (H)
                    co[j] = buf_load_half(rin, lm, (j < d ? j : 0) * G * ES);
                else
                    co[j] = __uint_as_float(NT ? buf_load_nt(rin, lo, (j < d ? j : 0) * G * 4)
                                               : buf_load(rin, lo, (j < d ? j : 0) * G * 4));
            }
#pragma unroll
            for (int j = 0; j < DMAX; ++j) q[j] -= co[j];
        }
    }
    // the caller's next loads go out while this check's are in flight
    prefetch();
    // Signs ride in the IEEE sign bits (q + 0 turns -0 into +0: sgn(0) =
    // +1), so the sign product is an XOR of words; slots past the degree
    // contribute no sign.
    uint32_t sxb = zbit << 31;
    if constexpr (ALGO == kNMS) {
        // slots past the degree enter the running minima as +inf, which
        // leaves them unchanged; m2 = med3(m1, a, m2) is the second minimum
        // after taking a, as m1 <= m2 always
        float m1 = INFINITY, m2 = INFINITY;
        int i1 = 0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const bool real = j < d;
            q[j] = q[j] + 0.0f;
            sxb ^= real ? __float_as_uint(q[j]) : 0u;
            const float aj = real ? fminf(fabsf(q[j]), clip) : INFINITY;
            m2 = __builtin_amdgcn_fmed3f(m1, aj, m2);
            i1 = aj < m1 ? j : i1;
            m1 = fminf(m1, aj);
        }
        const float a1 = alpha * m1, a2 = alpha * m2;
        uint32_t signs = 0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const uint32_t sw = sign_word(__uint_as_float(sxb ^ __float_as_uint(q[j])));
            if constexpr (CST) signs |= (sw >> 31) << j;
            if (j < d && on) {
                const float mag = j == i1 ? a2 : a1;  // >= 0
                put(j, __float_as_uint(mag) | sw);
            }
        }
        if constexpr (CST) {
            if (on) {
                buf_store(__float_as_uint(a1), rst, lo, 0);
                buf_store(__float_as_uint(a2), rst, lo, G * 4);
                buf_store(signs | (static_cast<uint32_t>(i1) << kStateArgShift), rst, lo, 2 * G * 4);
            }
        }
    } else {
        // sum-product: the tanh product over the other edges, carried as
        // complements E = 1 - prod tanh(a/2) (a prefix and a suffix, merged
        // per edge), so magnitudes near the clip, where tanh rounds to 1,
        // keep their precision: 1 - (1 - x)(1 - y) = x + y - xy. Slots past
        // the degree hold the complement 0 (tanh = 1), for which both
        // running updates are exact no-ops. Each complement carries its
        // message's sign in its sign bit (read through fabsf, which costs
        // nothing).
        // From Bob's bits every message of a frame has the magnitude ym, so
        // its complement is formed once (the same value each slot would get).
        const float e_bits = BITS ? tanh_complement(fminf(fabsf(ym), clip)) : 0.0f;
        float ep[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const bool real = j < d;
            const float qj = q[j] + 0.0f;
            sxb ^= real ? __float_as_uint(qj) : 0u;
            const float mag = BITS ? e_bits : tanh_complement(fminf(fabsf(qj), clip));
            const float e = __uint_as_float(__float_as_uint(mag) | sign_word(qj));
            ep[j] = real ? e : 0.0f;
        }
        float run = 0.0f;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const float e = fabsf(ep[j]);
            q[j] = run;  // complement of the product before j
            run = fmaf(-run, e, run + e);
        }
        if constexpr (BITS) {
            // Every complement is e_bits, so the suffix at slot j (over the
            // d - 1 - j slots after it) is the prefix of d - 1 - j slots, and
            // slots j and d - 1 - j merge the same two values (fma and the sum
            // commute): their magnitudes are equal bit for bit. For a full or
            // nearly full row (the common case) each pair's magnitude is formed
            // once; other rows take the general suffix pass below.
            auto full_row = [&](auto dd) {
                constexpr int D = decltype(dd)::value;
#pragma unroll
                for (int j = 0; j <= D - 1 - j; ++j) {
                    const int k = D - 1 - j;  // slot j's mirror
                    const float mag = atanh2_of_complement(fmaf(-q[j], q[k], q[j] + q[k]));
                    if (on) {
                        const uint32_t sj = sign_word(__uint_as_float(sxb ^ __float_as_uint(ep[j])));
                        put(j, (__float_as_uint(mag) & 0x7fffffffu) | sj);
                        if (k != j) {
                            const uint32_t sk = sign_word(__uint_as_float(sxb ^ __float_as_uint(ep[k])));
                            put(k, (__float_as_uint(mag) & 0x7fffffffu) | sk);
                        }
                    }
                }
            };
            if (d == DMAX) {
                full_row(std::integral_constant<int, DMAX>());
                return;
            }
            if (d == DMAX - 1) {
                full_row(std::integral_constant<int, DMAX - 1>());
                return;
            }
        }
        float suf = 0.0f;
#pragma unroll
        for (int j = DMAX - 1; j >= 0; --j) {
            if (j < d && on) {
                const float E = fmaf(-q[j], suf, q[j] + suf);
                const float mag = atanh2_of_complement(E);
                const uint32_t sb = sign_word(__uint_as_float(sxb ^ __float_as_uint(ep[j])));
                put(j, (__float_as_uint(mag) & 0x7fffffffu) | sb);
            }
            const float e = fabsf(ep[j]);
            suf = fmaf(-suf, e, suf + e);
        }
    }
}

// Address of element `off` of a message array: 4-byte floats (or T), or
// (H) 2-byte binary16 slots.
template <bool H, typename P>
__device__ __forceinline__ P *msg_at(P *base, size_t off) {
    using B = typename std::conditional<std::is_const<P>::value, const uint16_t, uint16_t>::type;
    if constexpr (H)
        return reinterpret_cast<P *>(reinterpret_cast<B *>(base) + off);
    else
        return base + off;
}

// Check-node pass, iteration t. Each wave handles kRowsPerWave checks of one
// group. The check's edge indices are read up front as scalars (the column
// array is padded by kIndexPad entries so a full DMAX block is always in
// bounds), then all gathers of the check are issued before any is consumed;
// the messages stay in registers (q[j]) between the gather and the write.
// FP32 checks run check_row_f32; the body below is the FP64 one.
//
// c_in holds c^{t-1} (unused at t = 1) and c_out receives c^t; the plain
// decode passes the same array for both (each edge is read before it is
// written, by the same lane). The BITS instance runs the first iteration from
// Bob's bits instead of Lp (q = lambda, c^0 = 0): its gathers touch one
// 8-byte bit word per edge rather than a 256-byte row. alpha_l, if not null,
// gives the min-sum weight of each matrix for this iteration (row_mat maps a
// check to its matrix); otherwise a.alpha applies to every check. With H
// (FP32 only) c_in and c_out hold binary16 messages, two bytes per slot.
template <typename T, int ALGO, int DMAX, bool BITS = false, bool CST = false, bool H = false, bool SHORT = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SHORT && DMAX <= 34 ? 4 : 1))) void k_check(const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col,
                                                  const int32_t *__restrict__ row_mat,
                                                  const float *__restrict__ alpha_l,
                                                  const uint64_t *__restrict__ zb,
                                                  const uint64_t *__restrict__ act,
                                                  const T *__restrict__ Lp, const T *c_in, T *c_out,
                                                  const Dims a) {
    if (a.live && *a.live == 0) return;  // every frame retired
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const T clip = static_cast<T>(a.clip);
    const bool first = a.t == 1;
    const int64_t total = static_cast<int64_t>(a.ngroups) * a.ntiles;
    if constexpr (sizeof(T) == 4 && !BITS) {
        // FP32 from messages: the wave's checks (kRowsPerWave per work item,
        // items a grid stride apart, groups with running frames only) as one
        // software-pipelined stream. While a check's gathers are in flight
        // the wave loads the next check's column indices (one vector load:
        // lane j holds column j) and the scalars of the one after (one
        // per-lane gather), so no check waits on its own chain of index
        // loads. (The first pass from Bob's bits gathers from cache and is
        // bound by arithmetic; it takes the plain loop below.)
        __shared__ uint32_t live[kLiveWords];
        load_live(live, act, a.ngroups);
        const int rend = a.row1 < 0 ? a.M : a.row1;
        // A check's scalars travel in one register (lane 0: row_ptr[r],
        // 1: row_ptr[r + 1], 2-3: the group's running set, 4-5: the check's
        // syndrome word, 6: the group, 7: the check; r >= rend: none), so
        // three checks in flight hold few scalar registers; its column
        // indices in another (lane j < DMAX: col[row_ptr[r] + j], the array
        // padded past E).
        struct Row {
            int32_t info, cols;
        };
        // total < 2^31 (the host checks): 32-bit cursor over the block's work
        // items of running groups, and the check within the item
        const uint32_t tot = static_cast<uint32_t>(total), nt = static_cast<uint32_t>(a.ntiles);
        auto same = [](int g) { return g; };
        uint32_t cw = live_item(blockIdx.x, tot, nt, live, same);
        int ck = 0;
        auto meta = [&](Row &R) {
            if (cw >= tot) return false;
            const int g = static_cast<int>(cw / nt);
            const int tile = static_cast<int>(cw % nt);
            const int r = a.row0 + tile * kRowsPerTile + ck * kWaves + wave;
            const int rr = r < rend ? r : rend - 1;
            const int l = static_cast<int>(lane);
            // (SHORT: 8-9 the check's parity word, 10-11 and 12-13 the
            // group's lambda sign masks)
            const int32_t *src = l < 2 ? row_ptr + rr + l
                               : l < 4 ? reinterpret_cast<const int32_t *>(act + kStride * g + kRun) + (l - 2)
                               : l < 6 ? reinterpret_cast<const int32_t *>(zb + static_cast<size_t>(g) * a.M + rr) + (l - 4)
                               : !SHORT || l < 8 ? row_ptr + rr
                               : l < 10 ? reinterpret_cast<const int32_t *>(a.spar + static_cast<size_t>(g) * a.M + rr) + (l - 8)
                               : l < 14 ? reinterpret_cast<const int32_t *>(a.smask + 2 * static_cast<size_t>(g)) + (l - 10)
                                        : row_ptr + rr;
            const int32_t got = *src;
            R.info = l == 6 ? g : l == 7 ? r : got;
            if (++ck == kRowsPerWave) {
                ck = 0;
                cw = live_item(cw + gridDim.x, tot, nt, live, same);
            }
            return true;
        };
        auto cols = [&](Row &R) {
            R.cols = static_cast<int>(lane) < DMAX ? col[__builtin_amdgcn_readlane(R.info, 0) + static_cast<int>(lane)]
                                                   : 0;
        };
        Row cur, nxt, nn;
        // SHORT: the old messages' magnitudes of the wave's last (group,
        // degree), in the wave's own part of LDS (each lane its column)
        __shared__ float om[SHORT ? kWaves * DMAX * G : 1];
        __shared__ uint32_t ysh[SHORT ? kWaves * 2 * DMAX : 1];
        int om_key = -1;
        if (!meta(cur)) return;
        cols(cur);
        bool has_nxt = meta(nxt);
        for (;;) {
            bool has_nn = false;
            auto prefetch = [&]() {
                if (has_nxt) cols(nxt);
                has_nn = meta(nn);
            };
            const int r = __builtin_amdgcn_readlane(cur.info, 7);
            const uint64_t run = static_cast<uint32_t>(__builtin_amdgcn_readlane(cur.info, 2)) |
                                 (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(cur.info, 3))) << 32);
            if (r < rend && run != 0) {
                const int g = __builtin_amdgcn_readlane(cur.info, 6);
                const bool on = (run >> lane) & 1;
                const int e0 = __builtin_amdgcn_readlane(cur.info, 0);
                const int d = __builtin_amdgcn_readlane(cur.info, 1) - e0;
                const uint32_t zlo = static_cast<uint32_t>(__builtin_amdgcn_readlane(cur.info, 4));
                const uint32_t zhi = static_cast<uint32_t>(__builtin_amdgcn_readlane(cur.info, 5));
                const uint32_t zbit = ((lane < 32 ? zlo : zhi) >> (lane & 31u)) & 1u;
                const float alpha = alpha_l ? alpha_l[row_mat[r]] : static_cast<float>(a.alpha);
                const size_t cb = (static_cast<size_t>(g) * a.E + e0) * G;
                const T *Lg = Lp + static_cast<size_t>(g) * (a.lstride < 0 ? static_cast<int64_t>(a.n) * G : a.lstride);
                // independent decoders: the posterior of the check's own matrix
                const T *Lr = a.mstride ? Lg + row_mat[r] * a.mstride : Lg;
                uint32_t *st = CST ? static_cast<uint32_t *>(a.cstate) + (static_cast<size_t>(g) * a.M + r) * kStateRows * G
                                   : nullptr;
                const int32_t cs = cur.cols;
                auto v = [cs](int j) { return __builtin_amdgcn_readlane(cs, j); };
                FirstMsgs fm;
                if constexpr (SHORT) {
                    auto bit = [&](int k) {
                        const uint32_t lo32 = static_cast<uint32_t>(__builtin_amdgcn_readlane(cur.info, k));
                        const uint32_t hi32 = static_cast<uint32_t>(__builtin_amdgcn_readlane(cur.info, k + 1));
                        return ((lane < 32 ? lo32 : hi32) >> (lane & 31u)) & 1u;
                    };
                    // lane j: the bit word of slot j's variable (the column
                    // indices of lanes past the degree are in range too),
                    // put in the wave's part of LDS for every lane to read
                    const uint2 yw = reinterpret_cast<const uint2 *>(a.ybits + static_cast<size_t>(g) * a.n)[cs];
                    uint32_t *yrow = ysh + wave * 2 * DMAX;
                    // (the wave's LDS accesses run in order; the barriers
                    // keep the compiler from moving them across each other)
                    __builtin_amdgcn_wave_barrier();
                    if (static_cast<int>(lane) < DMAX) {
                        yrow[2 * lane] = yw.x;
                        yrow[2 * lane + 1] = yw.y;
                    }
                    __builtin_amdgcn_wave_barrier();
                    const uint32_t sbit = bit(8), flip = bit(10), nz = bit(12);
                    fm = FirstMsgs{yrow, 31u - (lane & 31u), (sbit ^ flip) << 31, nz << 31, nz ? 0u : sbit << 31};
                    // the old magnitudes depend on the group and the degree
                    // only: formed again when either changes (a wave's
                    // stream stays in one group for many checks, and most
                    // checks of a PEG code share one degree)
                    const int key = g * 128 + d;
                    if (key != om_key) {
                        const float ym = static_cast<const float *>(a.ymag)[static_cast<size_t>(g) * G + lane];
                        first_mags<ALGO, H>(d, ym, clip, alpha, om + wave * DMAX * G, lane);
                        om_key = key;
                    }
                }
                auto oldmag = [&](int j) { return om[(wave * DMAX + j) * G + lane]; };
                check_row_f32<ALGO, DMAX, false, CST, H, SHORT>(v, d, zbit, alpha, clip, first,
                                                                buf_rsrc(Lr, kBufAll), msg_at<H>(c_in, cb),
                                                                msg_at<H>(c_out, cb), lane, 0.0f, st, prefetch,
                                                                on, fm, oldmag);
            } else {
                prefetch();
            }
            if (!has_nxt) break;
            cur = nxt;
            nxt = nn;
            has_nxt = has_nn;
        }
        return;
    }
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int g = static_cast<int>(w / a.ntiles);
        const int tile = static_cast<int>(w % a.ntiles);
        const uint64_t gact = act[kStride * g + kRun];
        if (gact == 0) continue;  // whole group retired (uniform over the block)
        const bool on = (gact >> lane) & 1;
        // wave-uniform bases; every access below is base[lane], so addresses
        // are a scalar base plus one per-lane offset
        const T *Lg = Lp + static_cast<size_t>(g) * (a.lstride < 0 ? static_cast<int64_t>(a.n) * G : a.lstride);
        const uint64_t *zg = zb + static_cast<size_t>(g) * a.M;
        const uint64_t *yg = BITS ? a.ybits + static_cast<size_t>(g) * a.n : nullptr;
        const T ym = BITS ? static_cast<const T *>(a.ymag)[static_cast<size_t>(g) * G + lane] : T(0);
        for (int k = 0; k < kRowsPerWave; ++k) {
            const int r = a.row0 + tile * kRowsPerTile + k * kWaves + wave;
            if (r >= (a.row1 < 0 ? a.M : a.row1)) break;
            const int e0 = row_ptr[r];
            const int d = row_ptr[r + 1] - e0;
            const int zbit = static_cast<int>((zg[r] >> lane) & 1);
            const T alpha = alpha_l ? static_cast<T>(alpha_l[row_mat[r]]) : static_cast<T>(a.alpha);
            const size_t cb = (static_cast<size_t>(g) * a.E + e0) * G;
            const T *ci = c_in + cb;
            T *cg = c_out + cb;
            // independent decoders: the posterior of the check's own matrix
            const T *Lr = a.mstride ? Lg + row_mat[r] * a.mstride : Lg;
            int v[DMAX];
#pragma unroll
            for (int j = 0; j < DMAX; ++j) v[j] = col[e0 + j];
            if constexpr (sizeof(T) == 4) {
                uint32_t *st = CST ? static_cast<uint32_t *>(a.cstate) +
                                         (static_cast<size_t>(g) * a.M + r) * kStateRows * G
                                   : nullptr;
                if (on)
                    check_row_f32<ALGO, DMAX, BITS, CST, H>(
                        [&v](int j) { return v[j]; }, d, static_cast<uint32_t>(zbit), alpha, clip, first,
                        BITS ? buf_rsrc(yg, kBufAll) : buf_rsrc(Lr, kBufAll), msg_at<H>(c_in, cb),
                        msg_at<H>(c_out, cb), lane, ym, st);
            } else if (on) {
                // issue every gather of the check before using any of them
                T q[DMAX], co[DMAX];
                uint32_t yh[DMAX];
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    if (j < d) {
                        if constexpr (BITS) {
                            yh[j] = bit_half(yg, v[j], lane);
                        } else {
                            q[j] = (Lr + static_cast<size_t>(v[j]) * G)[lane];
                            co[j] = first ? T(0) : (ci + j * G)[lane];
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    if (j < d) {
                        if constexpr (BITS)
                            q[j] = lam_of_half(yh[j], lane, ym);
                        else
                            q[j] -= co[j];
                    }
                }
                uint64_t neg = 0;
                int sx = zbit;  // syndrome sign times every message sign
                // FP64 from here (FP32 takes check_row_f32)
                if constexpr (ALGO == kNMS) {
                    T m1 = T(INFINITY), m2 = T(INFINITY);
                    int i1 = 0;
#pragma unroll
                    for (int j = 0; j < DMAX; ++j) {
                        if (j < d) {
                            const int s = q[j] < T(0) ? 1 : 0;
                            sx ^= s;
                            neg |= static_cast<uint64_t>(s) << j;
                            T aj = fabs(q[j]);
                            aj = aj < clip ? aj : clip;
                            if (aj < m1) {
                                m2 = m1;
                                m1 = aj;
                                i1 = j;
                            } else if (aj < m2) {
                                m2 = aj;
                            }
                        }
                    }
#pragma unroll
                    for (int j = 0; j < DMAX; ++j) {
                        if (j < d) {
                            const T mag = alpha * (j == i1 ? m2 : m1);
                            const int s = sx ^ static_cast<int>((neg >> j) & 1);
                            (cg + j * G)[lane] = s ? -mag : mag;
                        }
                    }
                } else {
                    // sum-product, FP64: tanh domain with prefix/suffix products
                    T th[DMAX];
#pragma unroll
                    for (int j = 0; j < DMAX; ++j) {
                        if (j < d) {
                            const int s = q[j] < T(0) ? 1 : 0;
                            sx ^= s;
                            neg |= static_cast<uint64_t>(s) << j;
                            T aj = fabs(q[j]);
                            aj = aj < clip ? aj : clip;
                            th[j] = tanh(aj * T(0.5));
                        }
                    }
                    T run = T(1);
#pragma unroll
                    for (int j = 0; j < DMAX; ++j) {
                        if (j < d) {
                            q[j] = run;  // product of tanh over edges before j
                            run *= th[j];
                        }
                    }
                    T suf = T(1);
#pragma unroll
                    for (int j = DMAX - 1; j >= 0; --j) {
                        if (j < d) {
                            const T mag = T(2) * atanh(q[j] * suf);
                            suf *= th[j];
                            const int s = sx ^ static_cast<int>((neg >> j) & 1);
                            (cg + j * G)[lane] = s ? -mag : mag;
                        }
                    }
                }
            }
        }
    }
}

// The unrolled slot count of the check pass for a largest check degree d:
// every slot past a check's degree still costs its running updates, so the
// sizes sit just above common degrees of the codes in use (PEG rows of one
// code differ in degree by at most one or two).
inline int dmax_for(int d) {
    for (int c : {8, 10, 16, 18, 24, 32, 34, 48}) if (d <= c) return c;
    return 64;
}

// Edges of a check whose decision words the stopping test gathers at once.
constexpr int kStopChunk = 24;

// Stopping test of iteration t (Sec. 2: a frame succeeds once z^l = H_l x
// for every matrix l), on the decision words the variable pass wrote: bit k
// of D[g][i] is the decision on bit i of the frame in slot k of group g. One
// thread per check: the XOR of the check's decision words and its syndrome
// word gives, in one 64-bit operation, the frames whose parity differs; they
// are ORed into the group's kUnmet word. The last block to finish then
// settles every group: frames of the running set with no unmet check stop at
// t (ok = 1); on the last iteration (a.flag) the others stop too (ok = 0);
// the running set and the host-visible status become the frames still
// running. Slot s holds frame fid[s] (-1: none).
//
// Compaction (a.nspare > 0): when the running frames fit into at most 3/4 of
// the groups they occupy and at least two iterations remain, the same block
// assigns them, in group and lane order, to consecutive slots of the fewest
// unused spare groups (src[new slot] = old slot, fid moves along, the old
// groups stop running) and leaves the plan in the tail for k_move.
__global__ __launch_bounds__(kBlock) void k_stop_test(const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const uint64_t *__restrict__ zb,
                                                      const uint64_t *__restrict__ D, uint64_t *words,
                                                      uint64_t *status, int32_t *iters_out,
                                                      uint8_t *ok_out, int32_t *fid, int32_t *src,
                                                      StopTail *tail, const Dims a) {
    if (a.live && *a.live == 0) return;  // every frame retired
    __shared__ uint32_t sh_or[2 * kWaves];
    __shared__ uint32_t scan[kBlock];
    __shared__ uint32_t sh_base, sh_R, sh_L;
    __shared__ int sh_last;
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const int64_t total = static_cast<int64_t>(a.ngroups) * a.ntiles;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int g = static_cast<int>(w / a.ntiles);
        const int tile = static_cast<int>(w % a.ntiles);
        const uint64_t run = words[kStride * g + kRun];
        if (run == 0) continue;
        const int r = tile * kBlock + static_cast<int>(threadIdx.x);
        uint64_t unmet = 0;
        if (r < a.M) {
            const uint64_t *Dg = D + static_cast<size_t>(g) * a.n;
            uint64_t par = zb[static_cast<size_t>(g) * a.M + r];
            const int e1 = row_ptr[r + 1];
            // indices, then words, kStopChunk at a time (col is padded past E)
            for (int e = row_ptr[r]; e < e1; e += kStopChunk) {
                int v[kStopChunk];
#pragma unroll
                for (int j = 0; j < kStopChunk; ++j) v[j] = col[e + j];
                uint64_t dw[kStopChunk];
#pragma unroll
                for (int j = 0; j < kStopChunk; ++j) dw[j] = e + j < e1 ? Dg[v[j]] : 0;
#pragma unroll
                for (int j = 0; j < kStopChunk; ++j) par ^= dw[j];
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
            uint64_t b = 0;
            for (int i = 0; i < kWaves; ++i)
                b |= static_cast<uint64_t>(sh_or[2 * i]) | (static_cast<uint64_t>(sh_or[2 * i + 1]) << 32);
            or_unmet(&words[kStride * g + kUnmet], b);
        }
        __syncthreads();
    }
    // the last block to arrive settles the groups
    if (threadIdx.x == 0) {
        __threadfence();
        sh_last = atomicAdd(&tail->done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!sh_last) return;
    __threadfence();
    for (int s = threadIdx.x; s < a.ngroups * G; s += kBlock) {
        const int g = s / G, k = s % G;
        const uint64_t run = __hip_atomic_load(&words[kStride * g + kRun], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        if (!((run >> k) & 1)) continue;
        const uint64_t un = __hip_atomic_load(&words[kStride * g + kUnmet], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        const bool met = !((un >> k) & 1);
        if (met || a.flag) {
            const int f = fid[s];
            iters_out[f] = a.t;
            ok_out[f] = met ? 1 : 0;
        }
    }
    if (threadIdx.x == 0) {
        sh_R = 0;
        sh_L = 0;
    }
    __syncthreads();
    for (int g = threadIdx.x; g < a.ngroups; g += kBlock) {
        const uint64_t run = __hip_atomic_load(&words[kStride * g + kRun], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t un = __hip_atomic_load(&words[kStride * g + kUnmet], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t next = a.flag ? 0 : (run & un);
        words[kStride * g + kRun] = next;
        words[kStride * g + kUnmet] = 0;
        if (next) {
            atomicAdd(&sh_R, static_cast<uint32_t>(__popcll(next)));
            atomicAdd(&sh_L, 1u);
        }
    }
    __syncthreads();
    // compaction plan
    const uint32_t R = sh_R, L = sh_L, K = (R + G - 1) / G;
    const uint32_t used = tail->spare_used;
    const bool compact = a.nspare > 0 && !a.flag && a.t <= a.T - 2 && L >= 2 && 4 * K <= 3 * L &&
                         used + K <= static_cast<uint32_t>(a.nspare);
    const int first_new = a.spare0 + static_cast<int>(used);
    if (compact) {
        if (threadIdx.x == 0) sh_base = 0;
        __syncthreads();
        for (int c0 = 0; c0 < a.ngroups; c0 += kBlock) {
            const int g = c0 + static_cast<int>(threadIdx.x);
            const uint64_t run = g < a.ngroups ? words[kStride * g + kRun] : 0;
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
            for (uint64_t rr = run; rr && k < K * G; rr &= rr - 1) {
                const int l = __ffsll(static_cast<unsigned long long>(rr)) - 1;
                const size_t from = static_cast<size_t>(g) * G + l;
                const size_t to = static_cast<size_t>(first_new) * G + k;
                src[to] = static_cast<int32_t>(from);
                fid[to] = fid[from];
                fid[from] = -1;
                ++k;
            }
            if (run) words[kStride * g + kRun] = 0;
            __syncthreads();
            if (threadIdx.x == kBlock - 1) sh_base += scan[kBlock - 1];
            __syncthreads();
        }
        for (uint32_t j = threadIdx.x; j < K * G; j += kBlock)
            if (j >= R) src[static_cast<size_t>(first_new) * G + j] = -1;
        for (uint32_t j = threadIdx.x; j < K; j += kBlock) {
            const uint32_t lo = j * G, cnt = R - lo >= static_cast<uint32_t>(G) ? G : R - lo;
            words[kStride * (first_new + j) + kRun] = cnt >= static_cast<uint32_t>(G) ? ~0ull : ((1ull << cnt) - 1ull);
        }
        __syncthreads();
    }
    for (int g = threadIdx.x; g < a.ngroups; g += kBlock)
        __hip_atomic_store(&status[g], words[kStride * g + kRun], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (threadIdx.x == 0) {
        tail->move_first = first_new;
        tail->move_count = compact ? static_cast<int32_t>(K) : 0;
        if (compact) tail->spare_used = used + K;
        tail->live = R;
        tail->done = 0;
    }
}

// Rows of one k_move work item (kMoveRows / kWaves per wave, all loads of a
// wave issued before its stores).
constexpr int kMoveRows = 64;
constexpr int kMovePerWave = kMoveRows / kWaves;

// Fills the groups the last stopping test's compaction planned (none: the
// kernel does nothing): rows of c (E), L and lambda (n each) and syndrome
// words (M), each lane from its source slot src[]. With the channel given as
// bits (lam null), Bob's bit words (n, after the syndrome words) and the
// per-slot magnitudes move instead of the lambda rows; a compressed check
// state (cs, kStateRows rows per check) and stored per-matrix sums (ps, u
// rows per variable) move with the messages. Work items are runs of
// kMoveRows rows of one region of one group. With H the messages are
// binary16 (two bytes per slot) and there is no state or stored sum.
template <typename T, bool H = false>
__global__ __launch_bounds__(kBlock) void k_move(T *c, T *Lp, T *lam, uint64_t *zb, uint64_t *yb, T *ymag,
                                                 T *cs, T *ps, int32_t prows, const int32_t *src,
                                                 const StopTail *tail, int64_t E, int32_t n, int32_t M) {
    const int count = tail->move_count, first = tail->move_first;
    if (count == 0) return;
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const int64_t nw = M + (yb ? n : 0);  // word rows: syndromes, then Bob's bits
    // rows of one value per lane: messages (E), then the compressed check
    // state if there is one (kStateRows per check; 4-byte words moved as T),
    // then the stored per-matrix sums and posteriors if there are (prows
    // per variable)
    const int64_t ns = cs ? static_cast<int64_t>(kStateRows) * M : 0;
    const int64_t np = ps ? static_cast<int64_t>(prows) * n : 0;
    const int64_t nc = E + ns + np;
    const int64_t ic = (nc + kMoveRows - 1) / kMoveRows, il = (n + kMoveRows - 1) / kMoveRows,
                  iz = (nw + kMoveRows - 1) / kMoveRows, per_group = ic + il + iz;
    for (int64_t w = blockIdx.x; w < count * per_group; w += gridDim.x) {
        const int64_t g = first + w / per_group;
        int64_t item = w % per_group;
        const int32_t s = src[g * G + lane];
        const bool has = s >= 0;
        const int64_t sg = has ? s / G : g, sl = has ? s % G : 0;
        if (H && item < ic) {
            const int64_t r0 = item * kMoveRows + wave * kMovePerWave;
            uint16_t *ch = reinterpret_cast<uint16_t *>(c);
            uint16_t v[kMovePerWave];
#pragma unroll
            for (int j = 0; j < kMovePerWave; ++j) {
                const int64_t r = r0 + j;
                if (has && r < E) v[j] = ch[(sg * E + r) * G + sl];
            }
#pragma unroll
            for (int j = 0; j < kMovePerWave; ++j) {
                const int64_t r = r0 + j;
                if (has && r < E) ch[(g * E + r) * G + lane] = v[j];
            }
        } else if (item < ic) {
            const int64_t r0 = item * kMoveRows + wave * kMovePerWave;
            // row r of a group: its array, rows per group and row within
            auto at = [&](int64_t grp, int64_t r) -> T * {
                if (r < E) return c + (grp * E + r) * G;
                if (r < E + ns) return cs + (grp * ns + r - E) * G;
                return ps + (grp * np + r - E - ns) * G;
            };
            T v[kMovePerWave];
#pragma unroll
            for (int j = 0; j < kMovePerWave; ++j) {
                const int64_t r = r0 + j;
                if (has && r < nc) v[j] = at(sg, r)[sl];
            }
#pragma unroll
            for (int j = 0; j < kMovePerWave; ++j) {
                const int64_t r = r0 + j;
                if (has && r < nc) at(g, r)[lane] = v[j];
            }
        } else if ((item -= ic) < il) {
            const int64_t r0 = item * kMoveRows + wave * kMovePerWave;
            if (ymag && item == 0 && wave == 0 && has) ymag[g * G + lane] = ymag[sg * G + sl];
            T v[kMovePerWave], u[kMovePerWave];
#pragma unroll
            for (int j = 0; j < kMovePerWave; ++j) {
                if (has && r0 + j < n) {
                    v[j] = Lp[(sg * n + r0 + j) * G + sl];
                    if (lam) u[j] = lam[(sg * n + r0 + j) * G + sl];
                }
            }
#pragma unroll
            for (int j = 0; j < kMovePerWave; ++j) {
                if (has && r0 + j < n) {
                    Lp[(g * n + r0 + j) * G + lane] = v[j];
                    if (lam) lam[(g * n + r0 + j) * G + lane] = u[j];
                }
            }
        } else {
            item -= il;
            const int64_t r0 = item * kMoveRows + wave * kMovePerWave;
            uint64_t v[kMovePerWave];
#pragma unroll
            for (int j = 0; j < kMovePerWave; ++j) {
                const int64_t r = r0 + j;
                v[j] = !has || r >= nw ? 0 : r < M ? zb[sg * M + r] : yb[sg * n + (r - M)];
            }
#pragma unroll
            for (int j = 0; j < kMovePerWave; ++j) {
                const int64_t r = r0 + j;
                const uint64_t bits = __ballot((v[j] >> sl) & 1);
                if (lane == 0 && r < nw) {
                    if (r < M)
                        zb[g * M + r] = bits;
                    else
                        yb[g * n + (r - M)] = bits;
                }
            }
        }
    }
}

// [group][n][64] -> bits and L rows [frame][n], from every slot that holds a
// frame (fid >= 0) in its final state. Block (x, k): 64 variables of group
// k (launch_output_slots splits the groups over grids of at most 65535).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_output_slots(const T *Lp, const int32_t *fid, uint8_t *bits,
                                                         T *llr_out, int32_t n) {
    __shared__ T tile[64][65];
    __shared__ int32_t f_of[64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int k = blockIdx.y, i0 = blockIdx.x * 64;
    if (threadIdx.x < 64) f_of[threadIdx.x] = fid[static_cast<size_t>(k) * G + threadIdx.x];
    __syncthreads();
    bool any = false;
    for (int j = 0; j < 64; ++j) any |= f_of[j] >= 0;
    if (!any) return;  // uniform: an unused or vacated group
    for (int iy = ty; iy < 64; iy += kWaves) {
        const int i = i0 + iy;
        tile[iy][tx] = i < n ? Lp[(static_cast<size_t>(k) * n + i) * G + tx] : T(0);
    }
    __syncthreads();
    for (int fy = ty; fy < 64; fy += kWaves) {
        const int f = f_of[fy], i = i0 + tx;
        if (f < 0 || i >= n) continue;
        const T v = tile[tx][fy];
        const size_t o = static_cast<size_t>(f) * n + i;
        if (bits) bits[o] = v < T(0) ? 1 : 0;
        if (llr_out) llr_out[o] = v;
    }
}

// Variable-node pass, eq. (2) with its nesting: L = lambda + the sum, over
// the matrices in order, of each matrix's check messages at the variable
// (summed from 0 in check order). var_edge is the flagged list: an entry
// with bit 31 set starts the next matrix's run of the variable's edges, where
// the running matrix sum is added to L and restarted. Each wave takes VPW
// variables of degree at most DV and issues all their gathers before summing
// any. D, if not null, receives the decision word of
// each variable (bit k set when frame 64g+k decides 1, i.e. L < 0; frames
// not running leave 0).
template <typename T, int DV, int VPW, bool BITS = false>
__global__ __launch_bounds__(kBlock) void k_variable(
    const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_edge,
    const T *__restrict__ c, const T *__restrict__ lam, T *__restrict__ Lp,
    const uint64_t *__restrict__ act, uint64_t *__restrict__ D, const Dims a) {
    if (a.live && *a.live == 0) return;  // every frame retired
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const int64_t total = static_cast<int64_t>(a.ngroups) * a.ntiles;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int gw = static_cast<int>(w / a.ntiles);
        const int g = a.reverse ? a.ngroups - 1 - gw : gw;
        const int tile = static_cast<int>(w % a.ntiles);
        const uint64_t run = act[kStride * g + kRun];
        if (run == 0) continue;
        const bool on = (run >> lane) & 1;
        const size_t gb = static_cast<size_t>(g) * a.n * G;
        const T *cg = c + static_cast<size_t>(g) * a.E * G;
        const uint64_t *yg = BITS ? a.ybits + static_cast<size_t>(g) * a.n : nullptr;
        const T ym = BITS ? static_cast<const T *>(a.ymag)[static_cast<size_t>(g) * G + lane] : T(0);
        int i[VPW], k0[VPW], deg[VPW];
        bool in[VPW];
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            i[v] = (tile * VPW + v) * kWaves + wave;
            in[v] = i[v] < a.n;
            const int ii = in[v] ? i[v] : a.n - 1;
            k0[v] = var_ptr[ii];
            deg[v] = in[v] ? var_ptr[ii + 1] - k0[v] : 0;
        }
        T x[VPW][DV], s[VPW];
        if (on) {
            // emax >= 0 restricts the sum to stacked edges below it: the
            // matrices whose check messages exist so far in the first
            // iteration of the matrix-serial schedule
            const int64_t lim = a.emax < 0 ? INT64_MAX : a.emax;
            int ev[VPW][DV];
            bool fl[VPW][DV];
            uint32_t yh[VPW];
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
#pragma unroll
                for (int j = 0; j < DV; ++j) {
                    const int raw = var_edge[k0[v] + j];
                    fl[v][j] = raw < 0;
                    ev[v][j] = raw & 0x7fffffff;
                }
                if constexpr (BITS)
                    yh[v] = in[v] ? bit_half(yg, i[v], lane) : 0u;
                else
                    s[v] = in[v] ? (lam + gb + static_cast<size_t>(i[v]) * G)[lane] : T(0);
#pragma unroll
                for (int j = 0; j < DV; ++j)
                    if (j < deg[v] && ev[v][j] < lim) x[v][j] = (cg + static_cast<size_t>(ev[v][j]) * G)[lane];
            }
            if constexpr (BITS) {
#pragma unroll
                for (int v = 0; v < VPW; ++v) s[v] = in[v] ? lam_of_half(yh[v], lane, ym) : T(0);
            }
            // independent decoders: each matrix's posterior lambda + its sum
            T *lmg = static_cast<T *>(a.lm);
            if (lmg) lmg += static_cast<size_t>(g) * a.prows * a.n * G;
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                T acc = T(0);  // the running matrix's sum
                const T lam_v = s[v];
                int mrun = 0;  // the running matrix
                bool any = false;
#pragma unroll
                for (int j = 0; j < DV; ++j) {
                    if (j < deg[v] && ev[v][j] < lim) {
                        if (fl[v][j]) {
                            s[v] += acc;
                            if (lmg && in[v])
                                (lmg + (static_cast<size_t>(mrun) * a.n + i[v]) * G)[lane] = lam_v + acc;
                            acc = T(0);
                        }
                        if (lmg && (fl[v][j] || !any))
                            mrun = (ev[v][j] >= a.emat[0]) + (ev[v][j] >= a.emat[1]) + (ev[v][j] >= a.emat[2]);
                        acc += x[v][j];
                        any = true;
                    }
                }
                if (any) {
                    s[v] += acc;
                    if (lmg && in[v]) (lmg + (static_cast<size_t>(mrun) * a.n + i[v]) * G)[lane] = lam_v + acc;
                }
                if (in[v]) (Lp + gb + static_cast<size_t>(i[v]) * G)[lane] = s[v];
            }
        }
        if (D) {
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                const uint64_t bits = __ballot(on && in[v] && s[v] < T(0));
                if (lane == 0 && in[v]) D[static_cast<size_t>(g) * a.n + i[v]] = bits;
            }
        }
    }
}

// The variable pass of eq. (2) for FP32 flooding with the stacked graph
// (and the matrix-serial schedule of one matrix), specialised for
// instruction count. It runs over one degree class of variables [vbeg,
// vend), whose degrees fit DV slots, so few slots are spent past a
// variable's degree; each variable's matrix runs come as one precomputed
// bitmask instead of a flag per edge; the edge indices are scalar loads
// (one wave-uniform list per variable: a vector load read back lane by lane
// would make every item wait for the previous item's stores). Its cursor
// walks only the work items of groups with running frames. Same
// summation as k_variable, so the same results bit for bit.
template <int DV, int VPW, bool BITS, bool H = false>
__global__ __launch_bounds__(kBlock) void k_variable_fast(
    const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_edge,
    const float *__restrict__ c, const float *__restrict__ lam, float *__restrict__ Lp,
    const uint64_t *__restrict__ act, uint64_t *__restrict__ D, const Dims a) {
    if (a.live && *a.live == 0) return;  // every frame retired
    const unsigned lane = lane_id();
    const int wave = wave_id();
    __shared__ uint32_t live[kLiveWords];
    load_live(live, act, a.ngroups);
    // total < 2^31 (the host checks): a 32-bit cursor over the block's work
    // items of running groups
    const uint32_t tot = static_cast<uint32_t>(static_cast<int64_t>(a.ngroups) * a.ntiles);
    const uint32_t nt = static_cast<uint32_t>(a.ntiles);
    auto group = [&](int gw) { return a.reverse ? a.ngroups - 1 - gw : gw; };
    for (uint32_t w = live_item(blockIdx.x, tot, nt, live, group); w < tot;
         w = live_item(w + gridDim.x, tot, nt, live, group)) {
        const int gw = static_cast<int>(w / nt);
        const int g = group(gw);
        const int tile = static_cast<int>(w % nt);
        const uint64_t run = act[kStride * g + kRun];
        const bool on = (run >> lane) & 1;
        const size_t gb = static_cast<size_t>(g) * a.n * G;
        const float *cg = msg_at<H>(c, static_cast<size_t>(g) * a.E * G);
        int i[VPW], k0[VPW], deg[VPW];
        bool in[VPW];
        float x[VPW][DV], s[VPW];
        uint32_t yh[VPW];
        uint64_t rs[VPW];
        const uint64_t *yg = BITS ? a.ybits + static_cast<size_t>(g) * a.n : nullptr;
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            i[v] = a.vbeg + (tile * kWaves + wave) * VPW + v;
            in[v] = i[v] < a.vend;
            const int ii = in[v] ? i[v] : a.vend - 1;
            k0[v] = var_ptr[ii];
            deg[v] = in[v] ? var_ptr[ii + 1] - k0[v] : 0;
            rs[v] = a.runs[ii];
        }
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            if constexpr (BITS)
                yh[v] = in[v] ? bit_half(yg, i[v], lane) : 0u;
            else
                s[v] = in[v] ? (lam + gb + static_cast<size_t>(i[v]) * G)[lane] : 0.0f;
#pragma unroll
            for (int j = 0; j < DV; ++j) {
                if (j < deg[v]) {
                    const size_t at = static_cast<size_t>(var_edge[k0[v] + j]) * G + lane;
                    // binary16: the raw bits now, converted in the sum below
                    // (converting here would wait for each load in turn).
                    // Non-temporal: each message row is read once per pass,
                    // and L, written here, is gathered by the next check pass.
                    if constexpr (H)
                        x[v][j] = __uint_as_float(static_cast<uint32_t>(
                            __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(cg) + at)));
                    else
                        x[v][j] = __builtin_nontemporal_load(cg + at);
                }
            }
        }
        if constexpr (BITS) {
            const float ym = static_cast<const float *>(a.ymag)[static_cast<size_t>(g) * G + lane];
#pragma unroll
            for (int v = 0; v < VPW; ++v) s[v] = in[v] ? lam_of_half(yh[v], lane, ym) : 0.0f;
        }
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            float acc = 0.0f;  // the running matrix's sum
#pragma unroll
            for (int j = 0; j < DV; ++j) {
                if (j < deg[v]) {
                    if ((rs[v] >> j) & 1) {
                        s[v] += acc;
                        acc = 0.0f;
                    }
                    if constexpr (H)
                        acc += static_cast<float>(
                            __builtin_bit_cast(_Float16, static_cast<uint16_t>(__float_as_uint(x[v][j]))));
                    else
                        acc += x[v][j];
                }
            }
            if (deg[v] > 0) s[v] += acc;
            if (in[v] && on) (Lp + gb + static_cast<size_t>(i[v]) * G)[lane] = s[v];
        }
        if (D) {
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                const uint64_t bits = __ballot(on && in[v] && s[v] < 0.0f);
                if (lane == 0 && in[v]) D[static_cast<size_t>(g) * a.n + i[v]] = bits;
            }
        }
    }
}

// The degree classes of k_variable_fast: slots DV and variables per wave.
using VarFastFn = void (*)(const int32_t *, const int32_t *, const float *, const float *, float *,
                           const uint64_t *, uint64_t *, Dims);
template <bool BITS, bool H = false>
VarFastFn variable_fast_kernel(int dv, int *vars_per_tile) {
    if (dv <= 8) { *vars_per_tile = 8 * kWaves; return &k_variable_fast<8, 8, BITS, H>; }
    if (dv <= 12) { *vars_per_tile = 5 * kWaves; return &k_variable_fast<12, 5, BITS, H>; }
    if (dv <= 16) { *vars_per_tile = 4 * kWaves; return &k_variable_fast<16, 4, BITS, H>; }
    if (dv <= 32) { *vars_per_tile = 2 * kWaves; return &k_variable_fast<32, 2, BITS, H>; }
    *vars_per_tile = kWaves;
    return &k_variable_fast<64, 1, BITS, H>;
}

// The first iteration in closed form, when the channel is Bob's bits. Every
// lambda of a frame then has the same magnitude |ym|, so the first check
// pass's message from slot j of a check of degree d has a magnitude that
// depends only on (d, j) and the frame, and its sign is the check's syndrome
// bit times the signs of the check's other lambdas: S_r XOR s_j, with S_r the
// syndrome bit XOR every lambda sign bit of the check (its parity word) and
// s_j the sign bit of slot j's lambda. So that pass need not run: the
// variable pass of the first iteration and the check pass of the second
// rebuild each message from the table and two bits instead of moving the
// messages through HBM.
//
// k_first_table forms the magnitudes for every degree up to the code's
// largest, for each frame, with the operations of the check pass from bits
// in the same order (sum-product: the complements' prefix and suffix chains,
// merged per slot; min-sum: alpha times the smaller of |ym| and the clip,
// the second minimum +inf for a degree-1 check), so a rebuilt message
// equals the stored one bit for bit. With H each entry is rounded to
// binary16, as a stored message would be (the rounding is symmetric in the
// sign). Row r of group g, lane k: slot j of degree d in the frame of slot
// k, with rowdj[r] = (d << 8) | j (a row per slot of every check degree of
// the code).
template <int ALGO, bool H>
__device__ __forceinline__ void first_entry(float *__restrict__ tab, const uint32_t *__restrict__ rowdj,
                                            const Dims &a, int g, int idx) {
#pragma clang fp contract(off)  // as in first_mags
    const int row = idx / G, lane = idx % G;
    const int d = static_cast<int>(rowdj[row] >> 8), j = static_cast<int>(rowdj[row] & 0xffu), k = d - 1 - j;
    const float ym = static_cast<const float *>(a.ymag)[static_cast<size_t>(g) * G + lane];
    const float clip = static_cast<float>(a.clip);
    uint32_t bits;
    if constexpr (ALGO == kNMS) {
        const float alpha = static_cast<float>(a.alpha);
        const float m1 = fminf(fabsf(ym), clip);
        const float m2 = d >= 2 ? m1 : INFINITY;
        bits = __float_as_uint(j == 0 ? alpha * m2 : alpha * m1);
    } else {
        const float e = tanh_complement(fminf(fabsf(ym), clip));
        float run = 0.0f, pj = 0.0f, pk = 0.0f;
        for (int i = 0; i <= max(j, k); ++i) {
            if (i == j) pj = run;
            if (i == k) pk = run;
            run = fmaf(-run, e, run + e);
        }
        bits = __float_as_uint(atanh2_of_complement(fmaf(-pj, pk, pj + pk))) & 0x7fffffffu;
    }
    if constexpr (H) bits = __float_as_uint(static_cast<float>(static_cast<_Float16>(__uint_as_float(bits))));
    tab[(static_cast<size_t>(g) * a.mrows + row) * G + lane] = __uint_as_float(bits);
}

template <int ALGO, bool H>
__global__ __launch_bounds__(kBlock) void k_first_table(float *__restrict__ tab, const uint32_t *__restrict__ rowdj,
                                                        const Dims a) {
    const int64_t total = static_cast<int64_t>(a.ngroups) * a.mrows * G;
    for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
         idx += static_cast<int64_t>(gridDim.x) * kBlock)
        first_entry<ALGO, H>(tab, rowdj, a, static_cast<int>(idx / (static_cast<int64_t>(a.mrows) * G)),
                             static_cast<int>(idx % (static_cast<int64_t>(a.mrows) * G)));
}

// The checks' parity words of the first iteration: S[g][r] = z_r XOR the
// lambda sign bits of the check's variables, for the 64 frames at once. The
// sign bit of lambda = (1 - 2y)|ym| as the check pass sees it (after adding
// +0) is y XOR flip where lambda is nonzero and 0 where it is zero, with
// flip the sign of ym; per group the lanes with flip and with a nonzero ym
// are two masks (smask[g][0], [1]), formed here by a ballot. One thread per
// check, as the stopping test; only groups holding frames.
__global__ __launch_bounds__(kBlock) void k_first_parity(const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const uint64_t *__restrict__ zb,
                                                         const uint64_t *__restrict__ act,
                                                         uint64_t *__restrict__ spar, uint64_t *__restrict__ smask,
                                                         const Dims a) {
    const unsigned lane = lane_id();
    const int64_t total = static_cast<int64_t>(a.ngroups) * a.ntiles;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int g = static_cast<int>(w / a.ntiles);
        const int tile = static_cast<int>(w % a.ntiles);
        if (act[kStride * g + kRun] == 0) continue;
        const float ym = static_cast<const float *>(a.ymag)[static_cast<size_t>(g) * G + lane];
        const uint64_t flip = __ballot(__float_as_uint(ym) >> 31);
        const uint64_t nz = __ballot(ym != 0.0f);
        if (tile == 0 && threadIdx.x == 0) {
            smask[2 * static_cast<size_t>(g)] = flip;
            smask[2 * static_cast<size_t>(g) + 1] = nz;
        }
        const int r = tile * kBlock + static_cast<int>(threadIdx.x);
        if (r >= a.M) continue;
        const uint64_t *yg = a.ybits + static_cast<size_t>(g) * a.n;
        uint64_t par = 0;
        const int e0 = row_ptr[r], e1 = row_ptr[r + 1];
        // indices, then words, kStopChunk at a time (col is padded past E)
        for (int e = e0; e < e1; e += kStopChunk) {
            int v[kStopChunk];
#pragma unroll
            for (int j = 0; j < kStopChunk; ++j) v[j] = col[e + j];
            uint64_t yw[kStopChunk];
#pragma unroll
            for (int j = 0; j < kStopChunk; ++j) yw[j] = e + j < e1 ? yg[v[j]] : 0;
#pragma unroll
            for (int j = 0; j < kStopChunk; ++j) par ^= yw[j];
        }
        // XOR over the edges of (y XOR flip) AND nz
        if ((e1 - e0) & 1) par ^= flip;
        spar[static_cast<size_t>(g) * a.M + r] = zb[static_cast<size_t>(g) * a.M + r] ^ (par & nz);
    }
}

// Variable pass of the first iteration in closed form: L^1 = lambda + the
// first check pass's messages, each rebuilt from its table entry (row from
// var_rt) and its sign S_r XOR s_v (S_r gathered from the parity words, s_v
// the variable's own lambda sign bit), summed exactly as k_variable_fast
// sums the stored messages (so L^1 and the decision words are the same, bit
// for bit). Per edge two gathers from cache (the table and the parity words
// are small: a 256-byte table row and 8 bytes per wave) in place of one
// 256-byte message row from HBM; half as many variables per wave as
// k_variable_fast for the same registers. (Staging a group's table in LDS
// was slower: the copy each time a block's work moves to another group cost
// more than the cache reads it saved.)
template <int DV, int VPW>
__global__ __launch_bounds__(kBlock) void k_variable_first(const int32_t *__restrict__ var_ptr,
                                                           float *__restrict__ Lp, const uint64_t *__restrict__ act,
                                                           uint64_t *__restrict__ D, const Dims a) {
    if (a.live && *a.live == 0) return;  // every frame retired
    const unsigned lane = lane_id();
    const int wave = wave_id();
    __shared__ uint32_t live[kLiveWords];
    load_live(live, act, a.ngroups);
    const uint32_t tot = static_cast<uint32_t>(static_cast<int64_t>(a.ngroups) * a.ntiles);
    const uint32_t nt = static_cast<uint32_t>(a.ntiles);
    auto group = [&](int gw) { return a.reverse ? a.ngroups - 1 - gw : gw; };
    for (uint32_t w = live_item(blockIdx.x, tot, nt, live, group); w < tot;
         w = live_item(w + gridDim.x, tot, nt, live, group)) {
        const int g = group(static_cast<int>(w / nt));
        const int tile = static_cast<int>(w % nt);
        const uint64_t run = act[kStride * g + kRun];
        const bool on = (run >> lane) & 1;
        const size_t gb = static_cast<size_t>(g) * a.n * G;
        const uint32_t *tg = reinterpret_cast<const uint32_t *>(a.mtab) + static_cast<size_t>(g) * a.mrows * G;
        const uint32_t *sg = reinterpret_cast<const uint32_t *>(a.spar + static_cast<size_t>(g) * a.M);
        const uint64_t *yg = a.ybits + static_cast<size_t>(g) * a.n;
        int i[VPW], k0[VPW], deg[VPW];
        bool in[VPW];
        uint32_t m[VPW][DV], sp[VPW][DV], yh[VPW];
        uint64_t rs[VPW];
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            i[v] = a.vbeg + (tile * kWaves + wave) * VPW + v;
            in[v] = i[v] < a.vend;
            const int ii = in[v] ? i[v] : a.vend - 1;
            k0[v] = var_ptr[ii];
            deg[v] = in[v] ? var_ptr[ii + 1] - k0[v] : 0;
            rs[v] = a.runs[ii];
        }
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            yh[v] = in[v] ? bit_half(yg, i[v], lane) : 0u;
#pragma unroll
            for (int j = 0; j < DV; ++j) {
                if (j < deg[v]) {
                    const uint32_t rt = a.var_rt[k0[v] + j];
                    m[v][j] = tg[(rt & ((1u << kRtShift) - 1u)) * G + lane];
                    sp[v][j] = sg[(rt >> kRtShift) * 2 + (lane >> 5)];
                }
            }
        }
        const float ym = static_cast<const float *>(a.ymag)[static_cast<size_t>(g) * G + lane];
        const uint32_t flip = __float_as_uint(ym) >> 31, nz = ym != 0.0f ? 1u : 0u;
        float s[VPW];
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            s[v] = in[v] ? lam_of_half(yh[v], lane, ym) : 0.0f;
            const uint32_t sv = ((yh[v] >> (lane & 31u)) ^ flip) & nz & 1u;
            float acc = 0.0f;  // the running matrix's sum
#pragma unroll
            for (int j = 0; j < DV; ++j) {
                if (j < deg[v]) {
                    if ((rs[v] >> j) & 1) {
                        s[v] += acc;
                        acc = 0.0f;
                    }
                    const uint32_t sb = ((sp[v][j] >> (lane & 31u)) & 1u) ^ sv;
                    acc += __uint_as_float(m[v][j] | (sb << 31));
                }
            }
            if (deg[v] > 0) s[v] += acc;
            if (in[v] && on) (Lp + gb + static_cast<size_t>(i[v]) * G)[lane] = s[v];
        }
        if (D) {
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                const uint64_t bits = __ballot(on && in[v] && s[v] < 0.0f);
                if (lane == 0 && in[v]) D[static_cast<size_t>(g) * a.n + i[v]] = bits;
            }
        }
    }
}

using VarFirstFn = void (*)(const int32_t *, float *, const uint64_t *, uint64_t *, Dims);
inline VarFirstFn variable_first_kernel(int dv, int *vars_per_tile) {
    if (dv <= 8) { *vars_per_tile = 4 * kWaves; return &k_variable_first<8, 4>; }
    if (dv <= 12) { *vars_per_tile = 3 * kWaves; return &k_variable_first<12, 3>; }
    if (dv <= 16) { *vars_per_tile = 2 * kWaves; return &k_variable_first<16, 2>; }
    if (dv <= 32) { *vars_per_tile = kWaves; return &k_variable_first<32, 1>; }
    *vars_per_tile = kWaves;
    return &k_variable_first<64, 1>;
}

// Variable pass of phase l of the matrix-serial schedule, for codes of at
// most kPhaseMaxU matrices. Only matrix l's messages changed since the last
// variable pass, so only they are read: their sum at each variable (from 0,
// in check order) is formed and stored, and L = lambda + the per-matrix sums
// of every matrix in order, the others read back from where earlier passes
// stored them. This is eq. (2) with the nesting the full sum uses, so L is
// the same, bit for bit, as summing every message again. A matrix with no
// edge at the variable adds nothing, nor, in the first iteration, does a
// matrix not visited yet (its messages are still zero).
constexpr int kPhaseMaxU = 4;

template <typename T, int DV, int VPW, bool BITS = false>
__global__ __launch_bounds__(kBlock) void k_variable_phase(
    const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_edge,
    const T *__restrict__ c, const T *__restrict__ lam, T *__restrict__ Lp,
    const uint64_t *__restrict__ act, uint64_t *__restrict__ D, const Dims a) {
    if (a.live && *a.live == 0) return;  // every frame retired
    (void)var_ptr;
    const unsigned lane = lane_id();
    const int wave = wave_id();
    const int l = a.phase;
    const int64_t total = static_cast<int64_t>(a.ngroups) * a.ntiles;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int gw = static_cast<int>(w / a.ntiles);
        const int g = a.reverse ? a.ngroups - 1 - gw : gw;
        const int tile = static_cast<int>(w % a.ntiles);
        const uint64_t run = act[kStride * g + kRun];
        if (run == 0) continue;
        const bool on = (run >> lane) & 1;
        const size_t gb = static_cast<size_t>(g) * a.n * G;
        const T *cg = c + static_cast<size_t>(g) * a.E * G;
        T *sg = static_cast<T *>(a.psum) + static_cast<size_t>(g) * a.prows * a.n * G;
        T *lmg = static_cast<T *>(a.lm);
        if (lmg) lmg += static_cast<size_t>(g) * a.prows * a.n * G;
        const uint64_t *yg = BITS ? a.ybits + static_cast<size_t>(g) * a.n : nullptr;
        const T ym = BITS ? static_cast<const T *>(a.ymag)[static_cast<size_t>(g) * G + lane] : T(0);
        int i[VPW], k0[VPW], deg[VPW];
        bool in[VPW];
        int cnt[VPW][kPhaseMaxU];
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            i[v] = (tile * VPW + v) * kWaves + wave;
            in[v] = i[v] < a.n;
            const int ii = in[v] ? i[v] : a.n - 1;
#pragma unroll
            for (int m = 0; m < kPhaseMaxU; ++m)
                cnt[v][m] = m < a.u && in[v] ? a.vmptr[(m + 1) * a.n + ii] - a.vmptr[m * a.n + ii] : 0;
            k0[v] = a.vmptr[l * a.n + ii];
            deg[v] = cnt[v][0];
#pragma unroll
            for (int m = 1; m < kPhaseMaxU; ++m) deg[v] = m == l ? cnt[v][m] : deg[v];
        }
        T x[VPW][DV], s[VPW], part[VPW][kPhaseMaxU];
        if (on) {
            int ev[VPW][DV];
            uint32_t yh[VPW];
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
#pragma unroll
                for (int j = 0; j < DV; ++j) ev[v][j] = var_edge[k0[v] + j];
                if constexpr (BITS)
                    yh[v] = in[v] ? bit_half(yg, i[v], lane) : 0u;
                else
                    s[v] = in[v] ? (lam + gb + static_cast<size_t>(i[v]) * G)[lane] : T(0);
#pragma unroll
                for (int j = 0; j < DV; ++j)
                    if (j < deg[v]) x[v][j] = (cg + static_cast<size_t>(ev[v][j]) * G)[lane];
                // the other matrices' sums, as earlier passes stored them
#pragma unroll
                for (int m = 0; m < kPhaseMaxU; ++m)
                    if (m != l && cnt[v][m] > 0 && (a.t > 1 || m < l))
                        part[v][m] = (sg + (static_cast<size_t>(m) * a.n + i[v]) * G)[lane];
            }
            if constexpr (BITS) {
#pragma unroll
                for (int v = 0; v < VPW; ++v) s[v] = in[v] ? lam_of_half(yh[v], lane, ym) : T(0);
            }
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                T acc = T(0);
                const T lam_v = s[v];
#pragma unroll
                for (int j = 0; j < DV; ++j)
                    if (j < deg[v]) acc += x[v][j];
                // independent decoders: matrix l's posterior
                if (lmg && in[v] && deg[v] > 0)
                    (lmg + (static_cast<size_t>(l) * a.n + i[v]) * G)[lane] = lam_v + acc;
#pragma unroll
                for (int m = 0; m < kPhaseMaxU; ++m) {
                    if (m == l) {
                        if (cnt[v][m] > 0) s[v] += acc;
                    } else if (cnt[v][m] > 0 && (a.t > 1 || m < l)) {
                        s[v] += part[v][m];
                    }
                }
                if (in[v]) {
                    if (deg[v] > 0) (sg + (static_cast<size_t>(l) * a.n + i[v]) * G)[lane] = acc;
                    (Lp + gb + static_cast<size_t>(i[v]) * G)[lane] = s[v];
                }
            }
        }
        if (D) {
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                const uint64_t bits = __ballot(on && in[v] && s[v] < T(0));
                if (lane == 0 && in[v]) D[static_cast<size_t>(g) * a.n + i[v]] = bits;
            }
        }
    }
}

template <typename T, bool BITS = false>
using VarPhaseFn = void (*)(const int32_t *, const int32_t *, const T *, const T *, T *, const uint64_t *,
                            uint64_t *, Dims);

template <typename T, bool BITS = false>
VarPhaseFn<T> variable_phase_kernel(int dmax, int *vars_per_tile) {
    if (dmax <= 4) { *vars_per_tile = 4 * kWaves; return &k_variable_phase<T, 4, 4, BITS>; }
    if (dmax <= 8) { *vars_per_tile = 4 * kWaves; return &k_variable_phase<T, 8, 4, BITS>; }
    if (dmax <= 16) { *vars_per_tile = 2 * kWaves; return &k_variable_phase<T, 16, 2, BITS>; }
    if (dmax <= 32) { *vars_per_tile = kWaves; return &k_variable_phase<T, 32, 1, BITS>; }
    *vars_per_tile = kWaves;
    return &k_variable_phase<T, 64, 1, BITS>;
}

// The variable-pass instance for a joint variable degree up to dmax, and the
// variables one block covers (its tile).
template <typename T>
using VarFn = void (*)(const int32_t *, const int32_t *, const T *, const T *, T *, const uint64_t *,
                       uint64_t *, Dims);

template <typename T, bool BITS = false>
VarFn<T> variable_kernel(int dmax, int *vars_per_tile) {
    if (dmax <= 8) { *vars_per_tile = 4 * kWaves; return &k_variable<T, 8, 4, BITS>; }
    if (dmax <= 16) { *vars_per_tile = 4 * kWaves; return &k_variable<T, 16, 4, BITS>; }
    if (dmax <= 32) { *vars_per_tile = 2 * kWaves; return &k_variable<T, 32, 2, BITS>; }
    *vars_per_tile = kWaves;
    return &k_variable<T, 64, 1, BITS>;
}

// Running set of the plain and unrolled decodes before the first iteration:
// every valid frame of the first ngroups groups (then nspare empty spares);
// the unmet words and the stopping-test counters cleared; fid, if not null,
// maps slot 64g+k to frame 64g+k (-1 past the frames and in the spares).
__global__ void k_init_running(uint64_t *words, uint64_t *status, StopTail *tail, int32_t *fid,
                               int32_t nframes, int32_t ngroups, int32_t nspare) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0 && tail) *tail = StopTail{0, 0, 0, 0, static_cast<uint32_t>(nframes > 0 ? nframes : 0)};
    if (s >= (ngroups + nspare) * G) return;
    const int g = s / G, k = s % G;
    if (fid) fid[s] = g < ngroups && s < nframes ? s : -1;
    if (k) return;
    const int rem = nframes - g * G;
    const uint64_t valid = g >= ngroups ? 0 : rem >= G ? ~0ull : ((1ull << rem) - 1ull);
    words[kStride * g + kRun] = valid;
    words[kStride * g + kUnmet] = 0;
    __hip_atomic_store(&status[g], valid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Per-group masks of the batched decode before the first iteration, by
// iteration parity: iteration 1 reads parity 1; `both` also marks parity 0.
__global__ void k_init_groups(uint64_t *act, uint64_t *uns, uint64_t *status, int32_t nframes,
                              int32_t ngroups, int32_t both = 0) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    const int rem = nframes - g * G;
    const uint64_t valid = rem >= G ? ~0ull : ((1ull << rem) - 1ull);
    act[kStride * g + 1] = valid;
    act[kStride * g + 0] = both ? valid : 0;
    uns[kStride * g + 0] = 0;
    uns[kStride * g + 1] = 0;
    __hip_atomic_store(&status[g], valid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// [F][n] -> [g][n][64] for the channel LLRs, and into Lp as well (the
// initial L) when Lp is not null.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stage_llr(const T *llr, T *lam, T *Lp, int32_t nframes,
                                                      int32_t n) {
    __shared__ T tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int g = blockIdx.y, i0 = blockIdx.x * 64;
    for (int fy = ty; fy < 64; fy += kWaves) {
        const int f = g * G + fy, i = i0 + tx;
        tile[fy][tx] = (f < nframes && i < n) ? llr[static_cast<size_t>(f) * n + i] : T(0);
    }
    __syncthreads();
    for (int iy = ty; iy < 64; iy += kWaves) {
        const int i = i0 + iy;
        if (i < n) {
            const T v = tile[tx][iy];
            const size_t o = (static_cast<size_t>(g) * n + i) * G + tx;
            lam[o] = v;
            if (Lp) Lp[o] = v;
        }
    }
}

// |lambda| = ln((1 - e)/e) of every slot, for frames given as Bob's bits
// (eq. (5)); formed in FP64 and rounded once, as k_llr does. Slots past the
// frames get 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stage_mag(const double *e, T *mag, int32_t nframes, int32_t nslots) {
    const int s = blockIdx.x * kBlock + static_cast<int>(threadIdx.x);
    if (s >= nslots) return;
    T m = T(0);
    if (s < nframes) {
        const double ef = e[s];
        m = static_cast<T>(log((1.0 - ef) / ef));
    }
    mag[s] = m;
}

// [F][M] syndrome bytes -> [g][M] 64-bit lane masks. One thread per check
// gathers its bit of the group's 64 frames; for each frame the block reads
// kBlock consecutive bytes.
__global__ __launch_bounds__(kBlock) void k_stage_synd(const uint8_t *z, uint64_t *zb, int32_t nframes,
                                                       int32_t M) {
    const int g = blockIdx.y;
    const int r = blockIdx.x * kBlock + static_cast<int>(threadIdx.x);
    if (r >= M) return;
    const int nf = min(G, nframes - g * G);
    const uint8_t *zg = z + static_cast<size_t>(g) * G * M + r;
    uint64_t m = 0;
#pragma unroll 16
    for (int k = 0; k < nf; ++k) m |= static_cast<uint64_t>(zg[static_cast<size_t>(k) * M] != 0) << k;
    zb[static_cast<size_t>(g) * M + r] = m;
}

// [g][n][64] -> decided bits [F][n] and L [F][n] (either may be null).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_output(const T *Lp, uint8_t *bits, T *llr_out,
                                                   int32_t nframes, int32_t n) {
    __shared__ T tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int g = blockIdx.y, i0 = blockIdx.x * 64;
    for (int iy = ty; iy < 64; iy += kWaves) {
        const int i = i0 + iy;
        tile[iy][tx] = i < n ? Lp[(static_cast<size_t>(g) * n + i) * G + tx] : T(0);
    }
    __syncthreads();
    for (int fy = ty; fy < 64; fy += kWaves) {
        const int f = g * G + fy, i = i0 + tx;
        if (f < nframes && i < n) {
            const T v = tile[tx][fy];
            const size_t o = static_cast<size_t>(f) * n + i;
            if (bits) bits[o] = v < T(0) ? 1 : 0;
            if (llr_out) llr_out[o] = v;
        }
    }
}

// Channel LLR (1 - 2y) ln((1 - e)/e), computed in FP64. Block (x, f) covers
// kLlrPerBlock consecutive bits of frame f; each thread takes the logarithm
// once and converts kLlrPerThread consecutive bits. VEC (n a multiple of 8,
// rows aligned) moves them as one 8-byte load and 16-byte stores.
constexpr int kLlrPerThread = 8;
constexpr int kLlrPerBlock = kBlock * kLlrPerThread;

template <typename T, bool VEC>
__global__ __launch_bounds__(kBlock) void k_llr(const uint8_t *__restrict__ y,
                                                const double *__restrict__ e, T *__restrict__ out,
                                                int32_t n) {
    const size_t f = blockIdx.y;
    const double ef = e[f];
    const double lam = log((1.0 - ef) / ef);
    const T pos = static_cast<T>(lam), neg = static_cast<T>(-lam);
    const int i0 = blockIdx.x * kLlrPerBlock + static_cast<int>(threadIdx.x) * kLlrPerThread;
    if (i0 >= n) return;
    const uint8_t *yf = y + f * n + i0;
    T *of = out + f * n + i0;
    if constexpr (VEC) {
        const uint2 b = *reinterpret_cast<const uint2 *>(yf);
        T v[kLlrPerThread];
#pragma unroll
        for (int k = 0; k < kLlrPerThread; ++k) {
            const uint32_t w = k < 4 ? b.x : b.y;
            v[k] = ((w >> (8 * (k & 3))) & 0xffu) ? neg : pos;
        }
        constexpr int kPer16 = 16 / static_cast<int>(sizeof(T));
#pragma unroll
        for (int k = 0; k < kLlrPerThread; k += kPer16) {
            if constexpr (sizeof(T) == 4)
                *reinterpret_cast<float4 *>(of + k) = make_float4(v[k], v[k + 1], v[k + 2], v[k + 3]);
            else
                *reinterpret_cast<double2 *>(of + k) = make_double2(v[k], v[k + 1]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kLlrPerThread; ++k)
            if (i0 + k < n) of[k] = yf[k] ? neg : pos;
    }
}

// ---------------------------------------------------------------- host side
int blocks_per_cu(const void *fn) {
    static std::mutex mu;
    static std::unordered_map<const void *, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(fn);
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();  // the query is advisory: fall back to one block per CU
        nb = 1;
    }
    cache[fn] = nb;
    return nb;
}

int grid_for(const mbp_ctx *ctx, const void *fn, int64_t items) {
    const int64_t cap = static_cast<int64_t>(ctx->num_cus) * blocks_per_cu(fn);
    return static_cast<int>(std::max<int64_t>(1, std::min(items, cap)));
}

// k_output_slots over `groups` groups, in launches of at most 65535 groups
// (the grid's y limit).
template <typename T>
void launch_output_slots(const T *Lp, const int32_t *fid, uint8_t *bits, T *llr_out, int32_t n, int64_t groups,
                         hipStream_t stream) {
    constexpr int64_t kMaxY = 65535;
    for (int64_t g0 = 0; g0 < groups; g0 += kMaxY) {
        const int64_t ng = std::min(kMaxY, groups - g0);
        k_output_slots<T><<<dim3((n + 63) / 64, static_cast<unsigned>(ng)), kBlock, 0, stream>>>(
            Lp + g0 * n * G, fid + g0 * G, bits, llr_out, n);
    }
}

struct Timer {
    mbp_ctx *ctx;
    hipStream_t stream;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    size_t used = 0;

    hipError_t event(hipEvent_t *ev) {
        if (used == ctx->timing_events.size()) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            ctx->timing_events.push_back(e);
        }
        *ev = ctx->timing_events[used++];
        return hipSuccess;
    }
    template <typename F>
    hipError_t run(int which, F &&launch) {
        if (!((ctx->profiling >> which) & 1)) {
            launch();
            return hipGetLastError();
        }
        hipEvent_t a, b;
        hipError_t err;
        if ((err = event(&a)) != hipSuccess || (err = event(&b)) != hipSuccess) return err;
        if ((err = hipEventRecord(a, stream)) != hipSuccess) return err;
        launch();
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if ((err = hipEventRecord(b, stream)) != hipSuccess) return err;
        marks.push_back({which, {a, b}});
        return hipSuccess;
    }
    hipError_t collect() {
        for (auto &m : marks) {
            float ms = 0.f;
            hipError_t err = hipEventElapsedTime(&ms, m.second.first, m.second.second);
            if (err != hipSuccess) return err;
            ctx->stats[m.first].launches += 1;
            ctx->stats[m.first].total_ms += ms;
        }
        marks.clear();
        return hipSuccess;
    }
};

size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

int ensure_workspace(mbp_ctx *ctx, size_t bytes) {
    if (ctx->ws_bytes >= bytes) return MBP_OK;
    if (ctx->ws) {
        hipError_t e = hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
    }
    hipError_t e = hipMalloc(&ctx->ws, bytes);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        return hip_fail(e, "hipMalloc(workspace)");
    }
    ctx->ws_bytes = bytes;
    return MBP_OK;
}

int ensure_status(mbp_ctx *ctx, int32_t ngroups) {
    if (ctx->status_cap >= ngroups) return MBP_OK;
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
    ctx->status_host = nullptr;
    ctx->status_dev = nullptr;
    ctx->status_cap = 0;
    const int32_t cap = std::max<int32_t>(ngroups, 64);
    void *p = nullptr;
    hipError_t e = hipHostMalloc(&p, sizeof(uint64_t) * cap, hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(status)");
    void *d = nullptr;
    e = hipHostGetDevicePointer(&d, p, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(p);
        return hip_fail(e, "hipHostGetDevicePointer(status)");
    }
    ctx->status_host = static_cast<uint64_t *>(p);
    ctx->status_dev = static_cast<uint64_t *>(d);
    ctx->status_cap = cap;
    return MBP_OK;
}

}  // namespace
}  // namespace mbp
