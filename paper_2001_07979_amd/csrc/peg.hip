// Progressive edge-growth (PEG) construction of the u parity-check matrices
// on the GPU (mbp_peg_build). The paper builds its matrices with PEG (Sec. 2,
// citing Hu, Eleftheriou and Arnold) and gives no further detail; this is
// the published procedure:
//   - variables are taken one at a time in index order (non-decreasing
//     degree);
//   - a variable's first edge goes to a check of lowest current degree;
//   - each further edge goes to a lowest-degree check among those that a
//     breadth-first expansion of the current graph from the variable reaches
//     last (the farthest level), or, when the expansion stops growing or hits
//     the depth bound, among the checks it never reached;
//   - ties are broken at random from a seeded stream.
// Every edge depends on all earlier ones (the check degrees and the graph the
// search walks), so one workgroup builds one matrix edge by edge and only the
// search inside an edge runs in parallel; the u matrices are built by u
// workgroups at once. The level sets of the search do not depend on the
// order it visits nodes in, and every choice among candidates is made by a
// key that does not either (lowest degree, then a counter-based hash of the
// seed, the edge and the check), so the result depends only on the inputs.
// It is not the host generator's matrix: that one breaks ties by its own
// sequential draws.
#include "mbp_kernels.h"

namespace mbp {
namespace {

constexpr int kPegBlock = 1024;
constexpr int kPegWaves = kPegBlock / 64;
constexpr int kPegTries = 24;  // random picks in a degree bucket before scanning it
constexpr int kPegSegMax = 4096;  // degree buckets held in LDS: cap + 2 at most

// splitmix64's output function (Steele, Lea and Flood, 2014) applied to a
// counter: the k-th value of the stream seeded with `seed`.
__device__ __forceinline__ uint64_t sm64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Per-matrix state, in device memory. Check c's variables are
// adj[c * cap + i], i < len[c] (ascending: variables arrive in index order);
// order[] lists the checks by degree and pos[c] is c's index there; where
// degree d starts in order[] (seg[d]) is kept in LDS by the kernel.
struct PegState {
    const int32_t *var_off;  // [n + 1], shared by the u matrices
    int32_t *var_cnt;        // [n]
    int32_t *var_adj;        // [E]
    int32_t *len;            // [m]
    int32_t *adj;            // [m * cap]
    int32_t *order, *pos;    // [m]
    int32_t *cstamp;         // [m]
    int32_t *vstamp;         // [n]
    int32_t *front, *next;   // [m] each
    int32_t *err;            // 1: a check would exceed cap; 2: no check left for an edge
    uint64_t seed;
};

struct PegArgs {
    PegState st[4];  // filled for blockIdx.x < u; more matrices take more launches
    int32_t n, m, cap, max_depth;
};

// Lowest key over the block (a 64-bit min in LDS); every thread gets it.
__device__ __forceinline__ uint64_t block_min(uint64_t key, uint64_t *sh) {
    if (threadIdx.x == 0) *sh = ~0ull;
    __syncthreads();
    if (key != ~0ull) atomicMin(reinterpret_cast<unsigned long long *>(sh), static_cast<unsigned long long>(key));
    __syncthreads();
    const uint64_t r = *sh;
    __syncthreads();
    return r;
}

// The key of check c as a candidate for edge `edge`: degree first, then a
// 24-bit hash, then the check itself (so equal hashes still order).
__device__ __forceinline__ uint64_t cand_key(const PegState &S, int c, int deg, uint64_t edge) {
    const uint64_t h = sm64_at(S.seed ^ 0x5bd1e9955bd1e995ull, (edge << 32) | static_cast<uint32_t>(c)) >> 40;
    return (static_cast<uint64_t>(deg) << 56) | (h << 32) | static_cast<uint32_t>(c);
}

// Lowest-degree check not reached by the current search (cstamp != stamp):
// first a few random picks in each degree bucket (as a sequential PEG
// would), then the lowest key over the bucket's unreached checks. -1 if
// every check is reached. The degree buckets (seg) and the lowest degree
// with a check (d0) live in LDS, where every thread reads the same values,
// so all take the same path to each barrier.
__device__ int pick_unreached(const PegState &S, int cap, int stamp, uint64_t edge, uint64_t *draw,
                              uint64_t *sh_min, int *sh_pick, const int *seg, int d0) {
    for (int d = d0; d <= cap; ++d) {
        const int lo = seg[d], hi = seg[d + 1];
        if (hi <= lo) continue;
        if (threadIdx.x == 0) {
            int got = -1;
            const uint64_t cnt = static_cast<uint64_t>(hi - lo);
            for (int t = 0; t < kPegTries && got < 0; ++t) {
                const int c = S.order[lo + static_cast<int>(sm64_at(S.seed, (*draw)++) % cnt)];
                if (S.cstamp[c] != stamp) got = c;
            }
            *sh_pick = got;
        }
        __syncthreads();
        const int got = *sh_pick;
        __syncthreads();
        if (got >= 0) return got;
        uint64_t key = ~0ull;
        for (int i = lo + static_cast<int>(threadIdx.x); i < hi; i += kPegBlock) {
            const int c = S.order[i];
            if (S.cstamp[c] != stamp) {
                const uint64_t k = cand_key(S, c, d, edge);
                key = k < key ? k : key;
            }
        }
        const uint64_t best = block_min(key, sh_min);
        if (best != ~0ull) return static_cast<int>(static_cast<uint32_t>(best));
    }
    return -1;
}

// Raise check c's degree by one, keeping order[] sorted by degree, and the
// lowest degree with a check (thread 0).
__device__ void bump_degree(const PegState &S, int c, int *seg, int *d0) {
    const int d = S.len[c];
    const int last = seg[d + 1] - 1;
    const int pc = S.pos[c], other = S.order[last];
    S.order[pc] = other;
    S.pos[other] = pc;
    S.order[last] = c;
    S.pos[c] = last;
    seg[d + 1] = last;
    while (seg[*d0] == seg[*d0 + 1]) ++*d0;
}

__global__ __launch_bounds__(kPegBlock) void k_peg(PegArgs a, int32_t matrix0) {
    const PegState S = a.st[blockIdx.x];
    (void)matrix0;
    const int n = a.n, m = a.m, cap = a.cap;
    const int tid = static_cast<int>(threadIdx.x);
    const int wave = tid >> 6, lane = tid & 63;
    __shared__ uint64_t sh_min;
    __shared__ int sh_pick, sh_nlen, sh_stop, sh_d0;
    __shared__ int seg[kPegSegMax];
    // all checks start at degree 0
    for (int c = tid; c < m; c += kPegBlock) {
        S.order[c] = c;
        S.pos[c] = c;
        S.len[c] = 0;
        S.cstamp[c] = 0;
    }
    for (int i = tid; i < n; i += kPegBlock) {
        S.var_cnt[i] = 0;
        S.vstamp[i] = 0;
    }
    for (int d = tid; d < cap + 2; d += kPegBlock) seg[d] = d == 0 ? 0 : m;
    if (tid == 0) {
        sh_stop = 0;
        sh_d0 = 0;
    }
    __syncthreads();
    int stamp = 0;
    uint64_t edge = 0, draw = 0;  // draw: position in the tie-break stream (thread 0)
    for (int v = 0; v < n; ++v) {
        const int off = S.var_off[v], deg = S.var_off[v + 1] - off;
        for (int k = 0; k < deg; ++k, ++edge) {
            ++stamp;
            int c = -1;
            if (k == 0) {
                c = pick_unreached(S, cap, stamp, edge, &draw, &sh_min, &sh_pick, seg, sh_d0);
            } else {
                // level 0: the variable's checks
                if (tid < k) {
                    const int c0 = S.var_adj[off + tid];
                    S.cstamp[c0] = stamp;
                    S.front[tid] = c0;
                }
                if (tid == 0) {
                    S.vstamp[v] = stamp;
                    sh_nlen = 0;
                }
                int flen = k, count = k;
                int32_t *front = S.front, *next = S.next;
                __syncthreads();
                for (int level = 0;; ++level) {
                    if (a.max_depth >= 0 && level >= a.max_depth) {
                        c = pick_unreached(S, cap, stamp, edge, &draw, &sh_min, &sh_pick, seg, sh_d0);
                        break;
                    }
                    // the next level: unvisited variables of the frontier's
                    // checks, then their unreached checks (a wave per check)
                    for (int fi = wave; fi < flen; fi += kPegWaves) {
                        const int f = front[fi];
                        const int L = S.len[f];
                        for (int i = lane; i < L; i += 64) {
                            const int w = S.adj[static_cast<size_t>(f) * cap + i];
                            if (atomicExch(&S.vstamp[w], stamp) == stamp) continue;
                            const int wo = S.var_off[w], wc = S.var_cnt[w];
                            // the variable's checks eight at a time: all loads,
                            // then all claims, then the pushes, so the round
                            // trips overlap instead of chaining
                            for (int b0 = 0; b0 < wc; b0 += 8) {
                                int c2[8], old[8];
#pragma unroll
                                for (int j = 0; j < 8; ++j) c2[j] = b0 + j < wc ? S.var_adj[wo + b0 + j] : -1;
#pragma unroll
                                for (int j = 0; j < 8; ++j) old[j] = c2[j] >= 0 ? atomicExch(&S.cstamp[c2[j]], stamp) : stamp;
#pragma unroll
                                for (int j = 0; j < 8; ++j)
                                    if (old[j] != stamp) next[atomicAdd(&sh_nlen, 1)] = c2[j];
                            }
                        }
                    }
                    __syncthreads();
                    const int nlen = sh_nlen;
                    __syncthreads();
                    if (nlen == 0) {
                        c = pick_unreached(S, cap, stamp, edge, &draw, &sh_min, &sh_pick, seg, sh_d0);
                        break;
                    }
                    if (count + nlen == m) {
                        // every check reached: the lowest key among the last level
                        uint64_t key = ~0ull;
                        for (int i = tid; i < nlen; i += kPegBlock) {
                            const int c2 = next[i];
                            const uint64_t kk = cand_key(S, c2, S.len[c2], edge);
                            key = kk < key ? kk : key;
                        }
                        c = static_cast<int>(static_cast<uint32_t>(block_min(key, &sh_min)));
                        break;
                    }
                    count += nlen;
                    int32_t *t = front;
                    front = next;
                    next = t;
                    flen = nlen;
                    if (tid == 0) sh_nlen = 0;
                    __syncthreads();
                }
            }
            if (tid == 0) {
                if (c < 0) {
                    *S.err = 2;
                    sh_stop = 1;
                } else if (S.len[c] >= cap) {
                    *S.err = 1;
                    sh_stop = 1;
                } else {
                    bump_degree(S, c, seg, &sh_d0);
                    S.adj[static_cast<size_t>(c) * cap + S.len[c]] = v;
                    S.len[c] += 1;
                    S.var_adj[off + S.var_cnt[v]] = c;
                    S.var_cnt[v] += 1;
                }
            }
            __syncthreads();
            if (sh_stop) return;
        }
    }
}

// CSR rows of a built matrix: row_ptr from the check degrees (one block
// scans), then each check's variables copied in order.
__global__ __launch_bounds__(kPegBlock) void k_peg_row_ptr(const int32_t *len, int32_t *row_ptr, int32_t m) {
    __shared__ int32_t part[kPegBlock];
    const int tid = static_cast<int>(threadIdx.x);
    const int per = (m + kPegBlock - 1) / kPegBlock;
    const int c0 = tid * per, c1 = min(m, c0 + per);
    int32_t s = 0;
    for (int c = c0; c < c1; ++c) s += len[c];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < kPegBlock; o <<= 1) {
        const int32_t x = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    int32_t run = part[tid] - s;
    if (tid == 0) row_ptr[0] = 0;
    for (int c = c0; c < c1; ++c) {
        run += len[c];
        row_ptr[c + 1] = run;
    }
}

__global__ __launch_bounds__(kBlock) void k_peg_cols(const int32_t *len, const int32_t *adj, const int32_t *row_ptr,
                                                     int32_t *col, int32_t m, int32_t cap) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int c = static_cast<int>(i / cap), j = static_cast<int>(i % cap);
    if (c < m && j < len[c]) col[row_ptr[c] + j] = adj[static_cast<size_t>(c) * cap + j];
}

}  // namespace

int peg_build_impl(mbp_ctx *ctx, int32_t n, int32_t m, int32_t u, const int32_t *var_deg, const uint64_t *seeds,
                   int32_t max_depth, int32_t *row_ptr, int32_t *col_idx) {
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::vector<int32_t> off(static_cast<size_t>(n) + 1, 0);
    for (int32_t i = 0; i < n; ++i) off[i + 1] = off[i] + var_deg[i];
    const int64_t E = off[n];
    // check degrees stay near E / m (each edge goes to a lowest-degree
    // candidate); a check that would pass this bound stops the build
    const int32_t cap = static_cast<int32_t>((E + m - 1) / m) + 32;
    if (cap + 2 > kPegSegMax)
        return fail(MBP_EUNSUPPORTED, "mbp_peg_build: average check degree above " + std::to_string(kPegSegMax - 34));
    const size_t per = (2 * static_cast<size_t>(n) + E + 6 * static_cast<size_t>(m) +
                        static_cast<size_t>(m) * cap + 1) * sizeof(int32_t);
    char *ws = nullptr;
    const size_t total = (static_cast<size_t>(n) + 1) * sizeof(int32_t) + per * u +
                         (static_cast<size_t>(m) + 1) * sizeof(int32_t) + E * sizeof(int32_t);
    if ((e = hipMalloc(&ws, total)) != hipSuccess) return fail(MBP_ENOMEM, "mbp_peg_build: workspace");
    auto release = [&] { (void)hipFree(ws); };
    char *p = ws;
    auto take = [&](size_t count) {
        int32_t *at = reinterpret_cast<int32_t *>(p);
        p += count * sizeof(int32_t);
        return at;
    };
    int32_t *d_off = take(static_cast<size_t>(n) + 1);
    if ((e = hipMemcpy(d_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) {
        release();
        return hip_fail(e, "mbp_peg_build: upload");
    }
    std::vector<PegState> st(u);
    for (int32_t l = 0; l < u; ++l) {
        PegState &S = st[l];
        S.var_off = d_off;
        S.var_cnt = take(n);
        S.vstamp = take(n);
        S.var_adj = take(E);
        S.len = take(m);
        S.order = take(m);
        S.pos = take(m);
        S.cstamp = take(m);
        S.front = take(m);
        S.next = take(m);
        S.adj = take(static_cast<size_t>(m) * cap);
        S.err = take(1);
        S.seed = seeds[l];
    }
    int32_t *d_rp = take(static_cast<size_t>(m) + 1);
    int32_t *d_col = take(E);
    // error flags start at 0
    for (int32_t l = 0; l < u; ++l)
        if ((e = hipMemset(st[l].err, 0, sizeof(int32_t))) != hipSuccess) {
            release();
            return hip_fail(e, "mbp_peg_build: memset");
        }
    for (int32_t l0 = 0; l0 < u; l0 += 4) {
        PegArgs a{};
        const int32_t nb = std::min(4, u - l0);
        for (int32_t k = 0; k < nb; ++k) a.st[k] = st[l0 + k];
        a.n = n;
        a.m = m;
        a.cap = cap;
        a.max_depth = max_depth;
        k_peg<<<nb, kPegBlock>>>(a, l0);
        if ((e = hipGetLastError()) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
            release();
            return hip_fail(e, "mbp_peg_build: construction");
        }
    }
    for (int32_t l = 0; l < u; ++l) {
        int32_t err = 0;
        if ((e = hipMemcpy(&err, st[l].err, sizeof(err), hipMemcpyDeviceToHost)) != hipSuccess) {
            release();
            return hip_fail(e, "mbp_peg_build: status");
        }
        if (err == 1) {
            release();
            return fail(MBP_EUNSUPPORTED, "mbp_peg_build: a check degree passed ceil(E/m) + 32");
        }
        if (err == 2) {
            release();
            return fail(MBP_EINVAL, "mbp_peg_build: a variable has no check left for an edge");
        }
        k_peg_row_ptr<<<1, kPegBlock>>>(st[l].len, d_rp, m);
        const int64_t items = static_cast<int64_t>(m) * cap;
        k_peg_cols<<<static_cast<unsigned>((items + kBlock - 1) / kBlock), kBlock>>>(st[l].len, st[l].adj, d_rp,
                                                                                     d_col, m, cap);
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = hipMemcpy(row_ptr + static_cast<size_t>(l) * (m + 1), d_rp, (static_cast<size_t>(m) + 1) * sizeof(int32_t),
                           hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(col_idx + static_cast<size_t>(l) * E, d_col, E * sizeof(int32_t), hipMemcpyDeviceToHost)) !=
                hipSuccess) {
            release();
            return hip_fail(e, "mbp_peg_build: output");
        }
    }
    release();
    return MBP_OK;
}

}  // namespace mbp
