/*
 * Progressive edge-growth (PEG) construction of sparse parity-check matrices.
 *
 * The paper builds its u check matrices with PEG (Sec. 2, first paragraph,
 * citing Hu, Eleftheriou and Arnold) and gives no further detail, so this file
 * follows the published PEG procedure:
 *   - variable nodes are taken one at a time in the given (non-decreasing
 *     degree) order;
 *   - the first edge of a variable goes to a check of lowest current degree;
 *   - every further edge goes to a lowest-degree check among those that a
 *     breadth-first expansion of the current Tanner graph from the variable
 *     reaches last, i.e. the farthest checks; when the expansion stops growing,
 *     the candidates are all checks it never reached;
 *   - ties are broken uniformly at random with a seeded generator.
 * An optional depth bound stops the expansion early (candidates are then the
 * unreached checks): with bound b the new edge closes no cycle shorter than
 * 2*(b+2), and the cost drops from O(E) to the size of the explored ball.
 *
 * This is an input generator: it draws the codes that both the decoder and
 * its checker are run on, and holds none of the decoder's arithmetic.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* splitmix64 (Steele, Lea and Flood, 2014), used as a seeded stream. */
static uint64_t sm64_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Uniform integer in [0, k) by rejection (no modulo bias). */
static uint32_t rand_below(uint64_t *s, uint32_t k) {
    uint64_t lim = (UINT64_MAX / k) * k;
    uint64_t r;
    do { r = sm64_next(s); } while (r >= lim);
    return (uint32_t)(r % k);
}

typedef struct {
    int *data;
    int len, cap;
} ivec;

static int ivec_push(ivec *v, int x) {
    if (v->len == v->cap) {
        int nc = v->cap ? 2 * v->cap : 8;
        int *nd = (int *)realloc(v->data, (size_t)nc * sizeof(int));
        if (!nd) return -1;
        v->data = nd;
        v->cap = nc;
    }
    v->data[v->len++] = x;
    return 0;
}

typedef struct {
    int n, m;
    const int *var_deg;
    int *var_off, *var_cnt, *var_adj; /* checks of each variable */
    ivec *chk_adj;                    /* variables of each check (ascending) */
    /* checks ordered by degree: order[] is sorted by degree, seg[d] is the
       first index of degree d, pos[c] the index of check c in order[] */
    int *order, *pos, *seg, seg_len;
    int *cstamp, *vstamp, stamp;
    ivec frontier, next;
    uint64_t rng;
} peg_state;

static int chk_deg(const peg_state *s, int c) { return s->chk_adj[c].len; }

/* Raise the degree of check c by one, keeping order[] sorted. */
static void bump_degree(peg_state *s, int c) {
    int d = chk_deg(s, c); /* degree before the new edge was appended */
    int last = s->seg[d + 1] - 1;
    int pc = s->pos[c], other = s->order[last];
    s->order[pc] = other;
    s->pos[other] = pc;
    s->order[last] = c;
    s->pos[c] = last;
    s->seg[d + 1] = last;
}

static int reached(const peg_state *s, int c) { return s->cstamp[c] == s->stamp; }

/* Lowest-degree check not reached by the current expansion, uniform among
   ties. Returns -1 if every check is reached. */
static int pick_unreached(peg_state *s) {
    int d = chk_deg(s, s->order[0]);
    while (d + 1 < s->seg_len && s->seg[d] < s->m) {
        int lo = s->seg[d], hi = s->seg[d + 1];
        if (hi > lo) {
            uint32_t cnt = (uint32_t)(hi - lo);
            for (int tries = 0; tries < 24; ++tries) {
                int c = s->order[lo + (int)rand_below(&s->rng, cnt)];
                if (!reached(s, c)) return c;
            }
            uint32_t free_cnt = 0;
            for (int i = lo; i < hi; ++i) free_cnt += !reached(s, s->order[i]);
            if (free_cnt) {
                uint32_t r = rand_below(&s->rng, free_cnt);
                for (int i = lo; i < hi; ++i) {
                    int c = s->order[i];
                    if (!reached(s, c)) {
                        if (r == 0) return c;
                        --r;
                    }
                }
            }
        }
        ++d;
    }
    return -1;
}

/* Lowest-degree check in an explicit candidate list, uniform among ties. */
static int pick_from_list(peg_state *s, const ivec *cand) {
    int best = -1, bestd = 0;
    uint32_t ties = 0;
    for (int i = 0; i < cand->len; ++i) {
        int c = cand->data[i], d = chk_deg(s, c);
        if (best < 0 || d < bestd) {
            best = c;
            bestd = d;
            ties = 1;
        } else if (d == bestd) {
            ++ties;
            if (rand_below(&s->rng, ties) == 0) best = c;
        }
    }
    return best;
}

/* Choose the check for the next edge of variable v. */
static int choose_check(peg_state *s, int v, int max_depth) {
    ++s->stamp;
    if (s->var_cnt[v] == 0) return pick_unreached(s);
    s->frontier.len = 0;
    int count = 0;
    const int *adj = s->var_adj + s->var_off[v];
    for (int k = 0; k < s->var_cnt[v]; ++k) {
        s->cstamp[adj[k]] = s->stamp;
        if (ivec_push(&s->frontier, adj[k])) return -2;
        ++count;
    }
    s->vstamp[v] = s->stamp;
    for (int level = 0;; ++level) {
        if (max_depth >= 0 && level >= max_depth) return pick_unreached(s);
        s->next.len = 0;
        for (int fi = 0; fi < s->frontier.len; ++fi) {
            const ivec *vs = &s->chk_adj[s->frontier.data[fi]];
            for (int a = 0; a < vs->len; ++a) {
                int w = vs->data[a];
                if (s->vstamp[w] == s->stamp) continue;
                s->vstamp[w] = s->stamp;
                const int *wa = s->var_adj + s->var_off[w];
                for (int b = 0; b < s->var_cnt[w]; ++b) {
                    int c2 = wa[b];
                    if (s->cstamp[c2] == s->stamp) continue;
                    s->cstamp[c2] = s->stamp;
                    if (ivec_push(&s->next, c2)) return -2;
                }
            }
        }
        if (s->next.len == 0) return pick_unreached(s);
        if (count + s->next.len == s->m) return pick_from_list(s, &s->next);
        count += s->next.len;
        ivec tmp = s->frontier;
        s->frontier = s->next;
        s->next = tmp;
    }
}

/*
 * Build an m x n matrix with the given variable degrees.
 *   var_deg   [n] degrees, each in [1, m]
 *   seed      tie-break stream seed
 *   max_depth expansion bound (< 0: unbounded)
 *   row_ptr   [m+1] output CSR row offsets
 *   col_idx   [sum var_deg] output CSR columns, ascending within each row
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 */
int peg_build(int n, int m, const int *var_deg, uint64_t seed, int max_depth,
              int *row_ptr, int *col_idx) {
    if (n < 1 || m < 1 || !var_deg || !row_ptr || !col_idx) return -1;
    long long E = 0;
    for (int i = 0; i < n; ++i) {
        if (var_deg[i] < 1 || var_deg[i] > m) return -1;
        E += var_deg[i];
    }
    if (E > 0x7fffffffLL) return -1;

    peg_state s;
    memset(&s, 0, sizeof s);
    s.n = n;
    s.m = m;
    s.var_deg = var_deg;
    s.rng = seed;
    int rc = -2;
    s.var_off = (int *)malloc((size_t)(n + 1) * sizeof(int));
    s.var_cnt = (int *)calloc((size_t)n, sizeof(int));
    s.var_adj = (int *)malloc((size_t)E * sizeof(int));
    s.chk_adj = (ivec *)calloc((size_t)m, sizeof(ivec));
    s.order = (int *)malloc((size_t)m * sizeof(int));
    s.pos = (int *)malloc((size_t)m * sizeof(int));
    s.seg_len = n + 3; /* a check degree never exceeds n */
    s.seg = (int *)malloc((size_t)s.seg_len * sizeof(int));
    s.cstamp = (int *)calloc((size_t)m, sizeof(int));
    s.vstamp = (int *)calloc((size_t)n, sizeof(int));
    if (!s.var_off || !s.var_cnt || !s.var_adj || !s.chk_adj || !s.order || !s.pos ||
        !s.seg || !s.cstamp || !s.vstamp)
        goto done;
    s.var_off[0] = 0;
    for (int i = 0; i < n; ++i) s.var_off[i + 1] = s.var_off[i] + var_deg[i];
    for (int c = 0; c < m; ++c) {
        s.order[c] = c;
        s.pos[c] = c;
    }
    /* all checks start at degree 0: segment 0 is [0, m), the rest empty */
    s.seg[0] = 0;
    for (int d = 1; d < s.seg_len; ++d) s.seg[d] = m;

    for (int v = 0; v < n; ++v) {
        for (int k = 0; k < var_deg[v]; ++k) {
            int c = choose_check(&s, v, max_depth);
            if (c == -2) goto done;
            if (c < 0) { rc = -1; goto done; }
            bump_degree(&s, c);
            if (ivec_push(&s.chk_adj[c], v)) goto done;
            s.var_adj[s.var_off[v] + s.var_cnt[v]++] = c;
        }
    }
    row_ptr[0] = 0;
    for (int c = 0; c < m; ++c) {
        row_ptr[c + 1] = row_ptr[c] + s.chk_adj[c].len;
        memcpy(col_idx + row_ptr[c], s.chk_adj[c].data, (size_t)s.chk_adj[c].len * sizeof(int));
    }
    rc = 0;
done:
    if (s.chk_adj)
        for (int c = 0; c < m; ++c) free(s.chk_adj[c].data);
    free(s.frontier.data);
    free(s.next.data);
    free(s.var_off);
    free(s.var_cnt);
    free(s.var_adj);
    free(s.chk_adj);
    free(s.order);
    free(s.pos);
    free(s.seg);
    free(s.cstamp);
    free(s.vstamp);
    return rc;
}
