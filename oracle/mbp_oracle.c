/*
 * Plain FP64 CPU oracle for multi-matrix syndrome belief propagation (MBP).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the checker the GPU decoder is
 * compared against. It is called from the tests, from the smoke check and
 * from the CPU-baseline leg of the benchmark; the decoder library never
 * links, loads or calls it, and it shares no code with the decoder.
 *
 * What it computes follows the paper (arXiv 2001.07979):
 *   - Sec. 2: Bob holds u matrices H_1..H_u and Alice's u syndromes
 *     z^l = H_l x (eq. (1)); he decodes with belief propagation over all u
 *     matrices at once, forms the soft decision of eq. (2), decides the bits
 *     and stops once every syndrome is met or the iteration limit is reached.
 *   - Algorithm 1 (Sec. 3A): initialise every variable-to-check message to
 *     the channel LLR, then repeat check-to-variable and variable-to-check
 *     updates, decide, test the stopping rule.
 *   - Sec. 3B, eq. (6): the check-to-variable rule with the syndrome sign.
 *   - Sec. 3B, eq. (5): branch-free priors (read as P1 = e + y(1-2e),
 *     P0 = 1 - P1, because the printed form is negative for y = 1).
 *   - Sec. 2, eqs. (3)-(4): efficiency f and binary entropy h(e).
 * Readings where the paper is silent:
 *   - the u matrices form one stacked Tanner graph [H_1; ...; H_u] with
 *     syndrome [z^1; ...; z^u], updated with a flooding schedule (every check
 *     of every matrix from the previous iteration's messages, then every
 *     variable);
 *   - LLRs are ln(P0/P1); sgn(0) = +1; the decision at L = 0 is bit 0;
 *   - variable-to-check messages are clipped to [-C, C] before the check rule;
 *   - the first stopping test follows the first full update (iterations are
 *     counted from 1);
 *   - the normalized min-sum rule (not in the paper) replaces the tanh rule by
 *     alpha times the product of signs times the smallest other magnitude.
 *
 * A second reading of how the u matrices combine (coupling = 1): Sec. 2
 * forms the LLRs and variable-to-check messages "for all u matrices
 * respectively", so each matrix may run its own decoder: matrix l's
 * variable-to-check message on an edge is the channel LLR plus the other
 * check messages of matrix l alone at that variable (its own posterior
 * lambda + S^l minus the edge's message), and only the soft decision of
 * eq. (2), lambda + sum over l of S^l, joins the matrices. S^l is matrix
 * l's messages at the variable summed from 0 in check order.
 *
 * Everything is FP64, one frame at a time, with every exclusion ("all other
 * edges of the check") evaluated directly as its definition states.
 * Frames are spread over POSIX threads; each frame's arithmetic is serial.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

typedef struct {
    int32_t n;               /* key bits per frame (variable nodes) */
    int32_t u;               /* number of matrices */
    const int32_t *m;        /* [u] checks per matrix */
    const int32_t *row_ptr;  /* u CSR row-offset arrays back to back, m_l+1 each, each from 0 */
    const int32_t *col_idx;  /* u CSR column arrays back to back */
} oracle_code;

typedef struct {
    int32_t algo;            /* 0 = sum-product, eq. (6); 1 = normalized min-sum */
    int32_t max_iter;        /* iteration limit T (>= 1) */
    int32_t early_exit;      /* stop a frame once all syndromes hold */
    double alpha;            /* min-sum normalization */
    double clip;             /* C: messages entering the check rule lie in [-C, C] */
    const double *alpha_tl;  /* optional [T][u] per-iteration, per-matrix weights (min-sum) */
    double margin;           /* delta for the near-tie flag */
    int32_t schedule;        /* 0 = flooding; 1 = matrix-serial (see phase_rows) */
    int32_t coupling;        /* 0 = one stacked graph; 1 = u independent decoders (see below) */
    int32_t msg_half;        /* 1: every new check-to-variable message is stored rounded to
                                binary16 (see round_binary16); its sender and every reader
                                use the stored value */
} oracle_params;

/* ---------------------------------------------------------------------- */
/* Sec. 2, eq. (4): Shannon binary entropy in bits. */
double oracle_binary_entropy(double e) {
    if (e <= 0.0 || e >= 1.0) return 0.0;
    return -e * log2(e) - (1.0 - e) * log2(1.0 - e);
}

/* Sec. 2, eq. (3): reconciliation efficiency f = m / (n h(e)). */
double oracle_efficiency(int32_t m, int32_t n, double e) {
    return (double)m / ((double)n * oracle_binary_entropy(e));
}

/* Sec. 3B, eq. (5) (corrected) then the channel LLR of Sec. 2:
   P1 = e + y (1 - 2e) is the probability that Alice's bit is 1 given Bob's
   bit y; P0 = 1 - P1; llr = ln(P0 / P1). */
void oracle_llr_from_bits(const uint8_t *y, int32_t n, double e, double *llr) {
    for (int32_t i = 0; i < n; ++i) {
        double yi = y[i] ? 1.0 : 0.0;
        double p1 = e + yi * (1.0 - 2.0 * e);
        double p0 = 1.0 - p1;
        llr[i] = log(p0 / p1);
    }
}

/* ---------------------------------------------------------------------- */
/* The stacked Tanner graph: edges in check-major order (matrix, row,
   column), and for every variable its edges in the same order. */
typedef struct {
    int32_t n, u, M, E;
    int32_t *row_start;   /* [M+1] first edge of each stacked check */
    int32_t *row_matrix;  /* [M] which matrix the check belongs to */
    int32_t *edge_var;    /* [E] variable of each edge */
    int32_t *var_start;   /* [n+1] */
    int32_t *var_edges;   /* [E] edges of each variable, ascending */
    int32_t *edge_matrix; /* [E] which matrix the edge's check belongs to */
} graph;

static void graph_free(graph *g) {
    free(g->row_start);
    free(g->row_matrix);
    free(g->edge_var);
    free(g->var_start);
    free(g->var_edges);
    free(g->edge_matrix);
}

static int graph_build(const oracle_code *c, graph *g) {
    memset(g, 0, sizeof *g);
    g->n = c->n;
    g->u = c->u;
    int32_t M = 0, E = 0;
    const int32_t *rp = c->row_ptr;
    for (int32_t l = 0; l < c->u; ++l) {
        M += c->m[l];
        E += rp[c->m[l]];
        rp += c->m[l] + 1;
    }
    g->M = M;
    g->E = E;
    g->row_start = malloc(sizeof(int32_t) * (size_t)(M + 1));
    g->row_matrix = malloc(sizeof(int32_t) * (size_t)(M > 0 ? M : 1));
    g->edge_var = malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    g->var_start = calloc((size_t)c->n + 1, sizeof(int32_t));
    g->var_edges = malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    g->edge_matrix = malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    if (!g->row_start || !g->row_matrix || !g->edge_var || !g->var_start || !g->var_edges ||
        !g->edge_matrix) {
        graph_free(g);
        return -1;
    }
    int32_t r = 0, e = 0;
    rp = c->row_ptr;
    const int32_t *ci = c->col_idx;
    for (int32_t l = 0; l < c->u; ++l) {
        for (int32_t j = 0; j < c->m[l]; ++j) {
            g->row_start[r] = e;
            g->row_matrix[r] = l;
            if (rp[j + 1] - rp[j] < 2) { graph_free(g); return -1; } /* checks need two edges */
            for (int32_t k = rp[j]; k < rp[j + 1]; ++k) {
                int32_t v = ci[k];
                if (v < 0 || v >= c->n) { graph_free(g); return -1; }
                g->edge_matrix[e] = l;
                g->edge_var[e++] = v;
            }
            ++r;
        }
        ci += rp[c->m[l]];
        rp += c->m[l] + 1;
    }
    g->row_start[M] = E;
    for (e = 0; e < E; ++e) g->var_start[g->edge_var[e] + 1]++;
    for (int32_t i = 0; i < c->n; ++i) g->var_start[i + 1] += g->var_start[i];
    int32_t *fill = malloc(sizeof(int32_t) * (size_t)(c->n > 0 ? c->n : 1));
    if (!fill) { graph_free(g); return -1; }
    memcpy(fill, g->var_start, sizeof(int32_t) * (size_t)c->n);
    for (e = 0; e < E; ++e) g->var_edges[fill[g->edge_var[e]]++] = e;
    free(fill);
    return 0;
}

static double sgn(double x) { return x < 0.0 ? -1.0 : 1.0; }

/* The binary16 value nearest to x, ties to even, as IEEE 754 defines the
   format: 11 significant bits down to 2^-14, then a fixed quantum of 2^-24
   (subnormals); magnitudes that round beyond the largest finite value 65504
   become infinite. x / quantum is exact (a power-of-two scale), and nearbyint
   rounds it to the nearest integer, ties to even, in the default mode. */
static double round_binary16(double x) {
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(fabs(x), &e); /* |x| = f 2^e, f in [0.5, 1) */
    int q = e - 11;
    if (q < -24) q = -24;
    double r = ldexp(nearbyint(ldexp(fabs(x), -q)), q);
    if (r > 65504.0) r = INFINITY;
    return copysign(r, x);
}

double oracle_round_binary16(double x) { return round_binary16(x); }

static double clip_to(double x, double C) { return x > C ? C : (x < -C ? -C : x); }

/* Eq. (2) with its nesting: L_i = lambda_i + sum over matrices l (in order)
   of [sum over the checks j of H_l at variable i (in order) of c]. Each
   matrix's messages are summed first, from 0, and that sum is added to the
   running total; a matrix with no edge at the variable adds nothing. The
   binary32 variant does the same additions in binary32. */
static double vsum_d(const graph *g, int32_t i, double lam, const double *c) {
    double L = lam, S = 0.0;
    int32_t cur = -1;
    for (int32_t k = g->var_start[i]; k < g->var_start[i + 1]; ++k) {
        const int32_t e = g->var_edges[k];
        if (g->edge_matrix[e] != cur) {
            if (cur >= 0) L += S;
            S = 0.0;
            cur = g->edge_matrix[e];
        }
        S += c[e];
    }
    if (cur >= 0) L += S;
    return L;
}

static float vsum_f(const graph *g, int32_t i, float lam, const float *c) {
    float L = lam, S = 0.0f;
    int32_t cur = -1;
    for (int32_t k = g->var_start[i]; k < g->var_start[i + 1]; ++k) {
        const int32_t e = g->var_edges[k];
        if (g->edge_matrix[e] != cur) {
            if (cur >= 0) L += S;
            S = 0.0f;
            cur = g->edge_matrix[e];
        }
        S += c[e];
    }
    if (cur >= 0) L += S;
    return L;
}

/* the same over messages held as doubles of binary32 values */
static float vsum_fd(const graph *g, int32_t i, float lam, const double *c) {
    float L = lam, S = 0.0f;
    int32_t cur = -1;
    for (int32_t k = g->var_start[i]; k < g->var_start[i + 1]; ++k) {
        const int32_t e = g->var_edges[k];
        if (g->edge_matrix[e] != cur) {
            if (cur >= 0) L += S;
            S = 0.0f;
            cur = g->edge_matrix[e];
        }
        S += (float)c[e];
    }
    if (cur >= 0) L += S;
    return L;
}

/* Independent decoders: matrix l's posterior at variable i, lambda + S^l
   (S^l: matrix l's messages at i summed from 0 in check order), for every
   matrix; lambda alone where matrix l has no edge at i. */
static void matrix_posteriors_d(const graph *g, int32_t i, double lam, const double *c, double *Lm) {
    for (int32_t l = 0; l < g->u; ++l) {
        double S = 0.0;
        for (int32_t k = g->var_start[i]; k < g->var_start[i + 1]; ++k) {
            const int32_t e = g->var_edges[k];
            if (g->edge_matrix[e] == l) S += c[e];
        }
        Lm[(size_t)l * (size_t)g->n + (size_t)i] = lam + S;
    }
}

static void matrix_posteriors_f(const graph *g, int32_t i, float lam, const float *c, float *Lm) {
    for (int32_t l = 0; l < g->u; ++l) {
        float S = 0.0f;
        for (int32_t k = g->var_start[i]; k < g->var_start[i + 1]; ++k) {
            const int32_t e = g->var_edges[k];
            if (g->edge_matrix[e] == l) S += c[e];
        }
        Lm[(size_t)l * (size_t)g->n + (size_t)i] = lam + S;
    }
}

/* Sec. 3B, eq. (6): check-to-variable messages of one check, sum-product.
   For each edge k: c_k = (-1)^z * 2 atanh( prod over the other edges k' of
   tanh(q_k' / 2) ), with q clipped to [-C, C] first. */
static void check_rule_spa(int32_t d, const double *q, int z, double C, double *th,
                           double *out) {
    for (int32_t k = 0; k < d; ++k) th[k] = tanh(clip_to(q[k], C) / 2.0);
    double zs = z ? -1.0 : 1.0;
    for (int32_t k = 0; k < d; ++k) {
        double prod = 1.0;
        for (int32_t kk = 0; kk < d; ++kk)
            if (kk != k) prod *= th[kk];
        out[k] = zs * 2.0 * atanh(prod);
    }
}

/* Normalized min-sum: c_k = (-1)^z * alpha * prod sgn(q_k') * min |q_k'|
   over the other edges k', with |q| capped at C. */
static void check_rule_nms(int32_t d, const double *q, int z, double alpha, double C,
                           double *out) {
    double zs = z ? -1.0 : 1.0;
    for (int32_t k = 0; k < d; ++k) {
        double s = 1.0, mn = INFINITY;
        for (int32_t kk = 0; kk < d; ++kk) {
            if (kk == k) continue;
            s *= sgn(q[kk]);
            double a = fabs(q[kk]);
            if (a > C) a = C;
            if (a < mn) mn = a;
        }
        out[k] = zs * alpha * s * mn;
    }
}

/* Number of stacked checks whose parity over the decided bits differs from
   the syndrome bit (Sec. 2: success once z^l = H_l y for every l). */
static int32_t unsatisfied(const graph *g, const uint8_t *xhat, const uint8_t *z) {
    int32_t w = 0;
    for (int32_t r = 0; r < g->M; ++r) {
        int par = 0;
        for (int32_t e = g->row_start[r]; e < g->row_start[r + 1]; ++e) par ^= xhat[g->edge_var[e]];
        w += (par != (z[r] ? 1 : 0));
    }
    return w;
}

static double weight_of(const oracle_params *P, int32_t t, int32_t l, int32_t u) {
    return P->alpha_tl ? P->alpha_tl[(size_t)(t - 1) * (size_t)u + (size_t)l] : P->alpha;
}

typedef struct {
    double *c, *q, *L, *th, *tmp;
    double *Lm; /* [u][n] per-matrix posteriors lambda + S^l (independent decoders) */
    uint8_t *xhat;
} frame_buf;

static int buf_alloc(frame_buf *b, const graph *g, int32_t maxdeg) {
    b->c = malloc(sizeof(double) * (size_t)(g->E > 0 ? g->E : 1));
    b->q = malloc(sizeof(double) * (size_t)(g->E > 0 ? g->E : 1));
    b->L = malloc(sizeof(double) * (size_t)(g->n > 0 ? g->n : 1));
    b->th = malloc(sizeof(double) * (size_t)(maxdeg > g->n ? maxdeg : (g->n > 0 ? g->n : 1)));
    b->tmp = malloc(sizeof(double) * (size_t)(maxdeg > 0 ? maxdeg : 1));
    b->xhat = malloc((size_t)(g->n > 0 ? g->n : 1));
    b->Lm = malloc(sizeof(double) * (size_t)(g->n > 0 ? g->n : 1) * (size_t)g->u);
    return (b->c && b->q && b->L && b->th && b->tmp && b->xhat && b->Lm) ? 0 : -1;
}

static void buf_free(frame_buf *b) {
    free(b->c);
    free(b->q);
    free(b->L);
    free(b->th);
    free(b->tmp);
    free(b->xhat);
    free(b->Lm);
}

/* Rows (stacked checks) updated in phase ph of an iteration. Flooding: one
   phase, every check of every matrix from the previous iteration's
   messages. Matrix-serial (Algorithm 1 taken literally: inside an
   iteration the matrices are visited in turn, and each matrix's
   check-to-variable then variable-to-check updates finish before the next
   matrix starts): phase l holds the checks of matrix l, and the soft
   decisions are recomputed after each phase. */
static int32_t phase_count(const graph *g, const oracle_params *P) { return P->schedule ? g->u : 1; }

static void phase_rows(const graph *g, const oracle_params *P, int32_t ph, int32_t *r0, int32_t *r1) {
    if (!P->schedule) {
        *r0 = 0;
        *r1 = g->M;
        return;
    }
    int32_t a = 0;
    while (a < g->M && g->row_matrix[a] < ph) ++a;
    int32_t b = a;
    while (b < g->M && g->row_matrix[b] == ph) ++b;
    *r0 = a;
    *r1 = b;
}

/* One frame of MBP (Algorithm 1 over the stacked graph, flooding or
   matrix-serial). Writes the decided bits, success flag, iteration count,
   final soft decisions L and the near-tie flag. */
static void decode_frame(const graph *g, const oracle_params *P, const double *lam,
                         const uint8_t *z, frame_buf *b, uint8_t *bits, int32_t *iters,
                         uint8_t *ok, double *Lout, uint8_t *flag) {
    const int32_t n = g->n, E = g->E;
    /* Algorithm 1, first step: every variable-to-check message starts at the
       channel LLR; equivalently no check message yet (c = 0) and L = lambda. */
    for (int32_t e = 0; e < E; ++e) b->c[e] = 0.0;
    for (int32_t i = 0; i < n; ++i) b->L[i] = lam[i];
    for (int32_t l = 0; l < g->u; ++l)
        for (int32_t i = 0; i < n; ++i) b->Lm[(size_t)l * (size_t)n + (size_t)i] = lam[i];
    int32_t t_stop = P->max_iter;
    int stopped = 0;
    uint8_t fl = 0;
    for (int32_t t = 1; t <= P->max_iter; ++t) {
        for (int32_t ph = 0; ph < phase_count(g, P); ++ph) {
            int32_t r0, r1;
            phase_rows(g, P, ph, &r0, &r1);
            /* variable-to-check messages from the current soft decisions:
               the soft decision minus the message that came in on this edge
               (independent decoders: the posterior of the edge's own matrix) */
            for (int32_t e = g->row_start[r0]; e < g->row_start[r1]; ++e)
                b->q[e] = (P->coupling ? b->Lm[(size_t)g->edge_matrix[e] * (size_t)n + (size_t)g->edge_var[e]]
                                       : b->L[g->edge_var[e]]) - b->c[e];
            /* check-to-variable messages of the phase's checks */
            for (int32_t r = r0; r < r1; ++r) {
                int32_t e0 = g->row_start[r], d = g->row_start[r + 1] - e0;
                if (P->algo == 0)
                    check_rule_spa(d, b->q + e0, z[r], P->clip, b->th, b->tmp);
                else
                    check_rule_nms(d, b->q + e0, z[r], weight_of(P, t, g->row_matrix[r], g->u),
                                   P->clip, b->tmp);
                for (int32_t k = 0; k < d; ++k)
                    b->c[e0 + k] = P->msg_half ? round_binary16(b->tmp[k]) : b->tmp[k];
            }
            /* eq. (2): soft decision = channel LLR + every incoming check
               message, a sum per matrix added in matrix order */
            for (int32_t i = 0; i < n; ++i) b->L[i] = vsum_d(g, i, lam[i], b->c);
            if (P->coupling)
                for (int32_t i = 0; i < n; ++i) matrix_posteriors_d(g, i, lam[i], b->c, b->Lm);
        }
        /* decision: bit 1 iff L < 0 */
        for (int32_t i = 0; i < n; ++i) b->xhat[i] = b->L[i] < 0.0 ? 1 : 0;
        if (P->early_exit) {
            int32_t w = unsatisfied(g, b->xhat, z);
            if (w == 0) {
                /* near tie at the stopping iteration */
                for (int32_t i = 0; i < n; ++i)
                    if (fabs(b->L[i]) < P->margin) fl = 1;
                t_stop = t;
                stopped = 1;
                break;
            }
            /* an earlier near tie whose flips could have met the syndrome */
            long long degsum = 0;
            int32_t nsmall = 0;
            for (int32_t i = 0; i < n; ++i) {
                if (fabs(b->L[i]) < P->margin) {
                    ++nsmall;
                    degsum += g->var_start[i + 1] - g->var_start[i];
                }
            }
            if (nsmall > 0 && (long long)w <= degsum) fl = 1;
        }
    }
    if (!stopped) {
        for (int32_t i = 0; i < n; ++i)
            if (fabs(b->L[i]) < P->margin) fl = 1;
    }
    *ok = stopped ? 1 : (unsatisfied(g, b->xhat, z) == 0 ? 1 : 0);
    *iters = t_stop;
    for (int32_t i = 0; i < n; ++i) bits[i] = b->xhat[i];
    if (Lout)
        for (int32_t i = 0; i < n; ++i) Lout[i] = b->L[i];
    if (flag) *flag = fl;
}

/* Normalized min-sum in binary32 arithmetic. The same rule and schedule as
   decode_frame, with every quantity a float and every operation rounded to
   float in the order the definitions give: q = L - c; |q| capped at C; the
   smallest other magnitude; c = (-1)^z * alpha * (product of signs) * min;
   L = lambda + the incoming messages in (matrix, check) order. No near-tie
   flag is computed. */
static void decode_frame_nms_f32(const graph *g, const oracle_params *P, const double *lam64,
                                 const uint8_t *z, frame_buf *b, uint8_t *bits, int32_t *iters,
                                 uint8_t *ok, double *Lout) {
    const int32_t n = g->n, E = g->E;
    float *c = (float *)b->c, *q = (float *)b->q, *L = (float *)b->L, *lam = (float *)b->th;
    const float C = (float)P->clip;
    float *Lm = (float *)b->Lm;
    for (int32_t i = 0; i < n; ++i) lam[i] = (float)lam64[i];
    for (int32_t e = 0; e < E; ++e) c[e] = 0.0f;
    for (int32_t i = 0; i < n; ++i) L[i] = lam[i];
    for (int32_t l = 0; l < g->u; ++l)
        for (int32_t i = 0; i < n; ++i) Lm[(size_t)l * (size_t)n + (size_t)i] = lam[i];
    int32_t t_stop = P->max_iter;
    int stopped = 0;
    for (int32_t t = 1; t <= P->max_iter; ++t) {
        for (int32_t ph = 0; ph < phase_count(g, P); ++ph) {
            int32_t r0, r1;
            phase_rows(g, P, ph, &r0, &r1);
            for (int32_t e = g->row_start[r0]; e < g->row_start[r1]; ++e)
                q[e] = (P->coupling ? Lm[(size_t)g->edge_matrix[e] * (size_t)n + (size_t)g->edge_var[e]]
                                    : L[g->edge_var[e]]) - c[e];
            for (int32_t r = r0; r < r1; ++r) {
                int32_t e0 = g->row_start[r], d = g->row_start[r + 1] - e0;
                float zs = z[r] ? -1.0f : 1.0f;
                float alpha = (float)weight_of(P, t, g->row_matrix[r], g->u);
                float *tmp = (float *)b->tmp;
                for (int32_t k = 0; k < d; ++k) {
                    float sg = 1.0f, mn = INFINITY;
                    for (int32_t kk = 0; kk < d; ++kk) {
                        if (kk == k) continue;
                        sg *= q[e0 + kk] < 0.0f ? -1.0f : 1.0f;
                        float a = fabsf(q[e0 + kk]);
                        if (a > C) a = C;
                        if (a < mn) mn = a;
                    }
                    tmp[k] = zs * alpha * sg * mn;
                }
                for (int32_t k = 0; k < d; ++k)
                    c[e0 + k] = P->msg_half ? (float)round_binary16((double)tmp[k]) : tmp[k];
            }
            for (int32_t i = 0; i < n; ++i) L[i] = vsum_f(g, i, lam[i], c);
            if (P->coupling)
                for (int32_t i = 0; i < n; ++i) matrix_posteriors_f(g, i, lam[i], c, Lm);
        }
        for (int32_t i = 0; i < n; ++i) b->xhat[i] = L[i] < 0.0f ? 1 : 0;
        if (P->early_exit && unsatisfied(g, b->xhat, z) == 0) {
            t_stop = t;
            stopped = 1;
            break;
        }
    }
    *ok = stopped ? 1 : (unsatisfied(g, b->xhat, z) == 0 ? 1 : 0);
    *iters = t_stop;
    for (int32_t i = 0; i < n; ++i) bits[i] = b->xhat[i];
    if (Lout)
        for (int32_t i = 0; i < n; ++i) Lout[i] = (double)L[i];
}

/* ---------------------------------------------------------------------- */
typedef struct {
    const graph *g;
    const oracle_params *P;
    int32_t nframes;
    const double *llr;
    const uint8_t *synd;
    uint8_t *bits;
    int32_t *iters;
    uint8_t *ok;
    double *Lout;
    uint8_t *flag;
    int32_t maxdeg;
    int f32;    /* decode_frame_nms_f32 instead of decode_frame */
    int next;   /* next frame to take (atomic) */
    int failed; /* allocation failure in a worker (atomic) */
} job;

static void *worker(void *arg) {
    job *J = (job *)arg;
    frame_buf b;
    memset(&b, 0, sizeof b);
    if (buf_alloc(&b, J->g, J->maxdeg)) {
        __atomic_store_n(&J->failed, 1, __ATOMIC_SEQ_CST);
        buf_free(&b);
        return NULL;
    }
    const size_t n = (size_t)J->g->n, M = (size_t)J->g->M;
    for (;;) {
        int f = __atomic_fetch_add(&J->next, 1, __ATOMIC_SEQ_CST);
        if (f >= J->nframes) break;
        if (J->f32)
            decode_frame_nms_f32(J->g, J->P, J->llr + (size_t)f * n, J->synd + (size_t)f * M, &b,
                                 J->bits + (size_t)f * n, J->iters + f, J->ok + f,
                                 J->Lout ? J->Lout + (size_t)f * n : NULL);
        else
            decode_frame(J->g, J->P, J->llr + (size_t)f * n, J->synd + (size_t)f * M, &b,
                         J->bits + (size_t)f * n, J->iters + f, J->ok + f,
                         J->Lout ? J->Lout + (size_t)f * n : NULL, J->flag ? J->flag + f : NULL);
    }
    buf_free(&b);
    return NULL;
}

int32_t oracle_default_threads(void) {
    long k = sysconf(_SC_NPROCESSORS_ONLN);
    return k > 0 ? (int32_t)k : 1;
}

/* Decode nframes frames.
 *   llr   [nframes][n] channel LLRs (FP64)
 *   synd  [nframes][sum m_l] syndrome bits 0/1, matrices in order
 *   bits  [nframes][n] decided bits; iters [nframes]; ok [nframes]
 *   Lout  [nframes][n] final soft decisions, or NULL
 *   flag  [nframes] near-tie flags, or NULL
 *   nthreads <= 0 uses every online core.
 * Returns 0, or -1 on bad input or allocation failure. */
static int32_t run_decode(const oracle_code *code, const oracle_params *P, int32_t nframes,
                          const double *llr, const uint8_t *synd, uint8_t *bits,
                          int32_t *iters, uint8_t *ok, double *Lout, uint8_t *flag,
                          int32_t nthreads, int f32) {
    if (!code || !P || nframes < 0 || P->max_iter < 1 || code->u < 1 || code->n < 1) return -1;
    if (nframes == 0) return 0;
    graph g;
    if (graph_build(code, &g)) return -1;
    int32_t maxdeg = 0;
    for (int32_t r = 0; r < g.M; ++r) {
        int32_t d = g.row_start[r + 1] - g.row_start[r];
        if (d > maxdeg) maxdeg = d;
    }
    job J = {&g, P, nframes, llr, synd, bits, iters, ok, Lout, flag, maxdeg, f32, 0, 0};
    if (nthreads <= 0) nthreads = oracle_default_threads();
    if (nthreads > nframes) nthreads = nframes;
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!th) { graph_free(&g); return -1; }
    int started = 0;
    for (int k = 0; k < nthreads; ++k) {
        if (pthread_create(&th[k], NULL, worker, &J) != 0) break;
        ++started;
    }
    if (started == 0) worker(&J);
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
    free(th);
    graph_free(&g);
    return J.failed ? -1 : 0;
}

int32_t oracle_mbp_decode(const oracle_code *code, const oracle_params *P, int32_t nframes,
                          const double *llr, const uint8_t *synd, uint8_t *bits,
                          int32_t *iters, uint8_t *ok, double *Lout, uint8_t *flag,
                          int32_t nthreads) {
    return run_decode(code, P, nframes, llr, synd, bits, iters, ok, Lout, flag, nthreads, 0);
}

/* The same decode with normalized min-sum carried out in binary32 (see
   decode_frame_nms_f32); llr values are rounded to float on entry. */
int32_t oracle_mbp_decode_nms_f32(const oracle_code *code, const oracle_params *P,
                                  int32_t nframes, const double *llr, const uint8_t *synd,
                                  uint8_t *bits, int32_t *iters, uint8_t *ok, double *Lout,
                                  int32_t nthreads) {
    if (!P || P->algo != 1) return -1;
    return run_decode(code, P, nframes, llr, synd, bits, iters, ok, Lout, NULL, nthreads, 1);
}

/* Alice's syndromes, eq. (1): z^l = H_l x over GF(2) for every matrix, the
   u syndromes of a frame back to back in matrix order ([nframes][M] bytes,
   0 / 1). Each check's parity is the XOR of x at its variables (x bytes:
   0 = bit 0, nonzero = bit 1). */
int32_t oracle_syndrome(const oracle_code *code, int32_t nframes, const uint8_t *x, uint8_t *z) {
    graph g;
    if (graph_build(code, &g)) return -1;
    for (int32_t f = 0; f < nframes; ++f) {
        const uint8_t *xf = x + (size_t)f * (size_t)g.n;
        uint8_t *zf = z + (size_t)f * (size_t)g.M;
        for (int32_t r = 0; r < g.M; ++r) {
            int par = 0;
            for (int32_t e = g.row_start[r]; e < g.row_start[r + 1]; ++e) par ^= xf[g.edge_var[e]] ? 1 : 0;
            zf[r] = (uint8_t)par;
        }
    }
    graph_free(&g);
    return 0;
}

/* Residual syndrome weight of decided bits: per frame, the number of stacked
   checks whose parity over x differs from z. */
int32_t oracle_unsatisfied(const oracle_code *code, int32_t nframes, const uint8_t *x,
                           const uint8_t *synd, int32_t *weight) {
    graph g;
    if (graph_build(code, &g)) return -1;
    for (int32_t f = 0; f < nframes; ++f)
        weight[f] = unsatisfied(&g, x + (size_t)f * (size_t)g.n, synd + (size_t)f * (size_t)g.M);
    graph_free(&g);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Unrolled normalized min-sum and its exact reverse-mode gradient.
 *
 * Forward: K flooding iterations with no stopping test and weight
 * alpha[t][l] for the checks of matrix l at iteration t; output L^K.
 * Backward: given dJ/dL^K, the exact adjoint of that forward, with these
 * subgradients: sgn has derivative 0; min passes the whole derivative to the
 * smallest of the other edges (lowest edge position among equal values);
 * the cap min(|q|, C) passes sgn(q) when |q| < C and 0 otherwise. */
/* The forward of one iteration in binary32, with the rounding of
   decode_frame_nms_f32; states are held as the doubles of their float values. */
static void nms_iteration_f32(const graph *g, const double *alpha, int32_t t, double C,
                              const double *lam,
                              const uint8_t *z, const double *Lp, const double *cp, double *q,
                              double *c, double *L) {
    const int32_t n = g->n, E = g->E, M = g->M;
    const float Cf = (float)C;
    for (int32_t e = 0; e < E; ++e) q[e] = (double)((float)Lp[g->edge_var[e]] - (float)cp[e]);
    for (int32_t r = 0; r < M; ++r) {
        int32_t e0 = g->row_start[r], d = g->row_start[r + 1] - e0;
        float zs = z[r] ? -1.0f : 1.0f;
        float a_tl = (float)alpha[(size_t)(t - 1) * (size_t)g->u + (size_t)g->row_matrix[r]];
        for (int32_t k = 0; k < d; ++k) {
            float sg = 1.0f, mn = INFINITY;
            for (int32_t kk = 0; kk < d; ++kk) {
                if (kk == k) continue;
                float qf = (float)q[e0 + kk];
                sg *= qf < 0.0f ? -1.0f : 1.0f;
                float a = fabsf(qf);
                if (a > Cf) a = Cf;
                if (a < mn) mn = a;
            }
            c[e0 + k] = (double)(zs * a_tl * sg * mn);
        }
    }
    for (int32_t i = 0; i < n; ++i) L[i] = (double)vsum_fd(g, i, (float)lam[i], c);
}

static void nms_unrolled_frame(const graph *g, int32_t K, const double *alpha, double C,
                               const double *lam, const uint8_t *z, const double *gL_in,
                               double *Lout, double *glam, double *galpha,
                               double *cs /* [(K+1)*E] */, double *qs /* [K*E] */,
                               double *Ls /* [(K+1)*n] */, double *gL, double *gc,
                               double *gq, int f32) {
    const int32_t n = g->n, E = g->E, M = g->M, u = g->u;
    double *c0 = cs;
    for (int32_t e = 0; e < E; ++e) c0[e] = 0.0;
    for (int32_t i = 0; i < n; ++i) Ls[i] = f32 ? (double)(float)lam[i] : lam[i];
    for (int32_t t = 1; t <= K; ++t) {
        const double *Lp = Ls + (size_t)(t - 1) * n, *cp = cs + (size_t)(t - 1) * E;
        double *q = qs + (size_t)(t - 1) * E, *c = cs + (size_t)t * E, *L = Ls + (size_t)t * n;
        if (f32) {
            nms_iteration_f32(g, alpha, t, C, lam, z, Lp, cp, q, c, L);
            continue;
        }
        for (int32_t e = 0; e < E; ++e) q[e] = Lp[g->edge_var[e]] - cp[e];
        for (int32_t r = 0; r < M; ++r) {
            int32_t e0 = g->row_start[r], d = g->row_start[r + 1] - e0;
            check_rule_nms(d, q + e0, z[r], alpha[(size_t)(t - 1) * u + g->row_matrix[r]], C,
                           c + e0);
        }
        for (int32_t i = 0; i < n; ++i) L[i] = vsum_d(g, i, lam[i], c);
    }
    for (int32_t i = 0; i < n; ++i) Lout[i] = Ls[(size_t)K * n + i];
    if (!gL_in) return;

    /* reverse sweep */
    for (int32_t i = 0; i < n; ++i) {
        gL[i] = gL_in[i];
        glam[i] = 0.0;
    }
    for (int32_t e = 0; e < E; ++e) gc[e] = 0.0; /* from q^{K+1}: none */
    for (int32_t t = K; t >= 1; --t) {
        const double *q = qs + (size_t)(t - 1) * E;
        /* L^t = lambda + sum of c^t over the variable's edges */
        for (int32_t i = 0; i < n; ++i) glam[i] += gL[i];
        for (int32_t e = 0; e < E; ++e) gc[e] += gL[g->edge_var[e]];
        /* c^t = rule(q^t, alpha_t) */
        for (int32_t e = 0; e < E; ++e) gq[e] = 0.0;
        for (int32_t r = 0; r < M; ++r) {
            int32_t e0 = g->row_start[r], d = g->row_start[r + 1] - e0;
            int32_t l = g->row_matrix[r];
            double a_tl = alpha[(size_t)(t - 1) * u + l];
            double zs = z[r] ? -1.0 : 1.0;
            for (int32_t k = 0; k < d; ++k) {
                double s = 1.0, mn = INFINITY;
                int32_t arg = -1;
                for (int32_t kk = 0; kk < d; ++kk) {
                    if (kk == k) continue;
                    s *= sgn(q[e0 + kk]);
                    double a = fabs(q[e0 + kk]);
                    if (a > C) a = C;
                    if (a < mn) { mn = a; arg = kk; }
                }
                double up = gc[e0 + k];
                /* dc/dalpha = (-1)^z * prod sgn * min */
                galpha[(size_t)(t - 1) * u + l] += zs * s * mn * up;
                /* dc/dq at the arg-min edge */
                double qa = q[e0 + arg];
                double dcap = fabs(qa) < C ? sgn(qa) : 0.0;
                gq[e0 + arg] += zs * a_tl * s * dcap * up;
            }
        }
        /* q^t = L^{t-1}[v] - c^{t-1} */
        for (int32_t i = 0; i < n; ++i) gL[i] = 0.0;
        for (int32_t e = 0; e < E; ++e) {
            gL[g->edge_var[e]] += gq[e];
            gc[e] = -gq[e];
        }
        if (t == 1) {
            /* L^0 = lambda; c^0 = 0 is constant */
            for (int32_t i = 0; i < n; ++i) glam[i] += gL[i];
        }
    }
}

/* Unrolled min-sum forward (and, if gL is not NULL, its gradient) for
 * nframes frames. alpha is [K][u]; llr, gL, Lout, glam are [nframes][n];
 * galpha [K][u] is the sum over frames. With f32 = 1 the forward runs in
 * binary32 (decode_frame_nms_f32's rounding) and the reverse sweep, still in
 * FP64, differentiates that binary32 trajectory: it takes its minima, signs
 * and caps from the float messages. Single-threaded.
 * Returns 0 or -1. */
int32_t oracle_nms_unrolled(const oracle_code *code, int32_t K, const double *alpha,
                            double clip, int32_t nframes, const double *llr,
                            const uint8_t *synd, const double *gL, double *Lout,
                            double *glam, double *galpha, int32_t f32) {
    if (!code || K < 1 || nframes < 0) return -1;
    graph g;
    if (graph_build(code, &g)) return -1;
    const size_t n = (size_t)g.n, E = (size_t)g.E, M = (size_t)g.M;
    double *cs = malloc(sizeof(double) * (size_t)(K + 1) * (E ? E : 1));
    double *qs = malloc(sizeof(double) * (size_t)K * (E ? E : 1));
    double *Ls = malloc(sizeof(double) * (size_t)(K + 1) * n);
    double *gLw = malloc(sizeof(double) * n);
    double *gc = malloc(sizeof(double) * (E ? E : 1));
    double *gq = malloc(sizeof(double) * (E ? E : 1));
    double *gaf = calloc((size_t)K * (size_t)g.u, sizeof(double));
    double *glw = malloc(sizeof(double) * n);
    int rc = -1;
    if (!cs || !qs || !Ls || !gLw || !gc || !gq || !gaf || !glw) goto out;
    if (galpha && gL)
        for (size_t k = 0; k < (size_t)K * (size_t)g.u; ++k) galpha[k] = 0.0;
    for (int32_t f = 0; f < nframes; ++f) {
        for (size_t k = 0; k < (size_t)K * (size_t)g.u; ++k) gaf[k] = 0.0;
        nms_unrolled_frame(&g, K, alpha, clip, llr + f * n, synd + f * M,
                           gL ? gL + f * n : NULL, Lout + f * n, glam ? glam + f * n : glw,
                           gaf, cs, qs, Ls, gLw, gc, gq, f32);
        if (galpha && gL)
            for (size_t k = 0; k < (size_t)K * (size_t)g.u; ++k) galpha[k] += gaf[k];
    }
    rc = 0;
out:
    free(cs);
    free(qs);
    free(Ls);
    free(gLw);
    free(gc);
    free(gq);
    free(gaf);
    free(glw);
    graph_free(&g);
    return rc;
}
